// Learned per-level smoothing parameters: a 4 -> 32 -> 32 -> 10 perceptron
// (tanh hidden layers, FP32) maps problem features to logits of the
// additive-Schwarz damping eta in (0, 1) of equation ASM (outputs 0..4) and
// to the number of smoothing steps (outputs 5..9), one per smoothed level,
// finest first.  Forward, loss gradient and Adam run on the device; the
// damping kernel writes eta straight into a solver's per-problem damping
// array.
#include "mlp.hpp"

#include <cmath>
#include <mutex>

#include "device_util.hpp"

namespace dfmg {

// Scratch of the allocation-free gradient entry point: the per-sample
// gradient rows (MLP_SCRATCH_SAMPLES x MLP_NPARAM floats) and the per-sample
// losses (MLP_SCRATCH_SAMPLES floats), 3.2 MB per GPU for the life of the
// process.  Host code never passes this name to a kernel: it is a host-side
// stand-in; the device address comes from hipGetSymbolAddress (mlp_scratch).
static __device__ __align__(256) float scratch[(size_t)MLP_SCRATCH_SAMPLES * (MLP_NPARAM + 1)];

namespace {

constexpr int oW1 = 0, ob1 = oW1 + MLP_H * MLP_IN, oW2 = ob1 + MLP_H, ob2 = oW2 + MLP_H * MLP_H,
              oW3 = ob2 + MLP_H, ob3 = oW3 + MLP_OUT * MLP_H;
static_assert(ob3 + MLP_OUT == MLP_NPARAM, "parameter layout");

__device__ void forward(const float *W, const float *x, float *h1, float *h2, float *z) {
    for (int i = 0; i < MLP_H; ++i) {
        float s = W[ob1 + i];
        for (int c = 0; c < MLP_IN; ++c) s = fmaf(W[oW1 + i * MLP_IN + c], x[c], s);
        h1[i] = tanhf(s);
    }
    for (int j = 0; j < MLP_H; ++j) {
        float s = W[ob2 + j];
        for (int i = 0; i < MLP_H; ++i) s = fmaf(W[oW2 + j * MLP_H + i], h1[i], s);
        h2[j] = tanhf(s);
    }
    for (int o = 0; o < MLP_OUT; ++o) {
        float s = W[ob3 + o];
        for (int j = 0; j < MLP_H; ++j) s = fmaf(W[oW3 + o * MLP_H + j], h2[j], s);
        z[o] = s;
    }
}

__global__ void k_mlp_forward(int n, const float *W, const float *X, float *Z) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    float h1[MLP_H], h2[MLP_H], z[MLP_OUT];
    forward(W, X + s * MLP_IN, h1, h2, z);
    for (int o = 0; o < MLP_OUT; ++o) Z[s * MLP_OUT + o] = z[o];
}

// Gradient of sum_{s,o} M (z - y)^2 * scale for one sample, by the chain rule
// through both tanh layers, written to its own row of work.
__global__ void k_mlp_sample_grad(int n, const float *W, const float *X, const float *Y, const float *Mk,
                                  float scale, float *work, float *lw) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float *x = X + s * MLP_IN;
    float h1[MLP_H], h2[MLP_H], z[MLP_OUT], dz[MLP_OUT], d2[MLP_H];
    forward(W, x, h1, h2, z);
    float *g = work + (int64_t)s * MLP_NPARAM;
    float l = 0.f;
    for (int o = 0; o < MLP_OUT; ++o) {
        const float e = z[o] - Y[s * MLP_OUT + o];
        const float mk = Mk[s * MLP_OUT + o];
        l += mk * e * e * scale;
        dz[o] = 2.f * mk * e * scale;
        g[ob3 + o] = dz[o];
        for (int j = 0; j < MLP_H; ++j) g[oW3 + o * MLP_H + j] = dz[o] * h2[j];
    }
    lw[s] = l;
    for (int j = 0; j < MLP_H; ++j) {
        float t = 0.f;
        for (int o = 0; o < MLP_OUT; ++o) t = fmaf(dz[o], W[oW3 + o * MLP_H + j], t);
        d2[j] = t * (1.f - h2[j] * h2[j]);
        g[ob2 + j] = d2[j];
        for (int i = 0; i < MLP_H; ++i) g[oW2 + j * MLP_H + i] = d2[j] * h1[i];
    }
    for (int i = 0; i < MLP_H; ++i) {
        float t = 0.f;
        for (int j = 0; j < MLP_H; ++j) t = fmaf(d2[j], W[oW2 + j * MLP_H + i], t);
        const float d1 = t * (1.f - h1[i] * h1[i]);
        g[ob1 + i] = d1;
        for (int c = 0; c < MLP_IN; ++c) g[oW1 + i * MLP_IN + c] = d1 * x[c];
    }
}

// G[p] = sum over samples of work[s][p] in sample order; loss likewise.
__global__ void k_mlp_reduce(int n, const float *work, const float *lw, float *G, float *loss) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < MLP_NPARAM) {
        float s = 0.f;
        for (int i = 0; i < n; ++i) s += work[(int64_t)i * MLP_NPARAM + p];
        G[p] = s;
    }
    if (p == 0) {
        float s = 0.f;
        for (int i = 0; i < n; ++i) s += lw[i];
        *loss = s;
    }
}

// Adam (Kingma and Ba) with bias correction, step t >= 1.
__global__ void k_mlp_adam(float *W, float *m, float *v, const float *G, int t, float lr, float b1, float b2,
                           float eps) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAM) return;
    const float g = G[p];
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (1.f - powf(b1, (float)t));
    const float vh = vv / (1.f - powf(b2, (float)t));
    W[p] -= lr * mh / (sqrtf(vh) + eps);
}

// eta[p][l] = sigmoid(z_{L-1-l}) for l = L-1 .. 1 (output 0 is the finest
// smoothed level; levels beyond the outputs reuse the last one).
__global__ void k_mlp_damping(int np, const float *W, const float *feat, int L, double *eta) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    float h1[MLP_H], h2[MLP_H], z[MLP_OUT];
    forward(W, feat + p * MLP_IN, h1, h2, z);
    for (int l = L - 1; l >= 1; --l) {
        const int o = min(L - 1 - l, MLP_ETA - 1);
        eta[(int64_t)p * L + l] = 1.0 / (1.0 + exp(-(double)z[o]));
    }
}

}  // namespace

void mlp_forward_host(const float *W, const float *x, double *z) {
    double h1[MLP_H], h2[MLP_H];
    for (int i = 0; i < MLP_H; ++i) {
        double s = W[ob1 + i];
        for (int c = 0; c < MLP_IN; ++c) s += (double)W[oW1 + i * MLP_IN + c] * x[c];
        h1[i] = std::tanh(s);
    }
    for (int j = 0; j < MLP_H; ++j) {
        double s = W[ob2 + j];
        for (int i = 0; i < MLP_H; ++i) s += (double)W[oW2 + j * MLP_H + i] * h1[i];
        h2[j] = std::tanh(s);
    }
    for (int o = 0; o < MLP_OUT; ++o) {
        double s = W[ob3 + o];
        for (int j = 0; j < MLP_H; ++j) s += (double)W[oW3 + o * MLP_H + j] * h2[j];
        z[o] = s;
    }
}

void launch_mlp_forward(int n, const float *W, const float *X, float *Z, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_mlp_forward, dim3((n + 63) / 64), dim3(64), 0, s, n, W, X, Z);
}

void launch_mlp_grad(int n, const float *W, const float *X, const float *Y, const float *Mk, float scale,
                     float *work, float *lw, float *G, float *loss, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_mlp_sample_grad, dim3((n + 63) / 64), dim3(64), 0, s, n, W, X, Y, Mk, scale, work, lw);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, n, work, lw, G, loss);
}

// Device address of `scratch` on `device`, looked up once per device with
// that device current (each GPU holds its own copy of the array).
float *mlp_scratch(int device, hipError_t *err) {
    constexpr int kMaxDevices = 64;
    static float *ptr[kMaxDevices] = {};
    static std::mutex mu;
    *err = hipSuccess;
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[device]) {
        int cur = -1;
        if ((*err = hipGetDevice(&cur)) != hipSuccess) return nullptr;
        if (cur != device && (*err = hipSetDevice(device)) != hipSuccess) return nullptr;
        void *p = nullptr;
        *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t e2 = hipSetDevice(cur);
            if (*err == hipSuccess) *err = e2;
        }
        if (*err != hipSuccess) return nullptr;
        ptr[device] = static_cast<float *>(p);
    }
    return ptr[device];
}

void launch_mlp_grad_scratch(int n, const float *W, const float *X, const float *Y, const float *Mk, float scale,
                             float *scr, float *G, float *loss, hipStream_t s) {
    launch_mlp_grad(n, W, X, Y, Mk, scale, scr, scr + (size_t)MLP_SCRATCH_SAMPLES * MLP_NPARAM, G, loss, s);
}

void launch_mlp_adam(float *W, float *m, float *v, const float *G, int t, float lr, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, s, W, m, v, G, t, lr, 0.9f, 0.999f,
                       1e-8f);
}

void launch_mlp_damping(int np, const float *W, const float *feat, int L, double *eta, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_damping, dim3((np + 63) / 64), dim3(64), 0, s, np, W, feat, L, eta);
}

}  // namespace dfmg
