// Single-workgroup V-cycle over the coarse levels (gfx950).  Below a few
// thousand DOFs per problem every kernel of a level runs for a few
// microseconds, set by launch and drain rather than by HBM, and a V-cycle
// launches about fifteen of them per level.  Here one workgroup of 1024
// threads per problem walks the whole sub-cycle top .. 0 .. top with
// workgroup barriers between the steps, so the coarse part of a cycle is one
// launch.  Every value is computed by the same device functions, in the same
// order, as the per-level kernels (residual with one lane per row, smoother
// rows, gathers, transfers, coarse product), so the results agree bit for bit.
// Mapped domains (velocity rows coupling every component) do not take it.
#include "schwarz_dev.hpp"
#include "spmv_dev.hpp"

namespace dfmg {

namespace {

constexpr int kSmallBlock = 1024;

// r = F - K U of level L for one problem
template <int D, int K, class T>
__device__ void small_residual(const SmallLevel<T> &L, int prob, const T *F, const T *U, T *r) {
    SpmvArgsT<T> a = L.sp;
    a.val += prob * a.sval;
    a.U = U;
    const int n = (int)L.n;
    if (a.win) {
        for (int g = threadIdx.x; g < n; g += blockDim.x) r[g] = F[g] - spmv_row<D, K, true, false, T>(a, g);
    } else {
        for (int g = threadIdx.x; g < n; g += blockDim.x) r[g] = F[g] - spmv_row<D, K, false, false, T>(a, g);
    }
}

// U = (assign ? 0 : U) + eta * sum_i E_i^T M_i E_i src, two passes
template <class T>
__device__ void small_smooth(const SmallLevel<T> &L, int prob, const T *src, T *U, bool assign) {
    T *delta = L.delta + prob * L.sdelta;
    const T *M = L.M + prob * L.sM;
    for (int q = threadIdx.x; q < L.nsmall; q += blockDim.x) {
        const int p = L.small[q];
        const int base = L.pptr[p];
        patch_small(M + L.moff[prob * L.smoff + p], L.pdofs + base, L.pptr[p + 1] - base, src, delta + base);
    }
    const int4 *ent = L.ent_info + prob * L.nent;
    for (int t = threadIdx.x; t < L.nbig; t += blockDim.x) {
        const int e = L.bigent[t];
        const int4 info = ent[e];
        delta[e] = patch_row(M + info.x, L.pdofs + info.y, info.z, src);
    }
    __syncthreads();
    const T eta = (T)L.eta[prob * L.seta];
    for (int j = threadIdx.x; j < (int)L.n; j += blockDim.x) {
        const T u = assign ? T(0) : U[j];
        U[j] = fma(eta, dof_sum(L.inv_ptr, L.inv_pos, delta, j), u);
    }
    __syncthreads();
}

template <int D, int K, class T>
__global__ __launch_bounds__(kSmallBlock) void k_vcycle_small(const SmallLevel<T> *__restrict__ lv, int top,
                                                              const int *stop) {
    const int prob = blockIdx.x;
    if (stop_flag(stop, prob)) return;
    for (int l = top; l >= 1; --l) {
        const SmallLevel<T> &L = lv[l];
        T *F = L.F + prob * L.n, *U = L.U + prob * L.n, *r = L.r + prob * L.n;
        const int nu1 = L.nu1;
        for (int s = 0; s < nu1; ++s) {
            if (s == 0) {
                small_smooth(L, prob, F, U, true);  // U = 0: the residual is F
            } else {
                small_residual<D, K, T>(L, prob, F, U, r);
                __syncthreads();
                small_smooth(L, prob, r, U, false);
            }
        }
        const SmallLevel<T> &C = lv[l - 1];
        T *Fc = C.F + prob * C.n;
        const T *src = F;
        if (nu1 == 0) {
            for (int j = threadIdx.x; j < (int)L.n; j += blockDim.x) U[j] = T(0);
        } else {
            small_residual<D, K, T>(L, prob, F, U, r);
            src = r;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < (int)C.n; i += blockDim.x) Fc[i] = T(0) + csr_row(L.R_rp, L.R_ci, L.R_v, src, i);
        __syncthreads();
    }
    {
        const SmallLevel<T> &C = lv[0];
        const int n = (int)C.n, wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
        const T *F = C.F + prob * C.n;
        T *U = C.U + prob * C.n;
        for (int row = wave; row < n; row += nw) {
            const double acc = gemv_row_wave(C.Kinv + prob * C.n * C.n, n, F, row, lane);
            if (lane == 0) U[row] = (T)acc;
        }
        __syncthreads();
    }
    for (int l = 1; l <= top; ++l) {
        const SmallLevel<T> &L = lv[l];
        const SmallLevel<T> &C = lv[l - 1];
        T *F = L.F + prob * L.n, *U = L.U + prob * L.n, *r = L.r + prob * L.n;
        const T *dU = C.U + prob * C.n;
        for (int i = threadIdx.x; i < (int)L.n; i += blockDim.x) U[i] = U[i] + csr_row(L.P_rp, L.P_ci, L.P_v, dU, i);
        __syncthreads();
        for (int s = 0; s < L.nu2; ++s) {
            small_residual<D, K, T>(L, prob, F, U, r);
            __syncthreads();
            small_smooth(L, prob, r, U, false);
        }
    }
}

}  // namespace

template <class T>
void launch_vcycle_small(int d, int k, const SmallLevel<T> *lv, int top, const int *stop, int nprob, hipStream_t s) {
    const dim3 grid(nprob), block(kSmallBlock);
    if (d == 2 && k == 1) hipLaunchKernelGGL((k_vcycle_small<2, 1, T>), grid, block, 0, s, lv, top, stop);
    else if (d == 2 && k == 2) hipLaunchKernelGGL((k_vcycle_small<2, 2, T>), grid, block, 0, s, lv, top, stop);
    else if (d == 3 && k == 1) hipLaunchKernelGGL((k_vcycle_small<3, 1, T>), grid, block, 0, s, lv, top, stop);
    else hipLaunchKernelGGL((k_vcycle_small<3, 2, T>), grid, block, 0, s, lv, top, stop);
}

template void launch_vcycle_small<double>(int, int, const SmallLevel<double> *, int, const int *, int, hipStream_t);
template void launch_vcycle_small<float>(int, int, const SmallLevel<float> *, int, const int *, int, hipStream_t);

}  // namespace dfmg
