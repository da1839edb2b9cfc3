// Right-hand sides of the time steps (Guermond's step: conv = 0, no
// convective terms, the advection being in the operator).
//
// Right-hand side of one Crank-Nicolson / Adams-Bashforth step of the
// Navier-Stokes equations posed as a generalized Stokes problem with
// sigma = 2 / dt (equation GS, with every term of the step doubled):
//   F_u = F2 - (K U^n)_u + (N_i, 2 sigma u^n - 3 (u^n . grad) u^n + (u^{n-1} . grad) u^{n-1}),
//   F_p = 0,
// first step: -2 (u^n . grad) u^n in place of the last two terms.  F2 - K U^n
// comes from the residual kernel; the quadrature load from two kernels: one
// thread per quadrature point evaluates the discrete fields and their
// gradients there (tensor-product B-spline tables of the finest grid) and
// stores the weighted integrand, then one thread per velocity DOF sums it
// against its basis function over the elements of its support, in a fixed
// order (no atomics).
#include "device_util.hpp"

namespace dfmg {

namespace {

// basis table entry: degree index a (0: k, 1: k+1), element e, point g, local function m
__device__ __forceinline__ int64_t tab(const CnabArgs &a, int deg, int e, int g, int m) {
    return (((int64_t)deg * a.N + e) * a.nq + g) * (a.k + 2) + m;
}

// value and gradient of velocity component c of field X (one problem) at
// element e, point g
__device__ void eval_comp(const CnabArgs &a, const double *X, int c, const int *e, const int *g, double &val,
                          double *grad) {
    int q[3], s[3], deg[3];
    for (int j = 0; j < 3; ++j) {
        deg[j] = (j == c) ? 1 : 0;
        q[j] = j < a.d ? a.k + deg[j] : 0;
        s[j] = (j == c) ? 1 : 0;
    }
    val = 0.0;
    for (int j = 0; j < 3; ++j) grad[j] = 0.0;
    for (int m2 = 0; m2 <= q[2]; ++m2)
        for (int m1 = 0; m1 <= q[1]; ++m1)
            for (int m0 = 0; m0 <= q[0]; ++m0) {
                const int m[3] = {m0, m1, m2};
                int64_t idx = 0, stride = 1;
                bool ok = true;
                double bv[3] = {1.0, 1.0, 1.0}, bd[3] = {0.0, 0.0, 0.0};
                for (int j = 0; j < a.d; ++j) {
                    const int st = e[j] + m[j] - s[j];
                    if (st < 0 || st >= a.nb[c][j]) ok = false;
                    idx += (int64_t)st * stride;
                    stride *= a.nb[c][j];
                    bv[j] = a.bval[tab(a, deg[j], e[j], g[j], m[j])];
                    bd[j] = a.bder[tab(a, deg[j], e[j], g[j], m[j])];
                }
                if (!ok) continue;
                const double u = X[a.off[c] + idx];
                double p = u;
                for (int j = 0; j < a.d; ++j) p *= bv[j];
                val += p;
                for (int j = 0; j < a.d; ++j) {
                    double t = u * bd[j];
                    for (int i = 0; i < a.d; ++i)
                        if (i != j) t *= bv[i];
                    grad[j] += t;
                }
            }
}

__global__ void k_cnab_points(CnabArgs a) {
    const int prob = blockIdx.y;
    const int64_t P = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (P >= a.npts) return;
    int64_t ppd = 1;
    for (int j = 0; j < a.d; ++j) ppd *= a.nq;
    int64_t el = P / ppd, pp = P % ppd;
    int e[3] = {0, 0, 0}, g[3] = {0, 0, 0};
    for (int j = 0; j < a.d; ++j) {
        e[j] = (int)(el % a.N);
        el /= a.N;
        g[j] = (int)(pp % a.nq);
        pp /= a.nq;
    }
    double w = 1.0;
    for (int j = 0; j < a.d; ++j) w *= a.wq[g[j]];
    const double *U = a.U + prob * a.svec;
    const double *Uo = a.Uold ? a.Uold + prob * a.svec : nullptr;
    double v[3] = {0, 0, 0}, gr[3][3] = {}, vo[3] = {0, 0, 0}, gro[3][3] = {};
    for (int c = 0; c < a.d; ++c) {
        eval_comp(a, U, c, e, g, v[c], gr[c]);
        if (Uo && a.conv) eval_comp(a, Uo, c, e, g, vo[c], gro[c]);
    }
    const double sigma = a.sigma[prob];
    double *G = a.G + prob * a.sG + P * a.d;
    for (int c = 0; c < a.d; ++c) {
        double conv = 0.0, convo = 0.0;
        for (int j = 0; j < a.d; ++j) {
            conv += v[j] * gr[c][j];
            convo += vo[j] * gro[c][j];
        }
        const double adv = a.conv ? (Uo ? 3.0 * conv - convo : 2.0 * conv) : 0.0;
        G[c] = w * (2.0 * sigma * v[c] - adv);
    }
}

__global__ void k_cnab_load(CnabArgs a) {
    const int prob = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.n) return;
    double *F = a.Fout + prob * a.svec;
    if (i >= a.off[a.d]) {  // pressure rows
        F[i] = 0.0;
        return;
    }
    int c = 0;
    while (i >= a.off[c + 1]) ++c;
    int64_t l = i - a.off[c];
    int t[3] = {0, 0, 0}, q[3] = {0, 0, 0}, deg[3] = {0, 0, 0};
    for (int j = 0; j < a.d; ++j) {
        t[j] = (int)(l % a.nb[c][j]) + (j == c ? 1 : 0);
        l /= a.nb[c][j];
        deg[j] = j == c ? 1 : 0;
        q[j] = a.k + deg[j];
    }
    int e0[3] = {0, 0, 0}, e1[3] = {0, 0, 0}, g1[3] = {0, 0, 0};
    for (int j = 0; j < a.d; ++j) {
        e0[j] = max(0, t[j] - q[j]);
        e1[j] = min(a.N - 1, t[j]);
        g1[j] = a.nq - 1;
    }
    const double *G = a.G + prob * a.sG;
    int64_t ppd = 1;
    for (int j = 0; j < a.d; ++j) ppd *= a.nq;
    double acc = 0.0;
    for (int ea = e0[2]; ea <= e1[2]; ++ea)
        for (int eb = e0[1]; eb <= e1[1]; ++eb)
            for (int ec = e0[0]; ec <= e1[0]; ++ec) {
                const int e[3] = {ec, eb, ea};
                int64_t el = 0, stride = 1;
                for (int j = 0; j < a.d; ++j) {
                    el += (int64_t)e[j] * stride;
                    stride *= a.N;
                }
                for (int ga = 0; ga <= g1[2]; ++ga)
                    for (int gb = 0; gb <= g1[1]; ++gb)
                        for (int gc = 0; gc <= g1[0]; ++gc) {
                            const int g[3] = {gc, gb, ga};
                            int64_t pp = 0, ps = 1;
                            double b = 1.0;
                            for (int j = 0; j < a.d; ++j) {
                                pp += (int64_t)g[j] * ps;
                                ps *= a.nq;
                                b *= a.bval[tab(a, deg[j], e[j], g[j], t[j] - e[j])];
                            }
                            acc = fma(G[(el * ppd + pp) * a.d + c], b, acc);
                        }
            }
    F[i] += acc;
}

}  // namespace

void launch_cnab_load(const CnabArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_cnab_points, dim3(blocks_for(a.npts), a.nprob), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_cnab_load, dim3(blocks_for(a.n), a.nprob), dim3(kBlock), 0, s, a);
}

}  // namespace dfmg
