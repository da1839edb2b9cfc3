// HIP kernels of the additive-Schwarz V-cycle (gfx950, wave64).
#include "kernels.hpp"

namespace dfmg {

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with a private L2.  Remapping the hardware block id so that each XCD works
// on one contiguous eighth of the rows keeps neighbouring rows (which share
// most of the vector entries a stencil row reads) in the same L2.
__device__ __forceinline__ int xcd_block(int hw, int grid) {
    const int per = grid >> 3;  // grid is a multiple of 8
    return (hw & 7) * per + (hw >> 3);
}

template <int D, int K>
struct Geo {
    __host__ __device__ static constexpr int q(int R, int dir) { return (R < D && dir == R) ? K + 1 : K; }
    __host__ __device__ static constexpr int s(int R, int dir) { return (R < D && dir == R) ? 1 : 0; }
    __host__ __device__ static constexpr int lo(int R, int C, int dir) {
        return dir < D ? s(R, dir) - s(C, dir) - q(R, dir) : 0;
    }
    __host__ __device__ static constexpr int w(int R, int C, int dir) {
        return dir < D ? q(R, dir) + q(C, dir) + 1 : 1;
    }
};

__device__ __forceinline__ int clampi(int x, int lo, int hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Contribution of column block C to row (i0, i1, i2) of row block R.  Slots
// outside the grid hold 0 and read a clamped (valid) vector entry.
template <int D, int K, int R, int C>
__device__ __forceinline__ double block_dot(const SpmvArgs &a, int i0, int i1, int i2, const double *&vp,
                                            int64_t stride) {
    using G = Geo<D, K>;
    constexpr int W0 = G::w(R, C, 0), W1 = G::w(R, C, 1), W2 = G::w(R, C, 2);
    constexpr int L0 = G::lo(R, C, 0), L1 = G::lo(R, C, 1), L2 = G::lo(R, C, 2);
    const double *Uc = a.U + a.off[C];
    const int n0 = a.nb[C][0], n1 = a.nb[C][1], n2 = a.nb[C][2];
    double acc = 0.0;
#pragma unroll
    for (int o2 = 0; o2 < W2; ++o2) {
        const int j2 = (D == 3) ? clampi(i2 + L2 + o2, 0, n2 - 1) : 0;
#pragma unroll
        for (int o1 = 0; o1 < W1; ++o1) {
            const int j1 = clampi(i1 + L1 + o1, 0, n1 - 1);
            const double *urow = Uc + ((int64_t)j2 * n1 + j1) * n0;
#pragma unroll
            for (int o0 = 0; o0 < W0; ++o0) {
                const int j0 = clampi(i0 + L0 + o0, 0, n0 - 1);
                acc = fma(*vp, urow[j0], acc);
                vp += stride;
            }
        }
    }
    return acc;
}

template <int D, int K, int R>
__device__ __forceinline__ double row_dot(const SpmvArgs &a, int li) {
    const int nb0 = a.nb[R][0], nb1 = a.nb[R][1];
    const int i0 = li % nb0;
    const int t = li / nb0;
    const int i1 = t % nb1;
    const int i2 = t / nb1;
    const int64_t stride = a.off[R + 1] - a.off[R];
    const double *vp = a.val + a.val_off[R] + li;
    double acc;
    if constexpr (R < D) {
        acc = block_dot<D, K, R, R>(a, i0, i1, i2, vp, stride);
        acc += block_dot<D, K, R, D>(a, i0, i1, i2, vp, stride);
    } else {
        acc = block_dot<D, K, R, 0>(a, i0, i1, i2, vp, stride);
        acc += block_dot<D, K, R, 1>(a, i0, i1, i2, vp, stride);
        if constexpr (D == 3) acc += block_dot<D, K, R, 2>(a, i0, i1, i2, vp, stride);
    }
    return acc;
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
    // wave reduction then across the 4 waves, fixed order
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    return s;
}

// r = F - K U, optionally with per-block partial sums of r^2.
template <int D, int K>
__global__ __launch_bounds__(kBlock) void k_spmv(SpmvArgs a) {
    if (a.stop && *a.stop) return;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int g = b * kBlock + threadIdx.x;
    double rr = 0.0;
    if (b < a.nblocks && g < a.n) {
        double acc;
        if (g < a.off[1]) {
            acc = row_dot<D, K, 0>(a, g);
        } else if (g < a.off[2]) {
            acc = row_dot<D, K, 1>(a, g - (int)a.off[1]);
        } else if (D == 3 && g < a.off[3]) {
            acc = row_dot<D, K, (D == 3 ? 2 : 1)>(a, g - (int)a.off[2]);
        } else {
            acc = row_dot<D, K, D>(a, g - (int)a.off[D]);
        }
        const double v = a.F[g] - acc;
        a.r[g] = v;
        rr = v * v;
    }
    if (a.partial) {
        __shared__ double sh[kBlock / 64];
        const double s = block_sum(rr, sh);
        if (threadIdx.x == 0 && b < a.nblocks) a.partial[b] = s;
    }
}

void launch_spmv(int d, int k, const SpmvArgs &a, hipStream_t s) {
    const int grid = padded_grid(a.nblocks);
    if (d == 2 && k == 1) hipLaunchKernelGGL((k_spmv<2, 1>), dim3(grid), dim3(kBlock), 0, s, a);
    else if (d == 2 && k == 2) hipLaunchKernelGGL((k_spmv<2, 2>), dim3(grid), dim3(kBlock), 0, s, a);
    else if (d == 3 && k == 1) hipLaunchKernelGGL((k_spmv<3, 1>), dim3(grid), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_spmv<3, 2>), dim3(grid), dim3(kBlock), 0, s, a);
}

// Additive Schwarz update, owner-computes form: DOF j gathers, from every
// subdomain i that holds it at local row m, the row m of M_i E_i r, so
// U_j += eta * sum_i (E_i^T M_i E_i r)_j with no atomics and a fixed order.
__global__ __launch_bounds__(kBlock) void k_schwarz_gather(PatchArgs a) {
    if (a.stop && *a.stop) return;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int j = b * kBlock + threadIdx.x;
    if (j >= a.n) return;
    double acc = 0.0;
    const int e1 = a.inv_ptr[j + 1];
    for (int e = a.inv_ptr[j]; e < e1; ++e) {
        const int ent = a.inv_ent[e];
        const int p = ent >> 10, row = ent & 1023;
        const int base = a.pptr[p];
        const int nn = a.pptr[p + 1] - base;
        const double *m = a.M + a.moff[p] + row * nn;
        const int32_t *dofs = a.pdofs + base;
        for (int c = 0; c < nn; ++c) acc = fma(m[c], a.r[dofs[c]], acc);
    }
    const double eta = *a.eta;
    a.U[j] = a.assign ? eta * acc : fma(eta, acc, a.U[j]);
}

void launch_schwarz_gather(const PatchArgs &a, hipStream_t s) {
    const int grid = padded_grid(blocks_for(a.n));
    hipLaunchKernelGGL(k_schwarz_gather, dim3(grid), dim3(kBlock), 0, s, a);
}

// Coloured scatter form: the subdomains of one colour hold disjoint DOFs, so
// each thread solves one subdomain and adds its damped correction with plain
// read-modify-writes.
__global__ __launch_bounds__(kBlock) void k_schwarz_colour(PatchArgs a, const int32_t *list, int np) {
    if (a.stop && *a.stop) return;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= np) return;
    const int p = list[t];
    const int base = a.pptr[p];
    const int nn = a.pptr[p + 1] - base;
    const int32_t *dofs = a.pdofs + base;
    const double *m = a.M + a.moff[p];
    const double eta = *a.eta;
    for (int row = 0; row < nn; ++row) {
        double acc = 0.0;
        for (int c = 0; c < nn; ++c) acc = fma(m[row * nn + c], a.r[dofs[c]], acc);
        const int g = dofs[row];
        a.U[g] = fma(eta, acc, a.U[g]);
    }
}

void launch_schwarz_colour(const PatchArgs &a, const int32_t *list, int np, hipStream_t s) {
    if (np <= 0) return;
    hipLaunchKernelGGL(k_schwarz_colour, dim3(blocks_for(np)), dim3(kBlock), 0, s, a, list, np);
}

// y = (add ? y : 0) + A x for a CSR matrix (restriction and prolongation).
__global__ __launch_bounds__(kBlock) void k_csr(int nrows, const int32_t *rp, const int32_t *ci, const double *v,
                                                const double *x, double *y, int add, const int *stop) {
    if (stop && *stop) return;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int i = b * kBlock + threadIdx.x;
    if (i >= nrows) return;
    double acc = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) acc = fma(v[e], x[ci[e]], acc);
    y[i] = add ? y[i] + acc : acc;
}

void launch_csr(int nrows, const int32_t *rp, const int32_t *ci, const double *v, const double *x, double *y,
                int add, const int *stop, hipStream_t s) {
    const int grid = padded_grid(blocks_for(nrows));
    hipLaunchKernelGGL(k_csr, dim3(grid), dim3(kBlock), 0, s, nrows, rp, ci, v, x, y, add, stop);
}

// Dense y = A x, one wavefront per row.
__global__ __launch_bounds__(kBlock) void k_gemv(int n, const double *A, const double *x, double *y,
                                                 const int *stop) {
    if (stop && *stop) return;
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    double acc = 0.0;
    for (int j = lane; j < n; j += 64) acc = fma(A[(int64_t)row * n + j], x[j], acc);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if (lane == 0) y[row] = acc;
}

void launch_gemv(int n, const double *A, const double *x, double *y, const int *stop, hipStream_t s) {
    const int rows_per = kBlock / 64;
    hipLaunchKernelGGL(k_gemv, dim3((n + rows_per - 1) / rows_per), dim3(kBlock), 0, s, n, A, x, y, stop);
}

__global__ void k_fill(int64_t n, double *x, double v, const int *stop) {
    if (stop && *stop) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = v;
}
void launch_fill(int64_t n, double *x, double v, const int *stop, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, x, v, stop);
}

__global__ void k_fill_int(int n, int *x, int v) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = v;
}
void launch_fill_int(int n, int *x, int v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, x, v);
}

__global__ void k_copy(int64_t n, const double *x, double *y, const int *stop) {
    if (stop && *stop) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = x[i];
}
void launch_copy(int64_t n, const double *x, double *y, const int *stop, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, x, y, stop);
}

__global__ __launch_bounds__(kBlock) void k_dot_partial(int n, const double *x, const double *y, double *partial) {
    __shared__ double sh[kBlock / 64];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const double v = i < n ? x[i] * y[i] : 0.0;
    const double s = block_sum(v, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
void launch_dot_partial(int n, const double *x, const double *y, double *partial, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_partial, dim3(nblocks), dim3(kBlock), 0, s, n, x, y, partial);
}

__device__ double ordered_sum(int nparts, const double *partial, double *sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kBlock) v += partial[i];
    return block_sum(v, sh);
}

__global__ __launch_bounds__(kBlock) void k_reduce(int nparts, const double *partial, double *out, double scale) {
    __shared__ double sh[kBlock / 64];
    const double s = ordered_sum(nparts, partial, sh);
    if (threadIdx.x == 0) *out = scale * s;
}
void launch_reduce(int nparts, const double *partial, double *out, double scale, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, s, nparts, partial, out, scale);
}

__global__ __launch_bounds__(kBlock) void k_check(int nparts, const double *partial, double *hist, int *counter,
                                                  int *stop, const double *thresh2, int max_hist) {
    if (*stop) return;
    __shared__ double sh[kBlock / 64];
    const double s = ordered_sum(nparts, partial, sh);
    if (threadIdx.x == 0) {
        const int c = *counter;
        const double res = sqrt(s);
        if (c < max_hist) hist[c] = res;
        *counter = c + 1;
        if (!(s <= 1e300)) {
            *stop = 2;  // NaN or Inf
        } else if (s <= *thresh2) {
            *stop = 1;
        } else if (c > 0 && res > 1e6 * hist[0]) {
            *stop = 2;  // growth by six orders: diverging
        }
    }
}
void launch_check(int nparts, const double *partial, double *hist, int *counter, int *stop, const double *thresh2,
                  int max_hist, hipStream_t s) {
    hipLaunchKernelGGL(k_check, dim3(1), dim3(kBlock), 0, s, nparts, partial, hist, counter, stop, thresh2, max_hist);
}

__global__ void k_sub_scalar(int n, double *x, const double *m) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] -= *m;
}
void launch_sub_scalar(int n, double *x, const double *m, hipStream_t s) {
    hipLaunchKernelGGL(k_sub_scalar, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, x, m);
}

// d = coefficients of div u_h in the pressure basis: the derivative of a
// degree k+1 spline in the direction of its component is the scaled forward
// difference c_{j+1} (u_{j+1} - u_j) of degree k splines.
__global__ void k_div(DivArgs a) {
    const int nq = a.N + a.k;
    const int64_t n = (a.d == 2) ? (int64_t)nq * nq : (int64_t)nq * nq * nq;
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= n) return;
    int j[3] = {(int)(g % nq), (int)((g / nq) % nq), a.d == 3 ? (int)(g / ((int64_t)nq * nq)) : 0};
    double dv = 0.0;
    for (int c = 0; c < a.d; ++c) {
        // stored index of u_c in direction c is true index - 1, valid range [0, nq-1)
        auto at = [&](int tc) -> double {
            if (tc <= 0 || tc >= nq) return 0.0;  // removed end functions
            int s[3] = {j[0], j[1], j[2]};
            s[c] = tc - 1;
            return a.U[a.off[c] + s[0] + (int64_t)a.nb[c][0] * (s[1] + (int64_t)a.nb[c][1] * s[2])];
        };
        dv += a.dcoef[j[c] + 1] * (at(j[c] + 1) - at(j[c]));
    }
    a.dvec[g] = dv;
}
void launch_div(const DivArgs &a, hipStream_t s) {
    const int nq = a.N + a.k;
    const int64_t n = (a.d == 2) ? (int64_t)nq * nq : (int64_t)nq * nq * nq;
    hipLaunchKernelGGL(k_div, dim3(blocks_for(n)), dim3(kBlock), 0, s, a);
}

// partial sums of d_i (M_q d)_i, M_q the tensor product of 1D pressure masses.
__global__ __launch_bounds__(kBlock) void k_div_mass(DivArgs a) {
    __shared__ double sh[kBlock / 64];
    const int nq = a.N + a.k, W = 2 * a.k + 1;
    const int64_t n = (a.d == 2) ? (int64_t)nq * nq : (int64_t)nq * nq * nq;
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v = 0.0;
    if (g < n) {
        const int j0 = (int)(g % nq), j1 = (int)((g / nq) % nq), j2 = a.d == 3 ? (int)(g / ((int64_t)nq * nq)) : 0;
        double md = 0.0;
        const int z0 = a.d == 3 ? -a.k : 0, z1 = a.d == 3 ? a.k : 0;
        for (int o2 = z0; o2 <= z1; ++o2) {
            const int i2 = j2 + o2;
            if (i2 < 0 || i2 >= nq) continue;
            const double m2 = a.d == 3 ? a.pmass[j2 * W + o2 + a.k] : 1.0;
            for (int o1 = -a.k; o1 <= a.k; ++o1) {
                const int i1 = j1 + o1;
                if (i1 < 0 || i1 >= nq) continue;
                const double m1 = a.pmass[j1 * W + o1 + a.k];
                for (int o0 = -a.k; o0 <= a.k; ++o0) {
                    const int i0 = j0 + o0;
                    if (i0 < 0 || i0 >= nq) continue;
                    md += m2 * m1 * a.pmass[j0 * W + o0 + a.k] * a.dvec[i0 + (int64_t)nq * (i1 + (int64_t)nq * i2)];
                }
            }
        }
        v = a.dvec[g] * md;
    }
    const double s = block_sum(v, sh);
    if (threadIdx.x == 0) a.partial[blockIdx.x] = s;
}
void launch_div_mass(const DivArgs &a, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_div_mass, dim3(nblocks), dim3(kBlock), 0, s, a);
}

}  // namespace dfmg
