// HIP kernels of the additive-Schwarz V-cycle (gfx950, wave64).
#include "schwarz_dev.hpp"

namespace dfmg {

// Additive Schwarz, step 1: local solves.  Thread t owns entry t of the
// subdomain-major correction buffer, i.e. local row m of subdomain p with
// t = pptr[p] + m, and computes delta_t = (M_p E_p r)_m.
template <class T>
__global__ __launch_bounds__(kBlock) void k_patch_solve(PatchArgsT<T> a) {
    const int prob = blockIdx.y;
    if (a.stop && a.stop[prob]) return;  // block-uniform: the problem has stopped
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int t = b * kBlock + threadIdx.x;
    if (t >= a.nent) return;
    // descriptor of entry t: offset of its row of M, first entry of its
    // subdomain, subdomain size
    const int4 info = a.ent_info[(int64_t)prob * a.nent + t];
    a.delta[prob * a.sdelta + t] = patch_row(a.M + prob * a.sM + info.x, a.pdofs + info.y, info.z, a.r + prob * a.svec);
}

// Additive Schwarz, step 1 with one thread per small subdomain (at most
// kSmallPatch DOFs, the interior ones): the thread gathers its subdomain's
// residual entries once (its DOFs are stored subdomain-minor, so the loads
// coalesce) and computes every row of M_p E_p r, written row-major over the
// small subdomains (coalesced stores).  Blocks past nb_small take one entry
// each of the larger (boundary) subdomains as k_patch_solve does.  Every row
// is summed in the order of k_patch_solve, so the corrections agree bit for
// bit; k_dof_update reads them through the relabelled inverse map.
template <class T>
__global__ __launch_bounds__(kBlock) void k_patch_solve_small(PatchArgsT<T> a, int nb_small) {
    const int prob = blockIdx.y;
    if (a.stop && a.stop[prob]) return;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const T *r = a.r + prob * a.svec;
    T *delta = a.delta + prob * a.sdelta;
    if (b < nb_small) {
        const int q = b * kBlock + threadIdx.x;
        if (q >= a.nsmall) return;
        const int p = a.small[q];
        const int nn = a.pptr[p + 1] - a.pptr[p];
        T rv[kSmallPatch];
        gather_small(a.small_dofs + q, a.nsmall, nn, r, rv);
        apply_small(a.M + prob * a.sM + a.moff[(int64_t)prob * a.smoff + p], nn, rv, delta + q, a.nsmall);
        if (a.psi)  // the subdomain's single potential
            a.beta[prob * a.nbeta + a.qptr[p]] = small_row(a.Q + prob * a.sQ + a.qoff[prob * a.smoff + p], nn, rv);
        return;
    }
    const int t = (b - nb_small) * kBlock + threadIdx.x;
    if (t < a.nbig) {
        const int e = a.bigent[t];
        const int4 info = a.ent_info[(int64_t)prob * a.nent + e];
        delta[(int64_t)kSmallPatch * a.nsmall + e] = patch_row(a.M + prob * a.sM + info.x, a.pdofs + info.y, info.z, r);
    } else if (a.psi && t < a.nbig + a.nbigbeta) {
        const int e = a.bigbeta[t - a.nbig], p = a.beta_patch[e];
        const int base = a.pptr[p];
        a.beta[prob * a.nbeta + e] =
            patch_row(a.Q + prob * a.sQ + a.beta_row[prob * a.nbeta + e], a.pdofs + base, a.pptr[p + 1] - base, r);
    }
}

// Additive Schwarz, step 2: U_j += eta * sum of the corrections of every
// subdomain holding DOF j (fixed order, no atomics).
template <class T>
__global__ __launch_bounds__(kBlock) void k_dof_update(PatchArgsT<T> a) {
    const int prob = blockIdx.y;
    if (a.stop && a.stop[prob]) return;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int j = b * kBlock + threadIdx.x;
    const T eta = (T)a.eta[prob * a.seta];
    if (j >= a.n) {  // potentials (tracked in the FP32 cycle)
        const int pj = j - a.n;
        if (!a.psi || pj >= a.npsi) return;
        double *psi = a.psi + (int64_t)prob * a.npsi;
        const double u = a.assign ? 0.0 : psi[pj];
        psi[pj] = fma((double)eta, (double)dof_sum(a.qinv_ptr, a.qinv_pos, a.beta + prob * a.nbeta, pj), u);
        return;
    }
    T *U = a.U + prob * a.svec;
    const T *delta = a.delta + prob * a.sdelta;
    const T u = a.assign ? T(0) : U[j];
    U[j] = fma(eta, dof_sum(a.inv_ptr, a.inv_pos, delta, j), u);
}

template <class T>
void launch_schwarz_gather(const PatchArgsT<T> &a, hipStream_t s) {
    hipLaunchKernelGGL(k_patch_solve<T>, dim3(padded_grid(blocks_for(a.nent)), a.nprob), dim3(kBlock), 0, s, a);
    hipLaunchKernelGGL(k_dof_update<T>, dim3(padded_grid(blocks_for(a.n)), a.nprob), dim3(kBlock), 0, s, a);
}

// One-pass form: DOF j recomputes the rows of the local solves that land on
// it, (M_i E_i r)_m for every entry (i, m) with dofs_i[m] = j, and adds their
// damped sum -- no correction buffer and one launch.  Each row is summed in
// the same order as k_patch_solve and the rows in the same order as
// k_dof_update, so the result equals the two-pass form bit for bit.
template <class T>
__global__ __launch_bounds__(kBlock) void k_schwarz_fused(PatchArgsT<T> a) {
    const int prob = blockIdx.y;
    if (a.stop && a.stop[prob]) return;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int j = b * kBlock + threadIdx.x;
    const T *r = a.r + prob * a.svec;
    const T eta = (T)a.eta[prob * a.seta];
    if (j >= a.n) {  // potentials: the betas landing on potential pj, recomputed
        const int pj = j - a.n;
        if (!a.psi || pj >= a.npsi) return;
        double *psi = a.psi + (int64_t)prob * a.npsi;
        const double u = a.assign ? 0.0 : psi[pj];
        const T *Q = a.Q + prob * a.sQ;
        const int32_t *brow = a.beta_row + prob * a.nbeta;
        T acc = 0;
        for (int e = a.qinv_ptr[pj]; e < a.qinv_ptr[pj + 1]; ++e) {
            const int be = a.qinv_pos[e], p = a.beta_patch[be];
            acc += patch_row(Q + brow[be], a.pdofs + a.pptr[p], a.pptr[p + 1] - a.pptr[p], r);
        }
        psi[pj] = fma((double)eta, (double)acc, u);
        return;
    }
    T *U = a.U + prob * a.svec;
    const T *M = a.M + prob * a.sM;
    const int4 *ent = a.ent_info + (int64_t)prob * a.nent;
    const T u = a.assign ? T(0) : U[j];
    T acc = 0;
    const int e0 = a.inv_ptr[j], e1 = a.inv_ptr[j + 1];
    for (int e = e0; e < e1; ++e) {
        const int4 info = ent[a.inv_pos[e]];
        acc += patch_row(M + info.x, a.pdofs + info.y, info.z, r);
    }
    U[j] = fma(eta, acc, u);
}

template <class T>
void launch_schwarz_small(const PatchArgsT<T> &a, hipStream_t s) {
    const int nbs = blocks_for(a.nsmall), nbb = blocks_for(a.nbig + (a.psi ? a.nbigbeta : 0));
    hipLaunchKernelGGL(k_patch_solve_small<T>, dim3(padded_grid(nbs + nbb), a.nprob), dim3(kBlock), 0, s, a, nbs);
    const int64_t rows = a.n + (a.psi ? a.npsi : 0);
    hipLaunchKernelGGL(k_dof_update<T>, dim3(padded_grid(blocks_for(rows)), a.nprob), dim3(kBlock), 0, s, a);
}

template <class T>
void launch_schwarz_fused(const PatchArgsT<T> &a, hipStream_t s) {
    const int64_t rows = a.n + (a.psi ? a.npsi : 0);
    hipLaunchKernelGGL(k_schwarz_fused<T>, dim3(padded_grid(blocks_for(rows)), a.nprob), dim3(kBlock), 0, s, a);
}

// Coloured scatter form: the subdomains of one colour hold disjoint DOFs, so
// each thread solves one subdomain and adds its damped correction with plain
// read-modify-writes.
template <class T>
__global__ __launch_bounds__(kBlock) void k_schwarz_colour(PatchArgsT<T> a, const int32_t *list, int np) {
    const int prob = blockIdx.y;
    if (a.stop && a.stop[prob]) return;
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= np) return;
    const int p = list[t];
    const int base = a.pptr[p];
    const int nn = a.pptr[p + 1] - base;
    const int32_t *dofs = a.pdofs + base;
    const T *m = a.M + prob * a.sM + a.moff[prob * a.smoff + p];
    const T *r = a.r + prob * a.svec;
    T *U = a.U + prob * a.svec;
    const T eta = (T)a.eta[prob * a.seta];
    for (int row = 0; row < nn; ++row) {
        T acc = 0;
        for (int c = 0; c < nn; ++c) acc = fma(m[row * nn + c], r[dofs[c]], acc);
        const int g = dofs[row];
        U[g] = fma(eta, acc, U[g]);
    }
}

template <class T>
void launch_schwarz_colour(const PatchArgsT<T> &a, const int32_t *list, int np, hipStream_t s) {
    if (np <= 0) return;
    hipLaunchKernelGGL(k_schwarz_colour<T>, dim3(blocks_for(np), a.nprob), dim3(kBlock), 0, s, a, list, np);
}

// y = (add ? y : 0) + A x for a CSR matrix (restriction and prolongation).
template <class T>
__global__ __launch_bounds__(kBlock) void k_csr(int nrows, const int32_t *rp, const int32_t *ci, const T *v,
                                                const T *x, int64_t sx, T *y, int64_t sy, int add,
                                                const int *stop) {
    const int prob = blockIdx.y;
    if (stop && stop[prob]) return;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int i = b * kBlock + threadIdx.x;
    if (i >= nrows) return;
    x += prob * sx;
    y += prob * sy;
    const T y0 = add ? y[i] : T(0);
    y[i] = y0 + csr_row(rp, ci, v, x, i);
}

template <class T>
void launch_csr(int nrows, const int32_t *rp, const int32_t *ci, const T *v, const T *x, int64_t sx, T *y,
                int64_t sy, int add, const int *stop, int nprob, hipStream_t s) {
    const dim3 grid(padded_grid(blocks_for(nrows)), nprob);
    hipLaunchKernelGGL(k_csr<T>, grid, dim3(kBlock), 0, s, nrows, rp, ci, v, x, sx, y, sy, add, stop);
}

// Dense y = A x (A FP64, row-major rows x cols), one wavefront per row, FP64
// accumulation.
template <class T>
__global__ __launch_bounds__(kBlock) void k_gemv(int rows, int cols, const double *A, int64_t sA, const T *x,
                                                 int64_t sx, T *y, int64_t sy, const int *stop) {
    const int prob = blockIdx.y;
    if (stop && stop[prob]) return;
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= rows) return;
    const double acc = gemv_row_wave(A + prob * sA, cols, x + prob * sx, row, lane);
    if (lane == 0) y[prob * sy + row] = (T)acc;
}

template <class T>
void launch_gemv(int rows, int cols, const double *A, int64_t sA, const T *x, int64_t sx, T *y, int64_t sy,
                 const int *stop, int nprob, hipStream_t s) {
    const int rows_per = kBlock / 64;
    hipLaunchKernelGGL(k_gemv<T>, dim3((rows + rows_per - 1) / rows_per, nprob), dim3(kBlock), 0, s, rows, cols, A,
                       sA, x, sx, y, sy, stop);
}

__global__ __launch_bounds__(kBlock) void k_gemv_f2d(int rows, int cols, const double *A, int64_t sA, const float *x,
                                                     int64_t sx, double *y, int64_t sy, const int *stop) {
    const int prob = blockIdx.y;
    if (stop && stop[prob]) return;
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= rows) return;
    const double acc = gemv_row_wave(A + prob * sA, cols, x + prob * sx, row, lane);
    if (lane == 0) y[prob * sy + row] = acc;
}

void launch_gemv_f2d(int rows, int cols, const double *A, int64_t sA, const float *x, int64_t sx, double *y,
                     int64_t sy, const int *stop, int nprob, hipStream_t s) {
    const int rows_per = kBlock / 64;
    hipLaunchKernelGGL(k_gemv_f2d, dim3((rows + rows_per - 1) / rows_per, nprob), dim3(kBlock), 0, s, rows, cols, A,
                       sA, x, sx, y, sy, stop);
}

template <class T>
__global__ void k_fill(int64_t n, T *x, int64_t sx, T v, const int *stop) {
    const int prob = blockIdx.y;
    if (stop && stop[prob]) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[prob * sx + i] = v;
}
template <class T>
void launch_fill(int64_t n, T *x, int64_t sx, T v, const int *stop, int nprob, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks_for(n), nprob), dim3(kBlock), 0, s, n, x, sx, v, stop);
}

__global__ void k_cast(int64_t n, const double *x, float *y, int64_t sv, const int *stop) {
    const int prob = blockIdx.y;
    if (stop && stop[prob]) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[prob * sv + i] = (float)x[prob * sv + i];
}
void launch_cast(int64_t n, const double *x, float *y, int64_t svec, const int *stop, int nprob, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_cast, dim3(blocks_for(n), nprob), dim3(kBlock), 0, s, n, x, y, svec, stop);
}

// U += [curl psi; X_p] in FP64, curl psi = (d_y psi, -d_x psi) by the scaled
// differences of the derivative formula (psi = 0 on the boundary).
__global__ void k_curl_update_2d(RefineArgs a) {
    const int prob = blockIdx.y;
    if (a.stop && a.stop[prob]) return;
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= a.n) return;
    const int m = a.N + a.k - 1, nq = a.N + a.k;
    const double *P = a.psi + prob * a.spsi;
    auto psi = [&](int pa, int pb) -> double {  // true indices, zero on the boundary
        if (pa <= 0 || pa >= nq || pb <= 0 || pb >= nq) return 0.0;
        return P[(pa - 1) + (int64_t)m * (pb - 1)];
    };
    double du;
    if (g < a.off_uy) {  // u_x(a, j): stored (a-1, j), dims m x nq
        const int ia = (int)(g % m), j = (int)(g / m);
        du = a.dcoef[j + 1] * (psi(ia + 1, j + 1) - psi(ia + 1, j));
    } else if (g < a.off_p) {  // u_y(i, b): stored (i, b-1), dims nq x m
        const int64_t l = g - a.off_uy;
        const int i = (int)(l % nq), ib = (int)(l / nq);
        du = -a.dcoef[i + 1] * (psi(i + 1, ib + 1) - psi(i, ib + 1));
    } else {
        du = (double)a.X[prob * a.svec + g];
    }
    a.U[prob * a.svec + g] += du;
}

void launch_refine_update_2d(const RefineArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_curl_update_2d, dim3(blocks_for(a.n), a.nprob), dim3(kBlock), 0, s, a);
}

template void launch_schwarz_gather<double>(const PatchArgsT<double> &, hipStream_t);
template void launch_schwarz_gather<float>(const PatchArgsT<float> &, hipStream_t);
template void launch_schwarz_fused<double>(const PatchArgsT<double> &, hipStream_t);
template void launch_schwarz_small<double>(const PatchArgsT<double> &, hipStream_t);
template void launch_schwarz_small<float>(const PatchArgsT<float> &, hipStream_t);
template void launch_schwarz_fused<float>(const PatchArgsT<float> &, hipStream_t);
template void launch_schwarz_colour<double>(const PatchArgsT<double> &, const int32_t *, int, hipStream_t);
template void launch_schwarz_colour<float>(const PatchArgsT<float> &, const int32_t *, int, hipStream_t);
template void launch_csr<double>(int, const int32_t *, const int32_t *, const double *, const double *, int64_t,
                                 double *, int64_t, int, const int *, int, hipStream_t);
template void launch_csr<float>(int, const int32_t *, const int32_t *, const float *, const float *, int64_t, float *,
                                int64_t, int, const int *, int, hipStream_t);
template void launch_gemv<double>(int, int, const double *, int64_t, const double *, int64_t, double *, int64_t,
                                  const int *, int, hipStream_t);
template void launch_gemv<float>(int, int, const double *, int64_t, const float *, int64_t, float *, int64_t,
                                 const int *, int, hipStream_t);
template void launch_fill<double>(int64_t, double *, int64_t, double, const int *, int, hipStream_t);
template void launch_fill<float>(int64_t, float *, int64_t, float, const int *, int, hipStream_t);

__global__ void k_fill_int(int n, int *x, int v) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = v;
}
void launch_fill_int(int n, int *x, int v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, x, v);
}

__global__ void k_copy(int64_t n, const double *x, int64_t sx, double *y, int64_t sy, const int *stop) {
    const int prob = blockIdx.y;
    if (stop && stop[prob]) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[prob * sy + i] = x[prob * sx + i];
}
void launch_copy(int64_t n, const double *x, int64_t sx, double *y, int64_t sy, const int *stop, int nprob,
                 hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy, dim3(blocks_for(n), nprob), dim3(kBlock), 0, s, n, x, sx, y, sy, stop);
}

__global__ void k_copy_int(int n, const int *x, int *y) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) y[i] = x[i];
}
void launch_copy_int(int n, const int *x, int *y, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_copy_int, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, x, y);
}

// problem p's vector at x + xoff[p] (or p * sx) copied to y + yoff[p] (or p * sy)
__global__ void k_copy_off(int64_t n, const double *x, const int64_t *xoff, int64_t sx, double *y,
                           const int64_t *yoff, int64_t sy) {
    const int prob = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t xo = xoff ? xoff[prob] : prob * sx, yo = yoff ? yoff[prob] : prob * sy;
    y[yo + i] = x[xo + i];
}
void launch_copy_off(int64_t n, const double *x, const int64_t *xoff, int64_t sx, double *y, const int64_t *yoff,
                     int64_t sy, int nprob, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy_off, dim3(blocks_for(n), nprob), dim3(kBlock), 0, s, n, x, xoff, sx, y, yoff, sy);
}

__global__ __launch_bounds__(kBlock) void k_dot_partial(int n, const double *x, const double *y, int64_t sxy,
                                                        double *partial, int64_t spart) {
    __shared__ double sh[kBlock / 64];
    const int prob = blockIdx.y;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const double v = i < n ? x[prob * sxy + i] * y[prob * sxy + i] : 0.0;
    const double s = block_sum(v, sh);
    if (threadIdx.x == 0) partial[prob * spart + blockIdx.x] = s;
}
void launch_dot_partial(int n, const double *x, const double *y, int64_t sxy, double *partial, int64_t spart,
                        int nblocks, int nprob, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_partial, dim3(nblocks, nprob), dim3(kBlock), 0, s, n, x, y, sxy, partial, spart);
}

__device__ double ordered_sum(int nparts, const double *partial, double *sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kBlock) v += partial[i];
    return block_sum(v, sh);
}

__global__ __launch_bounds__(kBlock) void k_reduce(int nparts, const double *partial, int64_t spart, double *out,
                                                   double scale) {
    __shared__ double sh[kBlock / 64];
    const int prob = blockIdx.x;
    const double s = ordered_sum(nparts, partial + prob * spart, sh);
    if (threadIdx.x == 0) out[prob] = scale * s;
}
void launch_reduce(int nparts, const double *partial, int64_t spart, double *out, double scale, int nprob,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_reduce, dim3(nprob), dim3(kBlock), 0, s, nparts, partial, spart, out, scale);
}

__global__ __launch_bounds__(kBlock) void k_check(int nparts, const double *partial, int64_t spart, double *hist,
                                                  int max_hist, int *counter, int *stop, const double *thresh2,
                                                  Fallback fb) {
    const int prob = blockIdx.x;
    if (stop[prob]) return;
    __shared__ double sh[kBlock / 64];
    const double s = ordered_sum(nparts, partial + prob * spart, sh);
    if (threadIdx.x == 0) {
        double *h = hist + (int64_t)prob * max_hist;
        const int c = counter[prob];
        const double res = sqrt(s);
        if (c < max_hist) h[c] = res;
        counter[prob] = c + 1;
        const bool grow = c > 0 && res > 1e6 * h[0];  // growth by six orders: diverging
        const bool can_fall = fb.rho && fb.rho[prob] > 0.0 && !fb.flag[prob];
        if (!(s <= 1e300)) {
            stop[prob] = 2;  // NaN or Inf
        } else if (s <= thresh2[prob]) {
            stop[prob] = 1;
        } else if (can_fall && (grow || (c >= 2 && c <= max_hist && res > 1.05 * fb.rho[prob] * h[c - 1]))) {
            // the learned dampings contract worse than the fixed ones did:
            // continue with the fixed dampings (the iteration stays linear,
            // so the iterate so far is a valid starting guess)
            fb.flag[prob] = 1;
            for (int l = 1; l < fb.L; ++l) fb.eta[(int64_t)prob * fb.L + l] = fb.eta_fixed[(int64_t)prob * fb.L + l];
        } else if (grow) {
            stop[prob] = 2;
        }
    }
}
void launch_check(int nparts, const double *partial, int64_t spart, double *hist, int max_hist, int *counter,
                  int *stop, const double *thresh2, const Fallback &fb, int nprob, hipStream_t s) {
    hipLaunchKernelGGL(k_check, dim3(nprob), dim3(kBlock), 0, s, nparts, partial, spart, hist, max_hist, counter,
                       stop, thresh2, fb);
}

__global__ void k_sub_scalar(int n, double *x, int64_t sx, const double *m) {
    const int prob = blockIdx.y;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[prob * sx + i] -= m[prob];
}
void launch_sub_scalar(int n, double *x, int64_t sx, const double *m, int nprob, hipStream_t s) {
    hipLaunchKernelGGL(k_sub_scalar, dim3(blocks_for(n), nprob), dim3(kBlock), 0, s, n, x, sx, m);
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
