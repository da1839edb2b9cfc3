// HIP kernels of the additive-Schwarz V-cycle (gfx950, wave64).
#include "schwarz_dev.hpp"

namespace dfmg {

// Additive Schwarz, step 1: local solves.  Thread t owns entry t of the
// subdomain-major correction buffer, i.e. local row m of subdomain p with
// t = pptr[p] + m, and computes delta_t = (M_p E_p r)_m.
template <class T>
__global__ __launch_bounds__(kBlock) void k_patch_solve(PatchArgsT<T> a) {
    const int prob = blockIdx.y;
    if (stop_flag(a.stop, prob)) return;  // block-uniform: the problem has stopped
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int t = b * kBlock + threadIdx.x;
    if (t >= a.nent) return;
    // descriptor of entry t: offset of its row of M, first entry of its
    // subdomain, subdomain size
    const int4 info = a.ent_info[(int64_t)prob * a.nent + t];
    a.delta[prob * a.sdelta + t] = patch_row(a.M + prob * a.sM + info.x, a.pdofs + info.y, info.z, a.r + prob * a.svec);
}

// Additive Schwarz, step 2: U_j += eta * sum of the corrections of every
// subdomain holding DOF j (fixed order, no atomics), from the fixed-width
// inverse map padded to WB columns (WB == 0: walk inv_ptr).  Blocks from nbu
// on take the potentials tracked by the FP32 cycle: psi += eta * sum of their
// betas (a block-uniform split, so neither part waits for the other's loads).
template <int WB, bool EXIT, class T>
__global__ __launch_bounds__(kBlock) void k_dof_update(PatchArgsT<T> a, int nbu) {
    const int prob = blockIdx.y;
    const int halt = stop_flag(a.stop, prob);  // gates the stores
    if (EXIT && halt) return;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const double eta = uniform_vload(a.eta + prob * a.seta);  // converted at its uses
    if (b >= nbu) {
        const int pj = (b - nbu) * kBlock + threadIdx.x;
        if (!a.psi || pj >= a.npsi) return;
        double *psi = a.psi + (int64_t)prob * a.npsi;
        const T *beta = a.beta + prob * a.nbeta;
        const double u = a.assign ? 0.0 : psi[pj];
        T sum;
        if (WB > 0 && a.qinv_w > 0 && a.qinv_w <= WB) sum = ell_sum<(WB > 0 ? WB : 1)>(a.qinv_ell, a.npsi, a.qinv_w, pj, beta);
        else sum = dof_sum(a.qinv_ptr, a.qinv_pos, beta, pj);
        if (!halt) psi[pj] = fma((double)(T)eta, (double)sum, u);  // the cycle's damping in T
        return;
    }
    const int j = b * kBlock + threadIdx.x;
    if (j >= a.n) return;
    T *U = a.U + prob * a.svec;
    const T *delta = a.delta + prob * a.sdelta;
    const T u = a.assign ? T(0) : U[j];
    T sum;
    if (WB > 0 && a.inv_w > 0 && a.inv_w <= WB) sum = ell_sum<(WB > 0 ? WB : 1)>(a.inv_ell, a.n, a.inv_w, j, delta);
    else sum = dof_sum(a.inv_ptr, a.inv_pos, delta, j);
    if (!halt) U[j] = fma((T)eta, sum, u);
}

// the DOF update with the width bucket of the level's inverse maps
template <int WB, class T>
static void launch_dof_w(const PatchArgsT<T> &a, dim3 grid, int nbu, hipStream_t s) {
    if (a.exit_early) hipLaunchKernelGGL((k_dof_update<WB, true, T>), grid, dim3(kBlock), 0, s, a, nbu);
    else hipLaunchKernelGGL((k_dof_update<WB, false, T>), grid, dim3(kBlock), 0, s, a, nbu);
}

template <class T>
void launch_dof_update(const PatchArgsT<T> &a, hipStream_t s) {
    int w = ell_bucket(a.inv_w);
    if (a.psi && a.qinv_w > 0) w = w ? std::max(w, ell_bucket(a.qinv_w)) : 0;
    const int nbu = blocks_for(a.n), nbp = a.psi ? blocks_for(a.npsi) : 0;
    const dim3 grid(padded_grid(nbu + nbp), a.nprob);
    if (w == 4) launch_dof_w<4, T>(a, grid, nbu, s);
    else if (w == 8) launch_dof_w<8, T>(a, grid, nbu, s);
    else if (w == 12) launch_dof_w<12, T>(a, grid, nbu, s);
    else if (w == 24) launch_dof_w<24, T>(a, grid, nbu, s);
    else launch_dof_w<0, T>(a, grid, nbu, s);
}

template <class T>
void launch_schwarz_gather(const PatchArgsT<T> &a, hipStream_t s) {
    hipLaunchKernelGGL(k_patch_solve<T>, dim3(padded_grid(blocks_for(a.nent)), a.nprob), dim3(kBlock), 0, s, a);
    launch_dof_update<T>(a, s);
}

// One-pass form: DOF j recomputes the rows of the local solves that land on
// it, (M_i E_i r)_m for every entry (i, m) with dofs_i[m] = j, and adds their
// damped sum -- no correction buffer and one launch.  Each row is summed in
// the same order as k_patch_solve and the rows in the same order as
// k_dof_update, so the result equals the two-pass form bit for bit.
template <class T>
__global__ __launch_bounds__(kBlock) void k_schwarz_fused(PatchArgsT<T> a) {
    const int prob = blockIdx.y;
    if (stop_flag(a.stop, prob)) return;
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
void launch_schwarz_fused(const PatchArgsT<T> &a, hipStream_t s) {
    const int64_t rows = a.n + (a.psi ? a.npsi : 0);
    hipLaunchKernelGGL(k_schwarz_fused<T>, dim3(padded_grid(blocks_for(rows)), a.nprob), dim3(kBlock), 0, s, a);
}

// Coloured scatter form: the subdomains of one colour hold disjoint DOFs, so
// each subdomain adds its damped correction with plain read-modify-writes.
// One wavefront per subdomain: the lanes gather its residual entries into
// LDS, then lane t sums row t (the order of patch_row) and updates DOF t.
template <class T>
__global__ __launch_bounds__(kBlock) void k_schwarz_colour(PatchArgsT<T> a, const int32_t *list, int np, int width) {
    const int prob = blockIdx.y;
    const int halt = stop_flag(a.stop, prob);
    extern __shared__ unsigned char smem[];
    T *sr = reinterpret_cast<T *>(smem) + (threadIdx.x >> 6) * width;
    const int lane = threadIdx.x & 63;
    const int t = __builtin_amdgcn_readfirstlane(blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6));
    const bool live = t < np;
    const int p = live ? list[t] : 0;
    const int base = a.pptr[p];
    const int nn = live ? a.pptr[p + 1] - base : 0;
    const int32_t *dofs = a.pdofs + base;
    const T *m = a.M + prob * a.sM + a.moff[prob * a.smoff + p];
    const T *r = a.r + prob * a.svec;
    T *U = a.U + prob * a.svec;
    const T eta = (T)uniform_vload(a.eta + prob * a.seta);
    for (int c = lane; c < nn; c += 64) sr[c] = r[dofs[c]];
    __syncthreads();
    for (int row = lane; row < nn; row += 64) {
        T acc = 0;
        for (int c = 0; c < nn; ++c) acc = fma(m[row * nn + c], sr[c], acc);
        const int g = dofs[row];
        const T u = U[g];
        if (!halt) U[g] = fma(eta, acc, u);
    }
}

template <class T>
void launch_schwarz_colour(const PatchArgsT<T> &a, const int32_t *list, int np, hipStream_t s) {
    if (np <= 0) return;
    constexpr int waves = kBlock / 64;
    const int width = std::max(a.max_big, kSmallPatch);
    hipLaunchKernelGGL(k_schwarz_colour<T>, dim3((np + waves - 1) / waves, a.nprob), dim3(kBlock),
                       (size_t)waves * width * sizeof(T), s, a, list, np, width);
}

// y = (add ? y : 0) + A x for a sparse transfer operator (restriction and
// prolongation), from its fixed-width form padded to WB columns (WB == 0:
// CSR).
template <int WB, bool EXIT, class T>
__global__ __launch_bounds__(kBlock) void k_csr(int nrows, SparseT<T> A, const T *x, int64_t sx, T *y, int64_t sy,
                                                int add, const int *stop) {
    const int prob = blockIdx.y;
    const int halt = stop_flag(stop, prob);  // gates the store
    if (EXIT && halt) return;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int i = b * kBlock + threadIdx.x;
    if (i >= nrows) return;
    x += prob * sx;
    y += prob * sy;
    const T y0 = add ? y[i] : T(0);
    T v;
    if (WB > 0 && A.w > 0 && A.w <= WB) v = ell_row<(WB > 0 ? WB : 1)>(A.eci, A.ev, nrows, A.w, i, x);
    else v = csr_row(A.rp, A.ci, A.v, x, i);
    if (!halt) y[i] = y0 + v;
}

template <int WB, class T>
static void launch_csr_w(dim3 grid, int nrows, const SparseT<T> &A, const T *x, int64_t sx, T *y, int64_t sy, int add,
                         const int *stop, hipStream_t s, int exit_early) {
    if (exit_early) hipLaunchKernelGGL((k_csr<WB, true, T>), grid, dim3(kBlock), 0, s, nrows, A, x, sx, y, sy, add, stop);
    else hipLaunchKernelGGL((k_csr<WB, false, T>), grid, dim3(kBlock), 0, s, nrows, A, x, sx, y, sy, add, stop);
}

template <class T>
void launch_csr(int nrows, const SparseT<T> &A, const T *x, int64_t sx, T *y, int64_t sy, int add, const int *stop,
                int nprob, hipStream_t s, int exit_early) {
    const dim3 grid(padded_grid(blocks_for(nrows)), nprob);
    const int w = ell_bucket(A.w);
    if (w == 4) launch_csr_w<4, T>(grid, nrows, A, x, sx, y, sy, add, stop, s, exit_early);
    else if (w == 8) launch_csr_w<8, T>(grid, nrows, A, x, sx, y, sy, add, stop, s, exit_early);
    else if (w == 12) launch_csr_w<12, T>(grid, nrows, A, x, sx, y, sy, add, stop, s, exit_early);
    else if (w == 24) launch_csr_w<24, T>(grid, nrows, A, x, sx, y, sy, add, stop, s, exit_early);
    else launch_csr_w<0, T>(grid, nrows, A, x, sx, y, sy, add, stop, s, exit_early);
}

// The prolongations of the FP32 cycle in one launch: blocks below nbu add
// P dU to the velocity-pressure rows (T), the others add Ps psi_coarse to
// the potentials (FP64), each from its fixed-width form padded to WB / WQ
// columns (0: CSR).  The same sums as two k_csr launches.
template <int WB, int WQ, bool EXIT, class T>
__global__ __launch_bounds__(kBlock) void k_prolong_pair(int nu, SparseT<T> P, const T *xu, int64_t sxu, T *yu,
                                                         int64_t syu, int nps, SparseT<double> Ps, const double *xp,
                                                         int64_t sxp, double *yp, int64_t syp, int nbu,
                                                         const int *stop) {
    const int prob = blockIdx.y;
    const int halt = stop_flag(stop, prob);
    if (EXIT && halt) return;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    if (b < nbu) {
        const int i = b * kBlock + threadIdx.x;
        if (i >= nu) return;
        xu += prob * sxu;
        yu += prob * syu;
        const T y0 = yu[i];
        T v;
        if (WB > 0 && P.w > 0 && P.w <= WB) v = ell_row<(WB > 0 ? WB : 1)>(P.eci, P.ev, nu, P.w, i, xu);
        else v = csr_row(P.rp, P.ci, P.v, xu, i);
        if (!halt) yu[i] = y0 + v;
        return;
    }
    const int i = (b - nbu) * kBlock + threadIdx.x;
    if (i >= nps) return;
    xp += prob * sxp;
    yp += prob * syp;
    const double y0 = yp[i];
    double v;
    if (WQ > 0 && Ps.w > 0 && Ps.w <= WQ) v = ell_row<(WQ > 0 ? WQ : 1)>(Ps.eci, Ps.ev, nps, Ps.w, i, xp);
    else v = csr_row(Ps.rp, Ps.ci, Ps.v, xp, i);
    if (!halt) yp[i] = y0 + v;
}

template <class T>
void launch_prolong_pair(int nu, const SparseT<T> &P, const T *xu, int64_t sxu, T *yu, int64_t syu, int nps,
                         const SparseT<double> &Ps, const double *xp, int64_t sxp, double *yp, int64_t syp,
                         const int *stop, int nprob, hipStream_t s, int exit_early) {
    const int bp = ell_bucket(P.w), bq = ell_bucket(Ps.w);
    const int nbu = blocks_for(nu);
    const dim3 grid(padded_grid(nbu + blocks_for(nps)), nprob);
#define DFMG_PAIR(W, Q)                                                                                        \
    do {                                                                                                       \
        if (exit_early)                                                                                        \
            hipLaunchKernelGGL((k_prolong_pair<W, Q, true, T>), grid, dim3(kBlock), 0, s, nu, P, xu, sxu, yu, syu, \
                               nps, Ps, xp, sxp, yp, syp, nbu, stop);                                          \
        else                                                                                                   \
            hipLaunchKernelGGL((k_prolong_pair<W, Q, false, T>), grid, dim3(kBlock), 0, s, nu, P, xu, sxu, yu,     \
                               syu, nps, Ps, xp, sxp, yp, syp, nbu, stop);                                     \
    } while (0)
    // the widths that occur in 2D (P: 4 or 8; P^psi: 4 or 12), else CSR for both
    if (bp == 4 && bq == 4) DFMG_PAIR(4, 4);
    else if (bp == 4 && bq == 12) DFMG_PAIR(4, 12);
    else if (bp == 8 && bq == 4) DFMG_PAIR(8, 4);
    else if (bp == 8 && bq == 12) DFMG_PAIR(8, 12);
    else if (bp == 8 && bq == 8) DFMG_PAIR(8, 8);
    else if (bp == 4 && bq == 8) DFMG_PAIR(4, 8);
    else DFMG_PAIR(0, 0);
#undef DFMG_PAIR
}

// The exact coarse solve of the FP32 cycle with the potentials of its
// solution in one launch: rows below n give y = Kinv x (T), the others
// psi = Q0 x (FP64); one wavefront per row, FP64 accumulation.
__global__ __launch_bounds__(kBlock) void k_coarse_pair(int n, int nps, const double *Kinv, int64_t sK,
                                                        const double *Q0, int64_t sQ, const float *x, int64_t sx,
                                                        float *y, int64_t sy, double *psi, int64_t sp,
                                                        const int *stop, int exit_early) {
    const int prob = blockIdx.y;
    const int halt = stop_flag(stop, prob);
    if (exit_early && halt) return;
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n + nps) return;
    if (row < n) {
        const double acc = gemv_row_wave(Kinv + prob * sK, n, x + prob * sx, row, lane);
        if (lane == 0 && !halt) y[prob * sy + row] = (float)acc;
    } else {
        const double acc = gemv_row_wave(Q0 + prob * sQ, n, x + prob * sx, row - n, lane);
        if (lane == 0 && !halt) psi[prob * sp + row - n] = acc;
    }
}

void launch_coarse_pair(int n, int nps, const double *Kinv, int64_t sK, const double *Q0, int64_t sQ, const float *x,
                        int64_t sx, float *y, int64_t sy, double *psi, int64_t sp, const int *stop, int nprob,
                        hipStream_t s, int exit_early) {
    const int rows_per = kBlock / 64;
    hipLaunchKernelGGL(k_coarse_pair, dim3((n + nps + rows_per - 1) / rows_per, nprob), dim3(kBlock), 0, s, n, nps,
                       Kinv, sK, Q0, sQ, x, sx, y, sy, psi, sp, stop, exit_early);
}

// Dense y = A x (A FP64, row-major rows x cols), one wavefront per row, FP64
// accumulation.
template <class T>
__global__ __launch_bounds__(kBlock) void k_gemv(int rows, int cols, const double *A, int64_t sA, const T *x,
                                                 int64_t sx, T *y, int64_t sy, const int *stop, int exit_early) {
    const int prob = blockIdx.y;
    const int halt = stop_flag(stop, prob);  // block-uniform; gates the store
    if (exit_early && halt) return;
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= rows) return;
    const double acc = gemv_row_wave(A + prob * sA, cols, x + prob * sx, row, lane);
    if (lane == 0 && !halt) y[prob * sy + row] = (T)acc;
}

template <class T>
void launch_gemv(int rows, int cols, const double *A, int64_t sA, const T *x, int64_t sx, T *y, int64_t sy,
                 const int *stop, int nprob, hipStream_t s, int exit_early) {
    const int rows_per = kBlock / 64;
    hipLaunchKernelGGL(k_gemv<T>, dim3((rows + rows_per - 1) / rows_per, nprob), dim3(kBlock), 0, s, rows, cols, A,
                       sA, x, sx, y, sy, stop, exit_early);
}

__global__ __launch_bounds__(kBlock) void k_gemv_f2d(int rows, int cols, const double *A, int64_t sA, const float *x,
                                                     int64_t sx, double *y, int64_t sy, const int *stop,
                                                     int exit_early) {
    const int prob = blockIdx.y;
    const int halt = stop_flag(stop, prob);
    if (exit_early && halt) return;
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= rows) return;
    const double acc = gemv_row_wave(A + prob * sA, cols, x + prob * sx, row, lane);
    if (lane == 0 && !halt) y[prob * sy + row] = acc;
}

void launch_gemv_f2d(int rows, int cols, const double *A, int64_t sA, const float *x, int64_t sx, double *y,
                     int64_t sy, const int *stop, int nprob, hipStream_t s, int exit_early) {
    const int rows_per = kBlock / 64;
    hipLaunchKernelGGL(k_gemv_f2d, dim3((rows + rows_per - 1) / rows_per, nprob), dim3(kBlock), 0, s, rows, cols, A,
                       sA, x, sx, y, sy, stop, exit_early);
}

template <class T>
__global__ void k_fill(int64_t n, T *x, int64_t sx, T v, const int *stop) {
    const int prob = blockIdx.y;
    const int halt = stop_flag(stop, prob);
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n && !halt) x[prob * sx + i] = v;
}
template <class T>
void launch_fill(int64_t n, T *x, int64_t sx, T v, const int *stop, int nprob, hipStream_t s, int) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks_for(n), nprob), dim3(kBlock), 0, s, n, x, sx, v, stop);
}

__global__ void k_cast(int64_t n, const double *x, float *y, int64_t sv, const int *stop, int exit_early) {
    const int prob = blockIdx.y;
    const int halt = stop_flag(stop, prob);
    if (exit_early && halt) return;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const float v = (float)x[prob * sv + i];
    if (!halt) y[prob * sv + i] = v;
}
void launch_cast(int64_t n, const double *x, float *y, int64_t svec, const int *stop, int nprob, hipStream_t s,
                 int exit_early) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_cast, dim3(blocks_for(n), nprob), dim3(kBlock), 0, s, n, x, y, svec, stop, exit_early);
}

// U += [curl psi; X_p] in FP64, curl psi = (d_y psi, -d_x psi) by the scaled
// differences of the derivative formula (psi = 0 on the boundary).
__global__ void k_curl_update_2d(RefineArgs a) {
    const int prob = blockIdx.y;
    const int halt = stop_flag(a.stop, prob);  // block-uniform; gates the store
    if (a.exit_early && halt) return;
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
    const double u = a.U[prob * a.svec + g];
    if (!halt) a.U[prob * a.svec + g] = u + du;
}

// 3D: U_g += (curl psi)_g on the velocity rows (u_x = d_y psi_z - d_z psi_y,
// u_y = d_z psi_x - d_x psi_z, u_z = d_x psi_y - d_y psi_x), U_g += X_g on the
// pressure rows.  Component o of psi has N + k functions in direction o
// (degree k, all kept) and N + k - 1 in the others (degree k + 1 without the
// end functions), stored component after component, x fastest; the
// derivative of a degree-(k+1) spline expansion in direction j at
// degree-k index t is c_{t+1} (psi(t + e_j) - psi(t)), with the removed end
// functions zero.
__global__ void k_curl_update_3d(RefineArgs a) {
    const int prob = blockIdx.y;
    const int halt = stop_flag(a.stop, prob);  // block-uniform; gates the store
    if (a.exit_early && halt) return;
    const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (g >= a.n) return;
    const int nq = a.N + a.k, m = nq - 1;
    const int64_t ncomp = (int64_t)nq * m * m;
    const double *P = a.psi + prob * a.spsi;
    // potential o at true index (t0, t1, t2); zero outside the kept box
    auto psi = [&](int o, int t0, int t1, int t2) -> double {
        const int t[3] = {t0, t1, t2};
        int64_t idx = 0, stride = 1;
        for (int j = 0; j < 3; ++j) {
            const int lo = j == o ? 0 : 1;
            if (t[j] < lo || t[j] >= nq) return 0.0;
            idx += (int64_t)(t[j] - lo) * stride;
            stride *= j == o ? nq : m;
        }
        return P[o * ncomp + idx];
    };
    double du;
    if (g < a.off_p) {
        const int R = g < a.off_uy ? 0 : (g < a.off_uz ? 1 : 2);
        int64_t l = g - (R == 0 ? 0 : (R == 1 ? a.off_uy : a.off_uz));
        int t[3];
        for (int j = 0; j < 3; ++j) {  // velocity component R keeps N + k - 1 functions in direction R
            const int nb = j == R ? m : nq;
            t[j] = (int)(l % nb) + (j == R ? 1 : 0);
            l /= nb;
        }
        auto d = [&](int o, int dir) {
            int u[3] = {t[0], t[1], t[2]};
            u[dir] += 1;
            return a.dcoef[t[dir] + 1] * (psi(o, u[0], u[1], u[2]) - psi(o, t[0], t[1], t[2]));
        };
        if (R == 0) du = d(2, 1) - d(1, 2);
        else if (R == 1) du = d(0, 2) - d(2, 0);
        else du = d(1, 0) - d(0, 1);
    } else {
        du = (double)a.X[prob * a.svec + g];
    }
    const double u = a.U[prob * a.svec + g];
    if (!halt) a.U[prob * a.svec + g] = u + du;
}

void launch_refine_update(const RefineArgs &a, hipStream_t s) {
    if (a.d == 3) hipLaunchKernelGGL(k_curl_update_3d, dim3(blocks_for(a.n), a.nprob), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL(k_curl_update_2d, dim3(blocks_for(a.n), a.nprob), dim3(kBlock), 0, s, a);
}

template void launch_schwarz_gather<double>(const PatchArgsT<double> &, hipStream_t);
template void launch_schwarz_gather<float>(const PatchArgsT<float> &, hipStream_t);
template void launch_schwarz_fused<double>(const PatchArgsT<double> &, hipStream_t);
template void launch_dof_update<double>(const PatchArgsT<double> &, hipStream_t);
template void launch_dof_update<float>(const PatchArgsT<float> &, hipStream_t);
template void launch_schwarz_fused<float>(const PatchArgsT<float> &, hipStream_t);
template void launch_schwarz_colour<double>(const PatchArgsT<double> &, const int32_t *, int, hipStream_t);
template void launch_schwarz_colour<float>(const PatchArgsT<float> &, const int32_t *, int, hipStream_t);
template void launch_csr<double>(int, const SparseT<double> &, const double *, int64_t, double *, int64_t, int,
                                 const int *, int, hipStream_t, int);
template void launch_csr<float>(int, const SparseT<float> &, const float *, int64_t, float *, int64_t, int, const int *,
                                int, hipStream_t, int);
template void launch_prolong_pair<float>(int, const SparseT<float> &, const float *, int64_t, float *, int64_t, int,
                                         const SparseT<double> &, const double *, int64_t, double *, int64_t,
                                         const int *, int, hipStream_t, int);
template void launch_gemv<double>(int, int, const double *, int64_t, const double *, int64_t, double *, int64_t,
                                  const int *, int, hipStream_t, int);
template void launch_gemv<float>(int, int, const double *, int64_t, const float *, int64_t, float *, int64_t,
                                 const int *, int, hipStream_t, int);
template void launch_fill<double>(int64_t, double *, int64_t, double, const int *, int, hipStream_t, int);
template void launch_fill<float>(int64_t, float *, int64_t, float, const int *, int, hipStream_t, int);

__global__ void k_fill_int(int n, int *x, int v) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) x[i] = v;
}
void launch_fill_int(int n, int *x, int v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_int, dim3(blocks_for(n)), dim3(kBlock), 0, s, n, x, v);
}

__global__ void k_copy(int64_t n, const double *x, int64_t sx, double *y, int64_t sy, const int *stop) {
    const int prob = blockIdx.y;
    if (stop_flag(stop, prob)) return;
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
                                                  int max_hist, int *counter, int *stop, int *stopw,
                                                  int *near, const double *thresh2, Fallback fb) {
    const int prob = blockIdx.x;
    if (stop[prob]) return;
    __shared__ double sh[kBlock / 64];
    __shared__ int flag;
    const double s = ordered_sum(nparts, partial + prob * spart, sh);
    if (threadIdx.x == 0) {
        double *h = hist + (int64_t)prob * max_hist;
        const int c = counter[prob];
        const double res = sqrt(s);
        if (c < max_hist) h[c] = res;
        counter[prob] = c + 1;
        const bool grow = c > 0 && res > 1e6 * h[0];  // growth by six orders: diverging
        const bool can_fall = fb.rho && fb.rho[prob] > 0.0 && !fb.flag[prob];
        int f = 0;
        if (!(s <= 1e300)) {
            f = 2;  // NaN or Inf
        } else if (s <= thresh2[prob]) {
            f = 1;
        } else if (can_fall && (grow || (c >= 2 && c <= max_hist && res > 1.05 * fb.rho[prob] * h[c - 1]))) {
            // the learned dampings contract worse than the fixed ones did:
            // continue with the fixed dampings (the iteration stays linear,
            // so the iterate so far is a valid starting guess)
            fb.flag[prob] = 1;
            for (int l = 1; l < fb.L; ++l) {
                const double e = fb.eta_fixed[(int64_t)prob * fb.L + l];
                fb.eta[(int64_t)prob * fb.L + l] = e;
                if (fb.sched)
                    for (int j = 0; j < kSchedPerLevel; ++j)
                        fb.sched[((int64_t)prob * fb.L + l) * kSchedPerLevel + j] = e;
            }
        } else if (grow) {
            f = 2;
        }
        if (f) stop[prob] = f;
        flag = f;
        // contracting as in the last cycle, the next check meets the threshold
        const double next = (c > 0 && c <= max_hist && h[c - 1] > 0.0) ? res * (res / h[c - 1]) : 1e300;
        near[prob] = (f || (c < max_hist && next * next <= thresh2[prob])) ? 1 : 0;
    }
    __syncthreads();
    if (flag && threadIdx.x < kStopLanes) stopw[prob * kStopLanes + threadIdx.x] = flag;
}
void launch_check(int nparts, const double *partial, int64_t spart, double *hist, int max_hist, int *counter,
                  int *stop, int *stopw, int *near, const double *thresh2, const Fallback &fb, int nprob,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_check, dim3(nprob), dim3(kBlock), 0, s, nparts, partial, spart, hist, max_hist, counter,
                       stop, stopw, near, thresh2, fb);
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

// partial sums of d_i (M_q d)_i, M_q the tensor product of 1D pressure masses
// (one per direction: on a mapped domain they carry the factors of 1 / det J).
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
            const double m2 = a.d == 3 ? a.pmass[(2 * nq + j2) * W + o2 + a.k] : 1.0;
            for (int o1 = -a.k; o1 <= a.k; ++o1) {
                const int i1 = j1 + o1;
                if (i1 < 0 || i1 >= nq) continue;
                const double m1 = a.pmass[(nq + j1) * W + o1 + a.k];
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
