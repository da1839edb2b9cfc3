// Device kernels of the V-cycle for gfx950 (wave64).  Every kernel that runs
// inside a V-cycle takes `stop`: once the residual check of the current solve
// has met the tolerance (or detected divergence) the remaining kernels of that
// cycle leave their outputs untouched, so cycles launched ahead of the host
// check are no-ops and the iterate is the one at which the check fired.
//
// Value type T is double (plain FP64 path) or float (the V-cycle inside the
// FP64 iterative refinement); the coarse-grid matrix is always FP64.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dfmg {

constexpr int kBlock = 256;

// One level's stencil-ELL operator and the vectors of r = F - K U.
template <class T>
struct SpmvArgsT {
    const T *val;
    int64_t val_off[4];
    int64_t off[5];
    int nb[4][3];
    int n;
    int nblocks;  // logical blocks covering n rows (spmv_blocks)
    const T *F;
    const T *U;
    T *r;
    double *partial;  // per-block sum of r^2 (nullable)
    const int *stop;  // nullable
};
using SpmvArgs = SpmvArgsT<double>;

template <class T>
struct PatchArgsT {
    int n;              // DOFs of the level
    int nent;           // entries of all subdomains (sum of their sizes)
    const int32_t *inv_ptr, *inv_pos, *pptr, *pdofs, *moff;
    const int4 *ent_info;  // per entry: (M row offset, subdomain start, subdomain size, 0)
    T *delta;           // per-entry local corrections
    const T *M;
    const T *r;
    T *U;
    const double *eta;  // device scalar
    int assign;         // 1: U = eta * S r (U known to be zero)
    const int *stop;
};
using PatchArgs = PatchArgsT<double>;

// blocks of the residual kernel with lpr lanes per row
inline int spmv_blocks(int64_t n, int lpr) { return (int)((n * lpr + 255) / 256); }

template <class T>
void launch_spmv(int d, int k, int lpr, const SpmvArgsT<T> &a, hipStream_t s);
template <class T>
void launch_schwarz_gather(const PatchArgsT<T> &a, hipStream_t s);
template <class T>
void launch_schwarz_colour(const PatchArgsT<T> &a, const int32_t *list, int np, hipStream_t s);
template <class T>
void launch_csr(int nrows, const int32_t *rp, const int32_t *ci, const T *v, const T *x, T *y, int add,
                const int *stop, hipStream_t s);
// y = A x with A row-major FP64 (rows x cols), x, y in T, FP64 accumulation
template <class T>
void launch_gemv(int rows, int cols, const double *A, const T *x, T *y, const int *stop, hipStream_t s);
template <class T>
void launch_fill(int64_t n, T *x, T v, const int *stop, hipStream_t s);
void launch_fill_int(int n, int *x, int v, hipStream_t s);
void launch_copy(int64_t n, const double *x, double *y, const int *stop, hipStream_t s);
void launch_cast(int64_t n, const double *x, float *y, const int *stop, hipStream_t s);
void launch_dot_partial(int n, const double *x, const double *y, double *partial, int nblocks, hipStream_t s);
// out = scale * sum(partial[0..nparts))  (single block, fixed order)
void launch_reduce(int nparts, const double *partial, double *out, double scale, hipStream_t s);
// residual check: hist[*counter] = sqrt(sum); stop = 1 if sum <= *thresh2, 2 on NaN/Inf/growth
void launch_check(int nparts, const double *partial, double *hist, int *counter, int *stop, const double *thresh2,
                  int max_hist, hipStream_t s);
// x[i] -= *m for i < n
void launch_sub_scalar(int n, double *x, const double *m, hipStream_t s);

// FP64 update of the refinement loop (2D): recover the streamfunction
// increment psi from the x-velocity part of the FP32 correction X by
// integrating along y, then U += [curl psi; X_p].
struct RefineArgs {
    int N, k;
    int64_t off_uy, off_p, n;  // block offsets of the finest level
    const float *X;
    const double *dcoef;
    double *psi;               // (N+k-1)^2
    double *U;
    const int *stop;
};
void launch_refine_update_2d(const RefineArgs &a, hipStream_t s);

// div-norm pieces (finest grid)
struct DivArgs {
    int d, k, N;
    int64_t off[4];
    int nb[4][3];
    const double *U;
    const double *dcoef;
    const double *pmass;
    double *dvec;
    double *partial;
};
void launch_div(const DivArgs &a, hipStream_t s);
void launch_div_mass(const DivArgs &a, int nblocks, hipStream_t s);

inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }
// Grid size used by the XCD-aware launches: logical blocks rounded up to 8.
inline int padded_grid(int nblocks) { return ((nblocks + 7) / 8) * 8; }

}  // namespace dfmg
