// Device kernels of the V-cycle for gfx950 (wave64).  Every kernel that runs
// inside a V-cycle takes `stop`: when the residual check of the current solve
// has already met the tolerance (or detected divergence) the remaining
// kernels of that cycle return at once, so cycles launched ahead of the host
// check are no-ops and the iterate is the one at which the check fired.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace dfmg {

constexpr int kBlock = 256;

// One level's stencil-ELL operator, FP64.
struct SpmvArgs {
    const double *val;
    int64_t val_off[4];
    int64_t off[5];
    int nb[4][3];
    int n;
    int nblocks;  // logical blocks covering n rows
    const double *F;
    const double *U;
    double *r;
    double *partial;  // per-block sum of r^2 (nullable)
    const int *stop;  // nullable
};

struct PatchArgs {
    int n;              // DOFs of the level
    int nent;           // entries of all subdomains (sum of their sizes)
    const int32_t *inv_ptr, *inv_pos, *pptr, *pdofs, *moff;
    const int4 *ent_info;  // per entry: (M row offset, subdomain start, subdomain size, 0)
    double *delta;      // per-entry local corrections
    const double *M;
    const double *r;
    double *U;
    const double *eta;  // device scalar
    int assign;         // 1: U = eta * S r (U known to be zero)
    const int *stop;
};

void launch_spmv(int d, int k, int lpr, const SpmvArgs &a, hipStream_t s);
// blocks of the residual kernel with lpr lanes per row
inline int spmv_blocks(int64_t n, int lpr) { return (int)((n * lpr + 255) / 256); }
void launch_schwarz_gather(const PatchArgs &a, hipStream_t s);
void launch_schwarz_colour(const PatchArgs &a, const int32_t *list, int np, hipStream_t s);
void launch_csr(int nrows, const int32_t *rp, const int32_t *ci, const double *v, const double *x, double *y,
                int add, const int *stop, hipStream_t s);
void launch_gemv(int n, const double *A, const double *x, double *y, const int *stop, hipStream_t s);
void launch_fill(int64_t n, double *x, double v, const int *stop, hipStream_t s);
void launch_fill_int(int n, int *x, int v, hipStream_t s);
void launch_copy(int64_t n, const double *x, double *y, const int *stop, hipStream_t s);
void launch_dot_partial(int n, const double *x, const double *y, double *partial, int nblocks, hipStream_t s);
// out = scale * sum(partial[0..nparts))  (single block, fixed order)
void launch_reduce(int nparts, const double *partial, double *out, double scale, hipStream_t s);
// residual check: hist[*counter] = sqrt(sum); stop = 1 if sum <= *thresh2, 2 on NaN/Inf/growth
void launch_check(int nparts, const double *partial, double *hist, int *counter, int *stop, const double *thresh2,
                  int max_hist, hipStream_t s);
// x[i] -= *m for i < n
void launch_sub_scalar(int n, double *x, const double *m, hipStream_t s);
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
