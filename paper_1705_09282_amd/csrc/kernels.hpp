// Device kernels of the V-cycle for gfx950 (wave64).
//
// Batches: every kernel works on a batch of independent problems that share
// one mesh (same dimension, degree, grid and number of levels).  blockIdx.y
// is the problem; arrays that depend on the problem's coefficients (matrix
// values, local inverses, vectors, flags) are offset by the problem index
// times a stride, arrays that depend only on the mesh (index maps, transfer
// operators) are shared.  A single problem is a batch of one.
//
// Every kernel that runs inside a V-cycle takes the per-problem `stop` flags:
// once a problem's residual check has met the tolerance (or detected
// divergence) the remaining kernels leave that problem's outputs untouched,
// so cycles launched ahead of the host check are no-ops for it and its
// iterate is the one at which the check fired.  Launches made once some
// problem has stopped (exit_early) return at once for stopped problems; the
// others read the flag beside their data and skip only the stores (below).
// The cycle kernels take the
// flags in their wide form: kStopLanes copies per problem, lane i of a
// wavefront reading copy i (the check writes all of them).  Kernels whose time
// is set by the latency of their load chains read the flag beside their other
// loads and skip only the stores (a per-lane address keeps the compiler from
// waiting for the flag before the other loads); the bandwidth-bound residual
// of large grids returns before loading anything.
//
// Value type T is double (plain FP64 path) or float (the V-cycle inside the
// FP64 iterative refinement); the coarse-grid matrix is always FP64.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "layout.hpp"

namespace dfmg {

constexpr int kBlock = 256;
constexpr int kStopLanes = 64;  // copies per problem of the wide stop flags
// per-step dampings of a level: kMaxSteps pre-smoothing steps, then
// kMaxSteps post-smoothing steps
constexpr int kMaxSteps = 16;
constexpr int kSchedPerLevel = 2 * kMaxSteps;

// One level's stencil-ELL operator and the vectors of r = F - K U.
template <class T>
struct SpmvArgsT {
    const T *val;
    int64_t sval;       // per-problem stride of val
    int64_t val_off[4];
    int64_t off[5];
    int nb[4][3];
    int n;
    int win;            // boxes stored as in-grid windows (see HostLevel)
    int xc;             // velocity rows couple every velocity component (mapped domain)
    int nt;             // stream the values with non-temporal loads (lanes per row 1)
    int nblocks;        // logical blocks covering n rows (spmv_blocks)
    const T *F;
    const T *U;
    T *r;
    int64_t svec;       // per-problem stride of F, U, r
    double *partial;    // per-block sum of r^2 (nullable)
    int64_t spart;      // per-problem stride of partial
    const int *stop;    // per-problem flags, wide form (nullable)
    int nprob;
    int exit_early;     // 1: stopped problems return at once
};
using SpmvArgs = SpmvArgsT<double>;

// Tile shape of the form-4 local solves (k_patch_solve_small): bs threads per
// workgroup (bs small subdomains, or bs / tb boundary subdomains, per
// workgroup); ms how a workgroup reads an inverse that all its small
// subdomains share (0: scalar loads per wavefront, 1: staged in LDS per
// workgroup, 2: per-thread vector loads); tb threads per boundary subdomain.
// Every shape sums in the same order, so all give the same bits.
struct TileShape {
    int bs = 256, ms = 0, tb = 64;
};

template <class T>
struct PatchArgsT {
    int n;              // DOFs of the level
    int nent;           // entries of all subdomains (sum of their sizes)
    const int32_t *inv_ptr, *inv_pos, *pptr, *pdofs;  // shared
    const int32_t *moff;   // per problem (stride smoff): local-inverse offset of each subdomain
    const int4 *ent_info;  // per problem (stride nent): (M row offset, subdomain start, size, 0)
    T *delta;           // per problem (stride nent): per-entry local corrections
    const T *M;         // per problem (stride sM)
    // form 4, levels whose inverses are mostly per subdomain: those of the
    // small subdomains interleaved in 16-byte chunks (W = 16 / sizeof(T)
    // coefficients), entry e = row * kSmallPatch + c of small subdomain q at
    // ((e / W) * nsmall + q) * W + e % W, per problem (stride kSmallPatch^2 *
    // nsmall); nullptr elsewhere
    const T *msoa;
    // with msoa in the FP32 cycle: the single potential row of each full
    // small subdomain, entry c of subdomain q at c * nsmall + q, per problem
    // (stride kSmallPatch * nsmall)
    const T *qsoa;
    const T *r;
    T *U;               // per problem (stride svec)
    const double *eta;  // per problem (stride seta)
    int64_t smoff, sM, svec, seta;
    int assign;         // 1: U = eta * S r (U known to be zero)
    const int *stop;
    int nprob;
    int exit_early;         // 1: stopped problems return at once
    const int32_t *small;   // subdomains with <= kSmallPatch DOFs (shared)
    const int32_t *bigent;  // entries of the other subdomains (shared)
    const int32_t *small_dofs;  // form 4: DOF c of small subdomain q at c * nsmall + q
    int nsmall, nbig;
    int64_t sdelta;         // per-problem stride of delta (nent + kSmallPatch * nsmall)
    // potential form (FP32 cycle inside the refinement, smoother form 4):
    // beta = Q_i E_i r per local potential, psi += eta * sum of the betas of
    // each potential.  psi is FP64: it is a sum of many local potentials whose
    // differences are the velocity, which FP32 storage would cancel away.
    // psi == nullptr: not tracked.
    double *psi;            // per problem (stride npsi)
    T *beta;                // per problem (stride nbeta)
    const T *Q;             // per problem (stride sQ)
    int64_t sQ, nbeta;
    int npsi, nbigbeta;
    const int32_t *qoff;      // per problem (stride smoff): offset of each subdomain's map in Q
    const int32_t *beta_row;  // per problem (stride nbeta): Q row of each beta entry
    const int32_t *qptr, *beta_patch, *bigbeta, *qinv_ptr, *qinv_pos;  // shared
    // form 4: small subdomain q of problem prob has sinfo[prob * nsmall + q] =
    // (size, offset of its inverse in M, offset of its map in Q, its beta
    // entry); the others (one wavefront each) bmesh[s] = (first entry, size,
    // first beta entry, beta count), shared, and binfo[prob * nbsub + s] =
    // (inverse offset, map offset); max_big = their largest size
    const int4 *sinfo, *bmesh;
    const int2 *binfo;
    int nbsub, max_big;
    // fixed-width forms of the inverse maps in use (inv_w == 0: walk inv_ptr;
    // qinv_w == 0: walk qinv_ptr)
    const int32_t *inv_ell, *qinv_ell;
    int inv_w, qinv_w;
    TileShape tile;         // form 4 only
};
using PatchArgs = PatchArgsT<double>;

// One level of the single-workgroup coarse cycle (k_vcycle_small): the
// level's operator, subdomains and transfers, with vectors and per-problem
// arrays given for problem 0 and the strides of the batch.
template <class T>
struct SmallLevel {
    SpmvArgsT<T> sp;            // operator fields (val, sval, val_off, off, nb, n, win)
    T *F, *U, *r, *delta;       // vectors: stride n; delta: stride sdelta (entry layout)
    int64_t sdelta;
    const T *M;                 // local inverses, stride sM
    int64_t sM, n, nent, smoff;
    const int32_t *pptr, *pdofs, *moff, *inv_ptr, *inv_pos, *small, *bigent;
    const int4 *ent_info;       // stride nent
    int nsmall, nbig;
    const double *eta;          // eta[prob * seta] is this level's damping
    int64_t seta;
    const int32_t *R_rp, *R_ci; // restriction to level l-1 (rows of level l-1)
    const T *R_v;
    const int32_t *P_rp, *P_ci; // prolongation from level l-1 (rows of level l)
    const T *P_v;
    const double *Kinv;         // level 0: dense inverse, stride n * n
    int nu1, nu2;               // smoothing steps of this level
};

// A V-cycle over levels top .. 0 of every problem by one workgroup each
// (levels small enough that launches, not bandwidth, would set the time):
// starts from U_top = 0 on F_top, each level's nu1 / nu2 smoothing steps,
// exact coarse solve; the same sums as the per-level kernels.  lv: device
// array of top + 1 levels.
template <class T>
void launch_vcycle_small(int d, int k, const SmallLevel<T> *lv, int top, const int *stop, int nprob,
                         hipStream_t s);

// blocks of the residual kernel with lpr lanes per row
inline int spmv_blocks(int64_t n, int lpr) { return (int)((n * lpr + 255) / 256); }

template <class T>
void launch_spmv(int d, int k, int lpr, const SpmvArgsT<T> &a, hipStream_t s);
template <class T>
void launch_schwarz_gather(const PatchArgsT<T> &a, hipStream_t s);
// two passes, small subdomains solved by one thread each, in the tile shape
// of a.tile (see TileShape)
template <class T>
void launch_schwarz_small(const PatchArgsT<T> &a, hipStream_t s);
// the second pass alone: U_j += eta * (sum of the corrections of DOF j)
template <class T>
void launch_dof_update(const PatchArgsT<T> &a, hipStream_t s);
// one pass: every DOF recomputes the local-solve rows it receives (no buffer)
template <class T>
void launch_schwarz_fused(const PatchArgsT<T> &a, hipStream_t s);
template <class T>
void launch_schwarz_colour(const PatchArgsT<T> &a, const int32_t *list, int np, hipStream_t s);

// One colour of the multiplicative sweep (equation MSM): for every entry of
// the colour's lane table, the residual row of its DOF from the operator
// (sp: values, F, U, strides, flags), then U += M_i E_i r for every
// subdomain of the colour, in place.
template <class T>
struct MultArgsT {
    SpmvArgsT<T> sp;       // operator and vectors (sp.r unused)
    T *U;                  // the same U as sp.U, written
    const int32_t *lanes;  // this colour's workgroups: entry of thread t of group w at w * width + t, -1 unused
    const int32_t *strides;  // per workgroup: threads between a subdomain's consecutive entries
    int nwaves;
    int width;             // threads per workgroup: kMultLanes or kMultLanesBig
    const int32_t *pdofs;  // shared
    const int4 *ent_info;  // per problem (stride nent): (M row offset, subdomain's first entry, size, 0)
    int64_t nent;
    const T *M;            // per problem (stride sM)
    int64_t sM;
    // the operator rows in lane order (nullptr: read them from sp.val): lane
    // l = lane0 + w * width + t holds its entry's row at (l / 64) * mslots *
    // 64 + (l % 64) * kEllVec, chunks 64 * kEllVec apart; per problem (stride smval)
    const T *mval;
    int64_t smval, lane0;
    int mslots;
};
template <class T>
void launch_schwarz_mult(int d, int k, const MultArgsT<T> &a, hipStream_t s);
// A sparse transfer operator shared by the batch: CSR, and its fixed-width
// form when w > 0 (column u of row i at u * rows + i, index -1 unused).
template <class T>
struct SparseT {
    const int32_t *rp, *ci;
    const T *v;
    int w;
    const int32_t *eci;
    const T *ev;
};
// y = (add ? y : 0) + A x; x, y per problem (strides sx, sy); exit_early as
// in the argument structs (also below)
template <class T>
void launch_csr(int nrows, const SparseT<T> &A, const T *x, int64_t sx, T *y, int64_t sy, int add, const int *stop,
                int nprob, hipStream_t s, int exit_early = 0);
// the FP32 cycle's prolongation of the velocity-pressure correction (P) and
// of the potentials (Ps, FP64) in one launch, both added
template <class T>
void launch_prolong_pair(int nu, const SparseT<T> &P, const T *xu, int64_t sxu, T *yu, int64_t syu, int nps,
                         const SparseT<double> &Ps, const double *xp, int64_t sxp, double *yp, int64_t syp,
                         const int *stop, int nprob, hipStream_t s, int exit_early = 0);
// the FP32 cycle's coarse solve y = Kinv x and its potentials psi = Q0 x
// (FP64 matrices, n x n and nps x n per problem) in one launch
void launch_coarse_pair(int n, int nps, const double *Kinv, int64_t sK, const double *Q0, int64_t sQ, const float *x,
                        int64_t sx, float *y, int64_t sy, double *psi, int64_t sp, const int *stop, int nprob,
                        hipStream_t s, int exit_early = 0);
// y = A x with A row-major FP64 (rows x cols) per problem (stride sA), x, y in
// T, FP64 accumulation
template <class T>
void launch_gemv(int rows, int cols, const double *A, int64_t sA, const T *x, int64_t sx, T *y, int64_t sy,
                 const int *stop, int nprob, hipStream_t s, int exit_early = 0);
// y (FP64) = A x with x in FP32 (the coarse potentials of the FP32 cycle)
void launch_gemv_f2d(int rows, int cols, const double *A, int64_t sA, const float *x, int64_t sx, double *y,
                     int64_t sy, const int *stop, int nprob, hipStream_t s, int exit_early = 0);
template <class T>
void launch_fill(int64_t n, T *x, int64_t sx, T v, const int *stop, int nprob, hipStream_t s, int exit_early = 0);
void launch_fill_int(int n, int *x, int v, hipStream_t s);
void launch_copy_int(int n, const int *x, int *y, hipStream_t s);
void launch_copy(int64_t n, const double *x, int64_t sx, double *y, int64_t sy, const int *stop, int nprob,
                 hipStream_t s);
// problem p: y[yoff[p] + i] = x[xoff[p] + i], i < n; a null offset table
// means p * stride (used for vectors of problems laid out in the caller's order)
void launch_copy_off(int64_t n, const double *x, const int64_t *xoff, int64_t sx, double *y, const int64_t *yoff,
                     int64_t sy, int nprob, hipStream_t s);
void launch_cast(int64_t n, const double *x, float *y, int64_t svec, const int *stop, int nprob, hipStream_t s,
                 int exit_early = 0);
// per problem: partial[p * spart + b] = block sums of x . y
void launch_dot_partial(int n, const double *x, const double *y, int64_t sxy, double *partial, int64_t spart,
                        int nblocks, int nprob, hipStream_t s);
// per problem: out[p] = scale * sum(partial[p * spart + 0 .. nparts))  (fixed order)
void launch_reduce(int nparts, const double *partial, int64_t spart, double *out, double scale, int nprob,
                   hipStream_t s);
// Learned-damping fallback used by the residual check: when a V-cycle after
// the first contracts problem p's residual by more than 1.05 * rho[p], or the
// residual has grown by six orders, its dampings eta[p][1..L-1] are reset to
// eta_fixed[p][..] and flag[p] is set (once; growth then means divergence).
// With a per-step damping schedule in use (sched, [p][level][kSchedPerLevel])
// every step of level l takes eta_fixed[p][l] as well.
struct Fallback {
    const double *rho;        // nullable: no fallback
    double *eta;
    const double *eta_fixed;
    double *sched;            // nullable: no schedule
    int *flag;
    int L;
};
// per problem residual check: hist[p][counter[p]] = sqrt(sum), stop[p] = 1 if
// sum <= thresh2[p], 2 on NaN/Inf/growth; stopw[p * kStopLanes + i] = stop[p]
// (the wide form the cycle kernels read); near[p] = 1 when the problem has
// stopped or, contracting as in its last cycle, will meet the threshold at
// the next check (a hint for the host's launch-ahead, no effect on results)
void launch_check(int nparts, const double *partial, int64_t spart, double *hist, int max_hist, int *counter,
                  int *stop, int *stopw, int *near, const double *thresh2, const Fallback &fb, int nprob,
                  hipStream_t s);
// per problem: x[p * sx + i] -= m[p] for i < n
void launch_sub_scalar(int n, double *x, int64_t sx, const double *m, int nprob, hipStream_t s);

// FP64 update of the refinement loop (2D): U += [curl psi; X_p] with psi the
// streamfunction coefficients of the FP32 cycle's velocity correction.
struct RefineArgs {
    int d, N, k;
    int64_t off_uy, off_uz, off_p, n;  // block offsets of the finest level (off_uz = off_p in 2D)
    const float *X;            // FP32 correction (pressure part used)
    const double *psi;         // potentials per problem: 2D (N+k-1)^2; 3D three components, see k_curl_update_3d
    const double *dcoef;
    double *U;
    int64_t svec, spsi;
    const int *stop;
    int nprob;
    int exit_early;
};
void launch_refine_update(const RefineArgs &a, hipStream_t s);

// Quadrature part of the Crank-Nicolson / Adams-Bashforth load (finest
// grid): G = weighted integrand 2 sigma u - 3 (u . grad) u + (uo . grad) uo
// at every quadrature point (first step, Uold null: - 2 (u . grad) u), then
// Fout_i += (N_i, G) on the velocity rows and Fout = 0 on the pressure rows.
struct CnabArgs {
    int d, k, N, nq;        // nq Gauss points per direction per element
    int64_t off[4];         // block offsets (velocity components, then pressure)
    int nb[3][3];           // stored functions per velocity component and direction
    int64_t n, svec;        // rows and per-problem vector stride
    const double *bval, *bder;  // [degree k / k+1][element][point][local function (k+2)]
    const double *wq;       // per direction: quadrature weights times h / 2
    const double *U, *Uold; // per problem (Uold nullable)
    const double *sigma;    // per problem
    double *G;              // per problem (stride sG): [point][component]
    int64_t sG, npts;
    double *Fout;
    int nprob;
    int conv;               // 1: the Adams-Bashforth convective terms; 0: none (2 sigma u only)
};
void launch_cnab_load(const CnabArgs &a, hipStream_t s);

// div-norm pieces (finest grid, one problem)
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
