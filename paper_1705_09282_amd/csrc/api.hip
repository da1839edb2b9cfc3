// C-ABI of the library: context, workspace binding, V-cycle orchestration,
// solve loop, diagnostics and exports.  See include/dfmg.h.
//
// A context holds a batch of problems on one mesh (a single problem is a
// batch of one).  Mesh-only data (index maps, transfer operators, pressure
// integrals) is stored once; coefficient-dependent data (matrix values, local
// inverses, coarse inverse, damping) and all vectors are stored per problem
// with a fixed stride, and every kernel launch covers the whole batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "../../include/dfmg.h"
#include "kernels.hpp"
#include "mlp.hpp"
#include "setup.hpp"

using namespace dfmg;

namespace {

thread_local std::string g_err;

struct HipError : std::runtime_error {
    using std::runtime_error::runtime_error;
};
struct StateError : std::runtime_error {
    using std::runtime_error::runtime_error;
};
struct ArgError : std::runtime_error {
    using std::runtime_error::runtime_error;
};

#define HIPCHK(x)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) throw HipError(std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

// flag arrays per problem (adjacent on the device and in the host copies):
// counter, stop, near
constexpr int kFlagSets = 3;
// flag states read by the host loop (bits)
constexpr int kAllNear = 1, kAllStopped = 2, kAnyStopped = 4;

// Typed values and vectors of one level: FP64 for the plain path, FP32 for
// the V-cycle inside the iterative refinement.  Per problem unless noted.
template <class T>
struct LevelData {
    T *val = nullptr, *U = nullptr, *F = nullptr, *r = nullptr, *M = nullptr, *delta = nullptr;
    T *P_v = nullptr, *R_v = nullptr;  // shared by the batch
    T *P_ev = nullptr, *R_ev = nullptr;  // fixed-width forms (when stored)
    T *mval = nullptr;  // multiplicative sweep: the operator rows in lane order (FP64 only)
    T *msoa = nullptr;  // the small subdomains' inverses interleaved (levels with per-subdomain inverses)
};

struct DevLevel {
    LevelData<double> d;
    LevelData<float> f;
    // shared by the batch
    int32_t *pptr = nullptr, *pdofs = nullptr, *inv_ptr = nullptr, *inv_pos = nullptr, *col_list = nullptr;
    int32_t *small = nullptr, *bigent = nullptr, *small_dofs = nullptr, *inv_pos4 = nullptr;
    int32_t *P_rp = nullptr, *P_ci = nullptr, *R_rp = nullptr, *R_ci = nullptr;
    int32_t *P_eci = nullptr, *R_eci = nullptr, *inv_ell = nullptr, *inv4_ell = nullptr;
    int32_t *mlane = nullptr;  // lane table of the multiplicative sweep
    int32_t *mstride = nullptr;  // its per-workgroup entry strides
    bool soa = false;  // the small subdomains' inverses also stored interleaved (msoa)
    int4 *bmesh = nullptr;
    // per problem (form 4): small-subdomain and remaining-subdomain tables
    int4 *sinfo = nullptr;
    int2 *binfo = nullptr;
    // per problem
    int32_t *moff = nullptr;
    int4 *ent_info = nullptr;
    double *Kinv = nullptr;
    // potential form of the FP32 cycle (precision 1, 2D)
    double *psi = nullptr, *Ps_v = nullptr;  // psi per problem (FP64: see PatchArgsT)
    float *beta = nullptr, *Q = nullptr;     // per problem
    float *qsoa = nullptr;  // the small subdomains' potential rows interleaved (with msoa)
    int32_t *qoff = nullptr, *qptr = nullptr, *beta_row = nullptr, *beta_patch = nullptr, *bigbeta = nullptr,
            *qinv_ptr = nullptr, *qinv_pos = nullptr, *Ps_rp = nullptr, *Ps_ci = nullptr;
    int32_t *qinv_ell = nullptr, *Ps_eci = nullptr;
    double *Ps_ev = nullptr;
    double *Q0 = nullptr;  // level 0, per problem
    int64_t npsi = 0, nbeta = 0, sQ = 0;
    // strides
    int64_t sval = 0, sM = 0, nent = 0, n = 0, sdelta = 0;
    int64_t smval = 0;  // per-problem stride of the lane-ordered rows (lanes x mslots)
    int mslots = 0;     // slots per lane-ordered row (the level's widest row block)
    template <class T>
    LevelData<T> &data();
};
template <>
LevelData<double> &DevLevel::data<double>() { return d; }
template <>
LevelData<float> &DevLevel::data<float>() { return f; }

// Bump allocator over the caller's workspace (256-byte aligned pieces).  With
// base == nullptr it only measures.
struct Arena {
    char *base = nullptr;
    size_t used = 0;
    template <class T>
    T *take(size_t count) {
        used = (used + 255) & ~(size_t)255;
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += count * sizeof(T);
        return p;
    }
};

}  // namespace

struct dfmg_ctx {
    std::vector<Hierarchy> P;  // one per problem, identical meshes
    int np = 1;
    dfmg_options opt{};
    bool bound = false;
    hipStream_t user = nullptr, s = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<DevLevel> dl;
    double *eta = nullptr;       // [problem][level]
    double *partial = nullptr;   // [problem][block]
    int nparts = 0;
    double *hist = nullptr;      // [problem][DFMG_MAX_HISTORY]
    // adjacent: counter, stop = counter + np, near = counter + 2 np (stopped or
    // expected to stop at the next check)
    int *counter = nullptr, *stop = nullptr, *near = nullptr;
    int *stopw = nullptr;        // wide copies of stop read by the cycle kernels
    int *hflags = nullptr;       // pinned host copies of counter, stop and near, two buffers
    hipEvent_t ev_flag[2] = {nullptr, nullptr};
    double *thresh2 = nullptr, *scal = nullptr;
    double *dvec = nullptr, *dcoef = nullptr, *pmass = nullptr, *rtmp = nullptr, *wfine = nullptr;
    // learned damping
    float *mlpW = nullptr, *feat = nullptr;
    double *rho_plain = nullptr, *eta_fixed = nullptr;
    int *fallback = nullptr;
    bool learned = false;
    // captured cycles, one per exit mode (0: FP64 cycle, 1: FP64 cycle with
    // check, 2: refinement step)
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_kind[2] = {-1, -1};
    // 1 once a problem of the running solve has stopped: launches return at
    // once for stopped problems instead of loading and skipping their stores
    int exit_mode = 0;
    std::vector<int> smoother;   // per level: 1 gather, 2 colour, 3 one-pass, 4 small-subdomain gather
    int small_top = 0;           // levels 1 .. small_top (and 0) run in the single-workgroup cycle; 0 = off
    SmallLevel<double> *small_d = nullptr;  // device level tables of that cycle
    SmallLevel<float> *small_f = nullptr;
    std::vector<int> lpr;        // per level: lanes per row of the residual kernel
    std::vector<TileShape> tile; // per level: tile shape of the form-4 local solves
    std::vector<int> nu1l, nu2l; // per level: pre- and post-smoothing steps
    std::vector<double> eta_host;  // [problem][level]
    // Chebyshev damping schedule (when sched_on): the smoothing steps of
    // level l take the dampings sched[p][l][..] instead of eta[p][l]
    double *sched = nullptr;       // device [problem][level][kSchedPerLevel]
    double *sched0 = nullptr;      // device copy as built (a fallback overwrites sched)
    double *unit = nullptr;        // device [problem]: 1.0 (undamped smoother, eigenvalue estimates)
    float *mlpZ = nullptr;         // device [problem][MLP_OUT]: network outputs
    // Crank-Nicolson / Adams-Bashforth load (options.time_stepping)
    double *qbval = nullptr, *qbder = nullptr, *qw = nullptr, *qG = nullptr, *fstep = nullptr, *sigma_dev = nullptr;
    int64_t npts = 0;
    bool sched_on = false;
    std::vector<double> alpha;     // [problem][level]: ratio b / a of the Chebyshev interval [a, b]
    std::vector<double> lmax;      // [problem][level]: estimate of the largest |eigenvalue| of S^-1 K
    std::vector<double> sched_host;
    const Hierarchy &S() const { return P[0]; }
    int L() const { return P[0].pb.L; }
    bool mixed() const { return opt.precision == 1; }
    bool mult() const { return opt.multiplicative == 1; }
};

namespace {

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

template <class F>
int guarded(F &&f) {
    try {
        f();
        return DFMG_OK;
    } catch (const ArgError &e) {
        return fail(DFMG_EINVAL, e.what());
    } catch (const StateError &e) {
        return fail(DFMG_ESTATE, e.what());
    } catch (const HipError &e) {
        return fail(DFMG_EHIP, e.what());
    } catch (const std::bad_alloc &) {
        return fail(DFMG_ENOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(DFMG_EINVAL, e.what());
    }
}

template <class T>
void take_level(Arena &A, const DevLevel &dv, int np, LevelData<T> &v, bool coarse, const HostLevel &h) {
    v.U = A.take<T>(dv.n * np);
    v.F = A.take<T>(dv.n * np);
    v.r = A.take<T>(dv.n * np);
    v.val = A.take<T>(dv.sval * np);
    if (coarse) return;
    v.M = A.take<T>(dv.sM * np);
    v.delta = A.take<T>(dv.sdelta * np);
    v.P_v = A.take<T>(h.P_v.size());
    v.R_v = A.take<T>(h.R_v.size());
    v.P_ev = A.take<T>(h.P_ev.size());
    v.R_ev = A.take<T>(h.R_ev.size());
}

void plan(dfmg_ctx *c, Arena &A) {
    const Hierarchy &H = c->S();
    const int L = H.pb.L, np = c->np;
    c->dl.assign(L, DevLevel());
    int maxblocks = 1;
    int64_t nmax = 0;
    for (int l = 0; l < L; ++l) {
        const HostLevel &h = H.lv[l];
        DevLevel &v = c->dl[l];
        v.n = h.n;
        v.sval = (int64_t)h.val.size();
        v.nent = (int64_t)h.pdofs.size();
        v.sdelta = v.nent + (int64_t)kSmallPatch * (int64_t)h.small_list.size();
        v.sM = 0;
        for (const Hierarchy &Q : c->P) v.sM = std::max(v.sM, (int64_t)Q.lv[l].M.size());
        take_level(A, v, np, v.d, l == 0, h);
        // levels whose inverses are mostly per subdomain (advection, mapped
        // domains): the small subdomains' inverses also interleaved, so that
        // a wavefront's loads of them coalesce
        if (l > 0) {
            int64_t ncls = 0;
            for (const Hierarchy &Q : c->P) ncls = std::max(ncls, Q.lv[l].n_class);
            v.soa = !h.small_list.empty() && 2 * ncls > h.n_patch;
        }
        const int64_t nsoa = (int64_t)kSmallPatch * kSmallPatch * (int64_t)h.small_list.size();
        if (v.soa) v.d.msoa = A.take<double>((size_t)nsoa * np);
        // the multiplicative sweep's rows in lane order (every smoothed level:
        // 42.9 -> 35.8 ms per solve of the 256^2 four-problem batch)
        if (c->mult() && l > 0) {
            v.mslots = 0;
            for (int R = 0; R < h.nblk; ++R) v.mslots = std::max(v.mslots, h.nslots[R]);
            v.smval = (int64_t)h.mlane.size() * v.mslots;
            v.d.mval = A.take<double>((size_t)v.smval * np);
        }
        if (c->mixed()) {
            take_level(A, v, np, v.f, l == 0, h);
            if (v.soa) v.f.msoa = A.take<float>((size_t)nsoa * np);
            v.npsi = h.n_psi;
            v.psi = A.take<double>((size_t)h.n_psi * np);
            if (l == 0) {
                v.Q0 = A.take<double>(h.Q0.size() * np);
            } else {
                v.nbeta = (int64_t)h.qpsi.size();
                v.sQ = 0;  // the shared maps differ between problems (coefficients)
                for (const Hierarchy &Q : c->P) v.sQ = std::max(v.sQ, (int64_t)Q.lv[l].Q.size());
                v.beta = A.take<float>((size_t)v.nbeta * np);
                v.Q = A.take<float>((size_t)v.sQ * np);
                if (v.soa) v.qsoa = A.take<float>((size_t)kSmallPatch * h.small_list.size() * np);
                v.Ps_v = A.take<double>(h.Ps_v.size());
                v.qoff = A.take<int32_t>(h.qoff.size() * np);
                v.qptr = A.take<int32_t>(h.qptr.size());
                v.beta_row = A.take<int32_t>(h.beta_row.size() * np);
                v.beta_patch = A.take<int32_t>(h.beta_patch.size());
                v.bigbeta = A.take<int32_t>(h.big_beta.size());
                v.qinv_ptr = A.take<int32_t>(h.qinv_ptr.size());
                v.qinv_pos = A.take<int32_t>(h.qinv_pos.size());
                v.Ps_rp = A.take<int32_t>(h.Ps_rp.size());
                v.Ps_ci = A.take<int32_t>(h.Ps_ci.size());
                v.qinv_ell = A.take<int32_t>(h.qinv_ell.size());
                v.Ps_eci = A.take<int32_t>(h.Ps_eci.size());
                v.Ps_ev = A.take<double>(h.Ps_ev.size());
            }
        }
        nmax = std::max(nmax, h.n);
        maxblocks = std::max(maxblocks, spmv_blocks(h.n, 4));
        if (l == 0) {
            v.Kinv = A.take<double>(h.Kinv.size() * np);
            continue;
        }
        v.pptr = A.take<int32_t>(h.pptr.size());
        v.pdofs = A.take<int32_t>(h.pdofs.size());
        v.inv_ptr = A.take<int32_t>(h.inv_ptr.size());
        v.inv_pos = A.take<int32_t>(h.inv_pos.size());
        v.col_list = A.take<int32_t>(h.col_list.size());
        v.small = A.take<int32_t>(h.small_list.size());
        v.bigent = A.take<int32_t>(h.big_ent.size());
        v.small_dofs = A.take<int32_t>(h.small_dofs.size());
        v.inv_pos4 = A.take<int32_t>(h.inv_pos4.size());
        v.inv_ell = A.take<int32_t>(h.inv_ell.size());
        v.inv4_ell = A.take<int32_t>(h.inv4_ell.size());
        v.bmesh = A.take<int4>(h.big_sub.size());
        v.sinfo = A.take<int4>(h.small_list.size() * np);
        v.binfo = A.take<int2>(h.big_sub.size() * np);
        v.P_eci = A.take<int32_t>(h.P_eci.size());
        v.R_eci = A.take<int32_t>(h.R_eci.size());
        v.P_rp = A.take<int32_t>(h.P_rp.size());
        v.P_ci = A.take<int32_t>(h.P_ci.size());
        v.R_rp = A.take<int32_t>(h.R_rp.size());
        v.R_ci = A.take<int32_t>(h.R_ci.size());
        v.moff = A.take<int32_t>(h.n_patch * np);
        v.ent_info = A.take<int4>(v.nent * np);
        if (c->mult()) {
            v.mlane = A.take<int32_t>(h.mlane.size());
            v.mstride = A.take<int32_t>(h.mstride.size());
        }
    }
    c->nparts = padded_grid(maxblocks);
    c->eta = A.take<double>((size_t)L * np);
    c->partial = A.take<double>((size_t)c->nparts * np);
    c->hist = A.take<double>((size_t)DFMG_MAX_HISTORY * np);
    c->counter = A.take<int>(kFlagSets * (size_t)np);
    c->stop = c->counter ? c->counter + np : nullptr;
    c->near = c->counter ? c->counter + 2 * np : nullptr;
    c->stopw = A.take<int>((size_t)kStopLanes * np);
    c->thresh2 = A.take<double>(np);
    c->scal = A.take<double>(np);
    c->dvec = A.take<double>(H.lv[L - 1].n_q);
    c->dcoef = A.take<double>(H.dcoef.size());
    c->pmass = A.take<double>(H.pmass.size());
    c->rtmp = A.take<double>((size_t)nmax * np);
    c->wfine = A.take<double>(H.lv[L - 1].n_q);
    c->small_d = A.take<SmallLevel<double>>(L);
    if (c->mixed()) c->small_f = A.take<SmallLevel<float>>(L);
    c->mlpW = A.take<float>(MLP_NPARAM);
    c->feat = A.take<float>((size_t)MLP_IN * np);
    c->rho_plain = A.take<double>(np);
    c->eta_fixed = A.take<double>((size_t)L * np);
    c->fallback = A.take<int>(np);
    c->sched = A.take<double>((size_t)L * np * kSchedPerLevel);
    c->sched0 = A.take<double>((size_t)L * np * kSchedPerLevel);
    c->unit = A.take<double>(np);
    c->mlpZ = A.take<float>((size_t)MLP_OUT * np);
    if (c->opt.time_stepping) {
        const int d = H.pb.d, nq = H.pb.k + 3;
        c->npts = 1;
        for (int j = 0; j < d; ++j) c->npts *= (int64_t)H.pb.N * nq;
        c->qbval = A.take<double>(H.qbval.size());
        c->qbder = A.take<double>(H.qbder.size());
        c->qw = A.take<double>(H.qw.size());
        c->qG = A.take<double>((size_t)c->npts * d * np);
        c->fstep = A.take<double>((size_t)H.lv[L - 1].n * np);
        c->sigma_dev = A.take<double>(np);
    }
}

template <class T>
void up(T *dst, const T *src, size_t count, hipStream_t s) {
    if (count) HIPCHK(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, s));
}
template <class T>
void up(T *dst, const std::vector<T> &src, hipStream_t s) {
    up(dst, src.data(), src.size(), s);
}

// FP32 copy of a host array (staging buffer is local: synchronous)
void up32(float *dst, const std::vector<double> &src, hipStream_t s) {
    if (src.empty()) return;
    std::vector<float> tmp(src.begin(), src.end());
    HIPCHK(hipMemcpyAsync(dst, tmp.data(), tmp.size() * sizeof(float), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
}

// operator values per residual launch (whole batch) above which they are
// streamed with non-temporal loads: twice the Infinity Cache
constexpr double kNtBytes = 512.0 * 1024 * 1024;

template <class T>
SpmvArgsT<T> spmv_args(dfmg_ctx *c, int l, const T *F, const T *U, T *r, double *partial, const int *stop) {
    const HostLevel &h = c->S().lv[l];
    const DevLevel &dv = c->dl[l];
    SpmvArgsT<T> a{};
    a.val = c->dl[l].data<T>().val;
    a.sval = dv.sval;
    for (int R = 0; R < 4; ++R) a.val_off[R] = R < h.nblk ? h.val_off[R] : 0;
    for (int R = 0; R < 5; ++R) a.off[R] = R <= h.nblk ? h.off[R] : h.n;
    for (int R = 0; R < 4; ++R)
        for (int j = 0; j < 3; ++j) a.nb[R][j] = R < h.nblk ? h.nb[R][j] : 1;
    a.n = (int)h.n;
    a.win = h.win ? 1 : 0;
    a.xc = c->S().pb.geometry != 0 ? 1 : 0;
    // values read once per launch and far beyond the 256 MB Infinity Cache:
    // non-temporal loads, so that they do not evict the vector's lines (below
    // that size the cache keeps part of them from one launch to the next, and
    // non-temporal loads measured slower)
    a.nt = (double)h.val.size() * sizeof(T) * c->np > kNtBytes ? 1 : 0;
    a.nblocks = spmv_blocks(h.n, c->lpr[l]);
    a.F = F;
    a.U = U;
    a.r = r;
    a.svec = h.n;
    a.partial = partial;
    a.spart = c->nparts;
    a.stop = stop;
    a.nprob = c->np;
    a.exit_early = c->exit_mode;
    return a;
}

// r = F - K_l U for every problem; returns the number of per-block partial
// sums written per problem
template <class T>
int spmv(dfmg_ctx *c, int l, const T *F, const T *U, T *r, double *partial, const int *stop) {
    const SpmvArgsT<T> a = spmv_args<T>(c, l, F, U, r, partial, stop);
    launch_spmv<T>(c->S().pb.d, c->S().pb.k, c->lpr[l], a, c->s);
    return a.nblocks;
}

// The FP32 cycle of the refinement (2D) tracks the potentials of its
// velocity corrections.
template <class T>
bool tracks_potentials(const dfmg_ctx *c) {
    return std::is_same<T, float>::value && c->mixed();
}

// Damping of smoothing step `step` of level l: before the coarse correction
// (phase 0) or after it (phase 1); device pointer and per-problem stride.
struct Damping {
    const double *eta;
    int64_t stride;
};
Damping step_damping(const dfmg_ctx *c, int l, int phase, int step) {
    if (c->sched_on)
        return {c->sched + (size_t)l * kSchedPerLevel + phase * kMaxSteps + std::min(step, kMaxSteps - 1),
                (int64_t)c->L() * kSchedPerLevel};
    return {c->eta + l, c->L()};
}

// eta * sum_i E_i^T M_i E_i r added to (or assigned into) U on level l, with
// the level's damping eta (dm: another damping, e.g. one step's of a schedule).
template <class T>
void schwarz(dfmg_ctx *c, int l, const T *r, T *U, bool assign, const int *stop, Damping dm = {nullptr, 0}) {
    const HostLevel &h = c->S().lv[l];
    DevLevel &v = c->dl[l];
    PatchArgsT<T> a{};
    a.n = (int)h.n;
    a.nent = (int)v.nent;
    a.inv_ptr = v.inv_ptr;
    a.inv_pos = v.inv_pos;
    a.pptr = v.pptr;
    a.pdofs = v.pdofs;
    a.moff = v.moff;
    a.ent_info = v.ent_info;
    a.delta = v.data<T>().delta;
    a.M = v.data<T>().M;
    a.msoa = v.soa ? v.data<T>().msoa : nullptr;
    a.r = r;
    a.U = U;
    a.eta = dm.eta ? dm.eta : c->eta + l;
    a.smoff = h.n_patch;
    a.sM = v.sM;
    a.svec = h.n;
    a.seta = dm.eta ? dm.stride : c->L();
    a.assign = assign ? 1 : 0;
    a.stop = stop;
    a.nprob = c->np;
    a.exit_early = c->exit_mode;
    a.small = v.small;
    a.bigent = v.bigent;
    a.small_dofs = v.small_dofs;
    a.nsmall = (int)h.small_list.size();
    a.nbig = (int)h.big_ent.size();
    a.sdelta = v.sdelta;
    a.sinfo = v.sinfo;
    a.bmesh = v.bmesh;
    a.binfo = v.binfo;
    a.nbsub = (int)h.big_sub.size();
    a.max_big = h.max_big;
    a.inv_w = h.inv_w;
    a.inv_ell = v.inv_ell;
    a.tile = c->tile[l];
    if (tracks_potentials<T>(c)) {
        // the FP32 cycle of the refinement also accumulates the potentials of
        // its velocity corrections (forms 3 and 4 do; the others run as 4)
        a.psi = v.psi;
        a.beta = reinterpret_cast<T *>(v.beta);
        a.Q = reinterpret_cast<const T *>(v.Q);
        a.qsoa = v.soa ? reinterpret_cast<const T *>(v.qsoa) : nullptr;
        a.sQ = v.sQ;
        a.nbeta = v.nbeta;
        a.npsi = (int)v.npsi;
        a.nbigbeta = (int)h.big_beta.size();
        a.qoff = v.qoff;
        a.qptr = v.qptr;
        a.beta_row = v.beta_row;
        a.beta_patch = v.beta_patch;
        a.bigbeta = v.bigbeta;
        a.qinv_ptr = v.qinv_ptr;
        a.qinv_pos = v.qinv_pos;
        a.qinv_w = h.qinv_w;
        a.qinv_ell = v.qinv_ell;
        if (c->smoother[l] == 3) {  // one pass (recomputes the rows, no buffer)
            launch_schwarz_fused<T>(a, c->s);
        } else {
            a.inv_pos = v.inv_pos4;
            a.inv_ell = v.inv4_ell;
            launch_schwarz_small<T>(a, c->s);
        }
        return;
    }
    if (c->smoother[l] == 2) {
        if (assign) launch_fill<T>(h.n, U, h.n, T(0), stop, c->np, c->s);
        for (size_t col = 0; col + 1 < h.col_ptr.size(); ++col)
            launch_schwarz_colour<T>(a, v.col_list + h.col_ptr[col], h.col_ptr[col + 1] - h.col_ptr[col], c->s);
    } else if (c->smoother[l] == 3) {
        launch_schwarz_fused<T>(a, c->s);
    } else if (c->smoother[l] == 4) {
        a.inv_pos = v.inv_pos4;
        a.inv_ell = v.inv4_ell;
        launch_schwarz_small<T>(a, c->s);
    } else {
        launch_schwarz_gather<T>(a, c->s);
    }
}

template <class T>
void restrict_to(dfmg_ctx *c, int l, const T *r, T *G, const int *stop) {
    const HostLevel &hc = c->S().lv[l - 1], &hf = c->S().lv[l];
    DevLevel &v = c->dl[l];
    const SparseT<T> R{v.R_rp, v.R_ci, v.data<T>().R_v, hf.R_w, v.R_eci, v.data<T>().R_ev};
    launch_csr<T>((int)hc.n, R, r, hf.n, G, hc.n, 0, stop, c->np, c->s, c->exit_mode);
}

template <class T>
void prolong_add(dfmg_ctx *c, int l, const T *dU, T *U, const int *stop) {
    const HostLevel &hc = c->S().lv[l - 1], &hf = c->S().lv[l];
    DevLevel &v = c->dl[l];
    const SparseT<T> P{v.P_rp, v.P_ci, v.data<T>().P_v, hf.P_w, v.P_eci, v.data<T>().P_ev};
    launch_csr<T>((int)hf.n, P, dU, hc.n, U, hf.n, 1, stop, c->np, c->s, c->exit_mode);
}

// the FP32 cycle's prolongation with its potentials, one launch
void prolong_pair(dfmg_ctx *c, int l, const int *stop) {
    const HostLevel &hc = c->S().lv[l - 1], &hf = c->S().lv[l];
    DevLevel &f = c->dl[l];
    const DevLevel &q = c->dl[l - 1];
    const SparseT<float> P{f.P_rp, f.P_ci, f.f.P_v, hf.P_w, f.P_eci, f.f.P_ev};
    const SparseT<double> Ps{f.Ps_rp, f.Ps_ci, f.Ps_v, hf.Ps_w, f.Ps_eci, f.Ps_ev};
    launch_prolong_pair<float>((int)hf.n, P, q.f.U, hc.n, f.f.U, hf.n, (int)f.npsi, Ps, q.psi, q.npsi, f.psi, f.npsi,
                               stop, c->np, c->s, c->exit_mode);
}

// the FP32 cycle's exact coarse solve with the potentials of its solution
void coarse_pair(dfmg_ctx *c, const int *stop) {
    const DevLevel &z = c->dl[0];
    const int64_t n = z.n;
    launch_coarse_pair((int)n, (int)z.npsi, z.Kinv, n * n, z.Q0, z.npsi * n, z.f.F, n, z.f.U, n, z.psi, z.npsi, stop,
                       c->np, c->s, c->exit_mode);
}

// exact coarse solve (FP64 bordered inverse, FP64 accumulation)
template <class T>
void coarse(dfmg_ctx *c, const T *G, T *dU, const int *stop) {
    const int64_t n = c->S().lv[0].n;
    launch_gemv<T>((int)n, (int)n, c->dl[0].Kinv, n * n, G, n, dU, n, stop, c->np, c->s, c->exit_mode);
}

// One multiplicative Schwarz step on level l (equation MSM): the
// coupling-free colours in order, one launch each, every subdomain of a
// colour computing its residual rows from the current U and correcting U in
// place (no damping).
template <class T>
void mult_sweep(dfmg_ctx *c, int l, const T *F, T *U, const int *stop) {
    const HostLevel &h = c->S().lv[l];
    DevLevel &v = c->dl[l];
    MultArgsT<T> a{};
    a.sp = spmv_args<T>(c, l, F, U, nullptr, nullptr, stop);
    a.U = U;
    a.pdofs = v.pdofs;
    a.ent_info = v.ent_info;
    a.nent = v.nent;
    a.M = v.data<T>().M;
    a.sM = v.sM;
    a.width = h.mwidth;
    a.mval = v.data<T>().mval;
    a.smval = v.smval;
    a.mslots = v.mslots;
    for (size_t col = 0; col + 1 < h.mwave_ptr.size(); ++col) {
        a.lane0 = (int64_t)h.mwave_ptr[col] * h.mwidth;
        a.lanes = v.mlane + (int64_t)h.mwave_ptr[col] * h.mwidth;
        a.strides = v.mstride + h.mwave_ptr[col];
        a.nwaves = h.mwave_ptr[col + 1] - h.mwave_ptr[col];
        launch_schwarz_mult<T>(c->S().pb.d, c->S().pb.k, a, c->s);
    }
}

// every problem running: the flags and their wide copies
void reset_flags(dfmg_ctx *c) {
    launch_fill_int(c->np, c->stop, 0, c->s);
    launch_fill_int(c->np, c->near, 0, c->s);
    launch_fill_int(c->np * kStopLanes, c->stopw, 0, c->s);
}

void check(dfmg_ctx *c, int np_blocks) {
    Fallback fb{};
    // the thresholds are read on the device (a captured graph keeps working
    // when they change); 0 disables the fallback of a problem
    fb.rho = c->rho_plain;
    fb.eta = c->eta;
    fb.eta_fixed = c->eta_fixed;
    fb.sched = c->sched_on ? c->sched : nullptr;
    fb.flag = c->fallback;
    fb.L = c->L();
    launch_check(np_blocks, c->partial, c->nparts, c->hist, DFMG_MAX_HISTORY, c->counter, c->stop, c->stopw,
                 c->near, c->thresh2, fb, c->np, c->s);
}

// dampings of every problem from the network (device), see dfmg_set_learned
void apply_learned(dfmg_ctx *c) {
    launch_mlp_damping(c->np, c->mlpW, c->feat, c->L(), c->eta, c->s);
}

template <class T>
SmallLevel<T> *small_table(dfmg_ctx *c);
template <>
SmallLevel<double> *small_table<double>(dfmg_ctx *c) { return c->small_d; }
template <>
SmallLevel<float> *small_table<float>(dfmg_ctx *c) { return c->small_f; }

// Host copy of the level tables of the single-workgroup coarse cycle (device
// pointers of the bound workspace).
template <class T>
std::vector<SmallLevel<T>> small_levels(dfmg_ctx *c) {
    const int L = c->L();
    std::vector<SmallLevel<T>> out(L);
    for (int l = 0; l < L; ++l) {
        const HostLevel &h = c->S().lv[l];
        DevLevel &v = c->dl[l];
        LevelData<T> &d = v.data<T>();
        SmallLevel<T> &q = out[l];
        q.sp = spmv_args<T>(c, l, nullptr, nullptr, nullptr, nullptr, nullptr);
        q.F = d.F;
        q.U = d.U;
        q.r = d.r;
        q.n = h.n;
        q.nu1 = c->nu1l[l];
        q.nu2 = c->nu2l[l];
        if (l == 0) {
            q.Kinv = v.Kinv;
            continue;
        }
        q.delta = d.delta;
        q.sdelta = v.sdelta;
        q.M = d.M;
        q.sM = v.sM;
        q.nent = v.nent;
        q.smoff = h.n_patch;
        q.pptr = v.pptr;
        q.pdofs = v.pdofs;
        q.moff = v.moff;
        q.inv_ptr = v.inv_ptr;
        q.inv_pos = v.inv_pos;
        q.small = v.small;
        q.bigent = v.bigent;
        q.ent_info = v.ent_info;
        q.nsmall = (int)h.small_list.size();
        q.nbig = (int)h.big_ent.size();
        q.eta = c->eta + l;
        q.seta = L;
        q.R_rp = v.R_rp;
        q.R_ci = v.R_ci;
        q.R_v = d.R_v;
        q.P_rp = v.P_rp;
        q.P_ci = v.P_ci;
        q.P_v = d.P_v;
    }
    return out;
}

// (re)load the level tables of the single-workgroup coarse cycle
void upload_small_tables(dfmg_ctx *c) {
    auto td = small_levels<double>(c);
    up(c->small_d, td, c->s);
    HIPCHK(hipStreamSynchronize(c->s));
    if (c->mixed()) {
        auto tf = small_levels<float>(c);
        up(c->small_f, tf, c->s);
        HIPCHK(hipStreamSynchronize(c->s));
    }
}

// One V-cycle (Algorithm 1) on the finest level's internal U, F of type T.
// norm: the first residual of the finest level also feeds the convergence
// check.  fine_zero: the finest U is known to be zero (its first smoothing
// step then needs no residual).
template <class T>
void cycle_body(dfmg_ctx *c, bool norm, bool fine_zero) {
    const int L = c->L();
    const int *stop = c->stopw;
    if (L == 1) {
        LevelData<T> &v = c->dl[0].data<T>();
        if (norm) check(c, spmv<T>(c, 0, v.F, v.U, v.r, c->partial, stop));
        coarse<T>(c, v.F, v.U, stop);  // exact solve of K U = F
        return;
    }
    const bool psi = tracks_potentials<T>(c);
    // levels <= top: single-workgroup cycle (level dampings only)
    const int top = (psi || c->sched_on || c->mult()) ? 0 : c->small_top;
    for (int l = L - 1; l > top; --l) {
        LevelData<T> &v = c->dl[l].data<T>();
        const HostLevel &h = c->S().lv[l];
        bool zero = (l < L - 1) || fine_zero;
        bool first_res = (l == L - 1) && norm;
        if (c->mult() && c->nu1l[l] > 0) {
            // multiplicative pre-smoothing: each sweep computes its own
            // residual rows; the check's residual comes first where asked
            if (first_res) {
                check(c, spmv<T>(c, l, v.F, v.U, v.r, c->partial, stop));
                first_res = false;
            }
            if (zero) launch_fill<T>(h.n, v.U, h.n, T(0), stop, c->np, c->s);
            zero = false;
            for (int s = 0; s < c->nu1l[l]; ++s) mult_sweep<T>(c, l, v.F, v.U, stop);
        }
        for (int s = 0; s < (c->mult() ? 0 : c->nu1l[l]); ++s) {
            if (zero && !first_res) {
                schwarz<T>(c, l, v.F, v.U, true, stop, step_damping(c, l, 0, s));  // U = 0: residual is F
                zero = false;
                continue;
            }
            const int npb = spmv<T>(c, l, v.F, v.U, v.r, first_res ? c->partial : nullptr, stop);
            if (first_res) {
                check(c, npb);
                first_res = false;
            }
            schwarz<T>(c, l, v.r, v.U, zero, stop, step_damping(c, l, 0, s));
            zero = false;
        }
        if (zero && !first_res) {
            launch_fill<T>(h.n, v.U, h.n, T(0), stop, c->np, c->s);
            if (psi) launch_fill<double>(c->dl[l].npsi, c->dl[l].psi, c->dl[l].npsi, 0.0, stop, c->np, c->s);
            restrict_to<T>(c, l, v.F, c->dl[l - 1].data<T>().F, stop);
        } else {
            const int npb = spmv<T>(c, l, v.F, v.U, v.r, first_res ? c->partial : nullptr, stop);
            if (first_res) check(c, npb);
            restrict_to<T>(c, l, v.r, c->dl[l - 1].data<T>().F, stop);
        }
    }
    if (top >= 1)
        launch_vcycle_small<T>(c->S().pb.d, c->S().pb.k, small_table<T>(c), top, stop, c->np, c->s);
    else if (psi)  // with the potentials of the coarse velocity solution
        coarse_pair(c, stop);
    else
        coarse<T>(c, c->dl[0].data<T>().F, c->dl[0].data<T>().U, stop);
    if (psi && top >= 1) {  // potentials of the coarse velocity solution
        const DevLevel &z = c->dl[0];
        launch_gemv_f2d((int)z.npsi, (int)z.n, z.Q0, z.npsi * z.n, z.f.F, z.n, z.psi, z.npsi, stop, c->np, c->s,
                        c->exit_mode);
    }
    for (int l = top + 1; l < L; ++l) {
        LevelData<T> &v = c->dl[l].data<T>();
        if (psi) prolong_pair(c, l, stop);
        else prolong_add<T>(c, l, c->dl[l - 1].data<T>().U, v.U, stop);
        if (c->mult()) {
            for (int s = 0; s < c->nu2l[l]; ++s) mult_sweep<T>(c, l, v.F, v.U, stop);
            continue;
        }
        for (int s = 0; s < c->nu2l[l]; ++s) {
            spmv<T>(c, l, v.F, v.U, v.r, nullptr, stop);
            schwarz<T>(c, l, v.r, v.U, false, stop, step_damping(c, l, 1, s));
        }
    }
}

// r = F - K U in FP64 with the convergence check, and its FP32 copy as the
// load of the next FP32 cycles (the check that ends a refinement step and the
// one before the first).
void refine_residual(dfmg_ctx *c) {
    const int L = c->L();
    const HostLevel &h = c->S().lv[L - 1];
    DevLevel &v = c->dl[L - 1];
    check(c, spmv<double>(c, L - 1, v.d.F, v.d.U, v.d.r, c->partial, c->stopw));
    launch_cast(h.n, v.d.r, v.f.F, h.n, c->stopw, c->np, c->s, c->exit_mode);
}

// One step of the FP64 iterative refinement (its residual is in place):
// inner_cycles FP32 V-cycles on K dU = r from dU = 0, U += [curl psi; dU_p]
// in FP64 with psi the streamfunction the cycles tracked for dU's velocity,
// then the residual and check of the new iterate.  The check ends the step,
// so the step in which a problem converges does no work after it.
void refine_body(dfmg_ctx *c) {
    const int L = c->L();
    const HostLevel &h = c->S().lv[L - 1];
    DevLevel &v = c->dl[L - 1];
    for (int i = 0; i < c->opt.inner_cycles; ++i) cycle_body<float>(c, false, i == 0);
    RefineArgs a{};
    a.d = c->S().pb.d;
    a.N = c->S().pb.N;
    a.k = c->S().pb.k;
    a.off_uy = h.off[1];
    a.off_uz = h.off[a.d - 1];
    a.off_p = h.off[a.d];
    a.n = h.n;
    a.X = v.f.U;
    a.dcoef = c->dcoef;
    a.psi = v.psi;
    a.U = v.d.U;
    a.svec = h.n;
    a.spsi = v.npsi;
    a.stop = c->stopw;
    a.nprob = c->np;
    a.exit_early = c->exit_mode;
    launch_refine_update(a, c->s);
    refine_residual(c);
}

void body(dfmg_ctx *c, int kind) {
    if (kind == 2) refine_body(c);
    else cycle_body<double>(c, kind == 1, false);
}

// Launch one cycle of the given kind, replaying a captured hipGraph when
// enabled (captured on first use, recaptured when the kind changes).
void run_cycle(dfmg_ctx *c, int kind) {
    if (!c->opt.use_graph) {
        body(c, kind);
        return;
    }
    const int x = c->exit_mode;
    if (c->graph[x] && c->graph_kind[x] != kind) {
        HIPCHK(hipGraphExecDestroy(c->graph[x]));
        c->graph[x] = nullptr;
    }
    if (!c->graph[x]) {
        hipGraph_t g;
        HIPCHK(hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal));
        body(c, kind);
        HIPCHK(hipStreamEndCapture(c->s, &g));
        HIPCHK(hipGraphInstantiate(&c->graph[x], g, nullptr, nullptr, 0));
        HIPCHK(hipGraphDestroy(g));
        c->graph_kind[x] = kind;
    }
    HIPCHK(hipGraphLaunch(c->graph[x], c->s));
}

void drop_graph(dfmg_ctx *c) {
    for (auto &g : c->graph)
        if (g) {
            HIPCHK(hipGraphExecDestroy(g));
            g = nullptr;
        }
}

// Order the internal stream after the caller's stream, and back.
void enter(dfmg_ctx *c) {
    if (!c->bound) throw StateError("workspace not bound (call dfmg_bind first)");
    HIPCHK(hipEventRecord(c->ev_in, c->user));
    HIPCHK(hipStreamWaitEvent(c->s, c->ev_in, 0));
}
void leave(dfmg_ctx *c) {
    HIPCHK(hipEventRecord(c->ev_out, c->s));
    HIPCHK(hipStreamWaitEvent(c->user, c->ev_out, 0));
}

void check_level(const dfmg_ctx *c, int level, int minlevel = 0) {
    if (level < minlevel || level >= c->L()) throw ArgError("level out of range");
}

// Largest |eigenvalue| of the undamped additive-Schwarz operator S^-1 K of
// every smoothed level and problem, by power iteration: x <- y / ||y||,
// y = S^-1 (0 - K x) (the level's residual and smoother kernels in FP64 with
// damping 1; the norms on the host).  The start vector is the same
// deterministic pseudo-random vector for every problem.
void estimate_lmax(dfmg_ctx *c, int iters) {
    const int L = c->L(), np = c->np;
    c->lmax.assign((size_t)np * L, 0.0);
    for (int l = 1; l < L; ++l) {
        const int64_t n = c->S().lv[l].n;
        LevelData<double> &v = c->dl[l].d;
        std::vector<double> x((size_t)n * np);
        uint64_t z = 0x9e3779b97f4a7c15ull;
        for (int64_t i = 0; i < n; ++i) {  // splitmix64 values in [-1, 1)
            z += 0x9e3779b97f4a7c15ull;
            uint64_t w = z;
            w = (w ^ (w >> 30)) * 0xbf58476d1ce4e5b9ull;
            w = (w ^ (w >> 27)) * 0x94d049bb133111ebull;
            w ^= w >> 31;
            const double u = (double)(w >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
            for (int p = 0; p < np; ++p) x[(size_t)p * n + i] = u;
        }
        for (int p = 0; p < np; ++p) {
            double s2 = 0.0;
            for (int64_t i = 0; i < n; ++i) s2 += x[(size_t)p * n + i] * x[(size_t)p * n + i];
            const double inv = 1.0 / std::sqrt(s2);
            for (int64_t i = 0; i < n; ++i) x[(size_t)p * n + i] *= inv;
        }
        launch_fill<double>(n, v.F, n, 0.0, nullptr, np, c->s);
        for (int it = 0; it < iters; ++it) {
            up(v.U, x, c->s);
            spmv<double>(c, l, v.F, v.U, v.r, nullptr, nullptr);
            schwarz<double>(c, l, v.r, v.U, true, nullptr, Damping{c->unit, 1});
            HIPCHK(hipMemcpyAsync(x.data(), v.U, x.size() * sizeof(double), hipMemcpyDeviceToHost, c->s));
            HIPCHK(hipStreamSynchronize(c->s));
            for (int p = 0; p < np; ++p) {
                double s2 = 0.0;
                for (int64_t i = 0; i < n; ++i) s2 += x[(size_t)p * n + i] * x[(size_t)p * n + i];
                const double nrm = std::sqrt(s2);
                if (!(nrm > 0.0 && nrm < 1e300)) throw HipError("eigenvalue estimate: zero or non-finite iterate");
                c->lmax[(size_t)p * L + l] = nrm;  // ||S^-1 K x|| with ||x|| = 1
                for (int64_t i = 0; i < n; ++i) x[(size_t)p * n + i] /= nrm;
            }
        }
        launch_fill<double>(n, v.U, n, 0.0, nullptr, np, c->s);
    }
    HIPCHK(hipStreamSynchronize(c->s));
}

// Chebyshev dampings of one smoothing phase: the nu steps of damped
// additive Schwarz with dampings 1 / theta_j, theta_j the zeros of the
// degree-nu Chebyshev polynomial mapped to [b / alpha, b], leave the error
// polynomial T_nu((b + a - 2 x) / (b - a)) / T_nu((b + a) / (b - a)),
// a = b / alpha, in the preconditioned operator: the smallest maximum on
// [a, b] of any polynomial of degree nu with value 1 at 0.  Pre-smoothing
// takes the zeros from the largest theta down, post-smoothing the reverse.
double chebyshev_damping(double b, double alpha, int nu, int j, bool reverse) {
    const double a = b / alpha;
    const int jj = reverse ? nu - 1 - j : j;
    const double pi = 3.14159265358979323846;
    const double theta = 0.5 * (b + a) + 0.5 * (b - a) * std::cos(pi * (2.0 * jj + 1.0) / (2.0 * nu));
    return 1.0 / theta;
}

// the upper end of the Chebyshev interval, relative to the estimate of the
// largest eigenvalue (power iteration approaches it from below)
constexpr double kLmaxSafety = 1.05;
// default interval ratios b / a of the schedule: 2D k = 2 Stokes gives the
// same cycle counts for ratios 8 .. 15 (32^2, 64^2 sweeps); 3D k = 1 Stokes
// on 32^3 is fastest near 60
constexpr double kChebAlpha2d = 10.0, kChebAlpha3d = 60.0;

// Per-step dampings of every problem and level from lmax, alpha and the
// current step counts; uploaded (stream-ordered) to sched.  Entries past
// a phase's step count repeat its last damping (unused).
void build_schedule(dfmg_ctx *c) {
    const int L = c->L(), np = c->np;
    c->sched_host.assign((size_t)np * L * kSchedPerLevel, 0.0);
    for (int p = 0; p < np; ++p)
        for (int l = 1; l < L; ++l) {
            const double b = kLmaxSafety * c->lmax[(size_t)p * L + l], al = c->alpha[(size_t)p * L + l];
            double *dst = &c->sched_host[((size_t)p * L + l) * kSchedPerLevel];
            for (int ph = 0; ph < 2; ++ph) {
                const int nu = ph ? c->nu2l[l] : c->nu1l[l];
                for (int j = 0; j < kMaxSteps; ++j)
                    dst[ph * kMaxSteps + j] =
                        nu > 0 ? chebyshev_damping(b, al, nu, std::min(j, nu - 1), ph == 1) : 0.0;
            }
        }
    up(c->sched0, c->sched_host, c->s);
    HIPCHK(hipMemcpyAsync(c->sched, c->sched0, c->sched_host.size() * sizeof(double), hipMemcpyDeviceToDevice,
                          c->s));
    HIPCHK(hipStreamSynchronize(c->s));
}

// the dampings of the schedule as built (a fallback of an earlier solve
// replaced a problem's)
void restore_schedule(dfmg_ctx *c) {
    if (c->sched_on)
        HIPCHK(hipMemcpyAsync(c->sched, c->sched0, (size_t)c->np * c->L() * kSchedPerLevel * sizeof(double),
                              hipMemcpyDeviceToDevice, c->s));
}

// no fallback thresholds: the fixed dampings are in use
void clear_fallback(dfmg_ctx *c) { HIPCHK(hipMemsetAsync(c->rho_plain, 0, c->np * sizeof(double), c->s)); }

void upload_eta(dfmg_ctx *c) {
    HIPCHK(hipMemcpyAsync(c->eta, c->eta_host.data(), c->eta_host.size() * sizeof(double), hipMemcpyHostToDevice,
                          c->s));
    HIPCHK(hipStreamSynchronize(c->s));
}

Problem make_problem(const dfmg_grid *grid, int k, double nu, double sigma, const dfmg_advection *adv,
                     const dfmg_options &o) {
    Problem pb;
    pb.d = grid->dim;
    pb.N = grid->n_elem;
    pb.L = grid->n_levels;
    pb.k = k;
    pb.nu = nu;
    pb.sigma = sigma;
    if (adv) {
        pb.adv_kind = adv->kind;
        pb.adv_c = adv->c;
        if (adv->kind == 3) {
            if (!adv->coeffs) throw ArgError("advection kind 3 needs its field's coefficients");
            const int64_t nv = (int64_t)pb.d * (pb.N + k - 1) * (int64_t)std::pow(pb.N + k, pb.d - 1);
            pb.adv_field.assign(adv->coeffs, adv->coeffs + nv);
        }
    }
    pb.geometry = grid->geometry;
    if (pb.geometry == 1) {
        pb.r_in = grid->r_inner;
        pb.r_out = grid->r_outer;
        pb.depth = grid->depth;
        if (o.time_stepping) throw ArgError("time stepping runs on the unit square / cube");
    } else if (pb.geometry != 0) {
        throw ArgError("geometry must be 0 or 1");
    }
    pb.share_inverses = o.share_inverses != 0;
    pb.potentials = o.precision == 1;
    pb.multiplicative = o.multiplicative == 1;
    return pb;
}

dfmg_options checked_options(const dfmg_options *opt, int dim) {
    dfmg_options o;
    dfmg_default_options(&o);
    if (opt) o = *opt;
    if (o.nu1 < 0 || o.nu2 < 0 || o.max_cycles < 1 || o.cycles_per_check < 1) throw ArgError("invalid options");
    if (o.max_cycles > DFMG_MAX_HISTORY - 2) throw ArgError("max_cycles too large");
    if (o.precision != 0 && o.precision != 1) throw ArgError("precision must be 0 or 1");
    if (o.inner_cycles < 1) throw ArgError("inner_cycles must be >= 1");
    if (o.smoother < 0 || o.smoother > 4) throw ArgError("smoother must be 0 .. 4");
    if (o.eta >= 1.0) throw ArgError("eta must be < 1");
    if (o.multiplicative != 0 && o.multiplicative != 1) throw ArgError("multiplicative must be 0 or 1");
    if (o.time_stepping != 0 && o.time_stepping != 1) throw ArgError("time_stepping must be 0 or 1");
    if (o.multiplicative == 1 && o.precision != 0)
        throw ArgError("multiplicative Schwarz runs in FP64 V-cycles (precision 0)");
    return o;
}

// the autotuner considers the single-workgroup coarse cycle for levels of at
// most this many DOFs per problem (off by default: one compute unit's
// bandwidth makes it slower than the per-level kernels on the benchmark grids)
constexpr int64_t kSmallCycleMax = 16384;

void init_ctx(dfmg_ctx *c, const dfmg_options &o) {
    c->opt = o;
    const int L = c->L();
    const double eta0 = o.eta > 0 ? o.eta : c->S().default_eta;
    c->eta_host.assign((size_t)L * c->np, eta0);
    for (int p = 0; p < c->np; ++p) c->eta_host[(size_t)p * L] = 0.0;  // level 0: exact solve
    c->smoother.assign(L, o.smoother == 0 ? 1 : o.smoother);
    c->lpr.assign(L, 1);
    for (int l = 0; l < L; ++l) {
        const int64_t n = c->S().lv[l].n * c->np;
        c->lpr[l] = c->S().pb.geometry != 0 ? 1 : (n < 20000 ? 4 : (n < 100000 ? 2 : 1));
    }
    c->small_top = 0;
    c->tile.assign(L, TileShape{});
    c->nu1l.assign(L, o.nu1);
    c->nu2l.assign(L, o.nu2);
}


// ---- pieces of a solve, shared by dfmg_solve and the mixed-mesh batch ----

int solve_kind(const dfmg_ctx *c) { return c->mixed() ? 2 : 1; }

// Reset the per-problem flags and counters, re-apply learned dampings (a
// fallback of an earlier solve replaced them), copy F and U in and set the
// thresholds tol^2 ||F||^2.  xoff: device table of the problems' offsets in
// F and U (null: problem p at p * n).
void solve_begin(dfmg_ctx *c, const double *F, const double *U, const int64_t *xoff, double tol) {
    const int L = c->L(), np = c->np;
    const int64_t n = c->S().lv[L - 1].n;
    LevelData<double> &v = c->dl[L - 1].d;
    const int nb = blocks_for(n);
    reset_flags(c);
    c->exit_mode = 0;
    launch_fill_int(np, c->counter, 0, c->s);
    launch_fill_int(np, c->fallback, 0, c->s);
    if (c->learned) apply_learned(c);
    restore_schedule(c);
    launch_copy_off(n, F, xoff, n, v.F, nullptr, n, np, c->s);
    launch_copy_off(n, U, xoff, n, v.U, nullptr, n, np, c->s);
    launch_dot_partial((int)n, v.F, v.F, n, c->partial, c->nparts, nb, np, c->s);
    launch_reduce(nb, c->partial, c->nparts, c->thresh2, tol * tol, np, c->s);
    if (solve_kind(c) == 2) refine_residual(c);  // the refinement steps end with their check
}

// state of host stop flags st[0..np) with the near flags at st + np
int flag_state(const int *st, int np) {
    bool all = true, near = true, any = false;
    for (int p = 0; p < np; ++p) {
        all = all && st[p];
        near = near && (st[p] || st[np + p]);
        any = any || st[p];
    }
    return (all ? kAllStopped : 0) | (near ? kAllNear : 0) | (any ? kAnyStopped : 0);
}

// queue a copy of the counters and stop flags into pinned buffer buf
void flags_async(dfmg_ctx *c, int buf) {
    HIPCHK(hipMemcpyAsync(c->hflags + buf * kFlagSets * c->np, c->counter, kFlagSets * c->np * sizeof(int),
                          hipMemcpyDeviceToHost,
                          c->s));
    HIPCHK(hipEventRecord(c->ev_flag[buf], c->s));
}

// wait for buffer buf: kAllStopped when every problem has stopped, kAllNear
// when each has stopped or is expected to stop at the next check,
// kAnyStopped when one has (later launches then use the exit mode)
int flags_wait(dfmg_ctx *c, int buf) {
    HIPCHK(hipEventSynchronize(c->ev_flag[buf]));
    const int st = flag_state(c->hflags + buf * kFlagSets * c->np + c->np, c->np);
    if (st & kAnyStopped) c->exit_mode = 1;
    return st;
}

// Run V-cycles in units of `chunk` until every problem has stopped or max
// cycles were launched, keeping one unit in flight while the host reads the
// flags of the previous one (a unit launched after the last problem stopped
// does no work for it), except when the flags read say that every problem is
// expected to stop within the unit in flight: then the next unit waits for
// its flags (one host round trip instead of a unit of wasted launches).
// launch_unit(k, buf) launches k cycles and queues the flags into buf;
// wait(buf) returns the flag state.  Returns the buffer holding the last
// flags read and whether all stopped.
template <class Launch, class Wait>
std::pair<int, bool> pipelined_cycles(int maxc, int chunk, Launch &&launch_unit, Wait &&wait) {
    int launched = 0, inflight = 0, next = 0, head = 0, last = 0;
    bool all = false, near = false;
    auto issue = [&] {
        const int k = std::min(chunk, maxc - launched);
        launch_unit(k, next);
        launched += k;
        next ^= 1;
        ++inflight;
    };
    issue();
    while (inflight > 0) {
        if (launched < maxc && inflight < 2 && !near) issue();
        const int st = wait(head);
        last = head;
        head ^= 1;
        --inflight;
        if (st & kAllStopped) {
            all = true;
            break;
        }
        near = (st & kAllNear) != 0;
        if (inflight == 0 && launched < maxc) issue();
    }
    return {last, all};
}

// cycle limit reached with V-cycles that check at their start: measure the
// residual of the last iterates (problems already stopped keep their flags
// and histories)
void solve_limit(dfmg_ctx *c) {
    const int L = c->L();
    LevelData<double> &v = c->dl[L - 1].d;
    check(c, spmv<double>(c, L - 1, v.F, v.U, v.r, c->partial, nullptr));
}

struct SolveOut {
    std::vector<double> hist, th;
    std::vector<int> fbk;
};

// Zero-mean pressure p <- p - (w^T p) 1 (partition of unity, |Omega| = 1),
// copy U out, and queue the copies of histories, thresholds and fallback
// flags into `so` (valid after the stream has been synchronized).
void solve_end_launch(dfmg_ctx *c, double *U, const int64_t *xoff, SolveOut &so) {
    const int L = c->L(), np = c->np;
    const HostLevel &h = c->S().lv[L - 1];
    const int64_t n = h.n;
    LevelData<double> &v = c->dl[L - 1].d;
    const int nbq = blocks_for(h.n_q);
    for (int p = 0; p < np; ++p)
        launch_dot_partial((int)h.n_q, v.U + p * n + h.n_v, c->wfine, 0, c->partial + p * c->nparts, 0, nbq, 1, c->s);
    launch_reduce(nbq, c->partial, c->nparts, c->scal, 1.0, np, c->s);
    launch_sub_scalar((int)h.n_q, v.U + h.n_v, n, c->scal, np, c->s);
    launch_copy_off(n, v.U, nullptr, n, U, xoff, n, np, c->s);
    so.hist.resize((size_t)np * DFMG_MAX_HISTORY);
    so.th.resize(np);
    so.fbk.resize(np);
    HIPCHK(hipMemcpyAsync(so.fbk.data(), c->fallback, np * sizeof(int), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipMemcpyAsync(so.hist.data(), c->hist, so.hist.size() * sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipMemcpyAsync(so.th.data(), c->thresh2, np * sizeof(double), hipMemcpyDeviceToHost, c->s));
}

// Fill one dfmg_stats per problem; returns the worst status.
int solve_stats(const dfmg_ctx *c, const SolveOut &so, const int *counter, const int *stopv, double tol, double secs,
                dfmg_stats *out) {
    int worst = DFMG_OK;
    for (int p = 0; p < c->np; ++p) {
        dfmg_stats &S = out[p];
        S = dfmg_stats{};
        const int cnt = std::min(counter[p], DFMG_MAX_HISTORY);
        S.cycles = counter[p] - 1;
        S.converged = stopv[p] == 1;
        S.fallback = so.fbk[p];
        S.fnorm = std::sqrt(so.th[p]) / tol;
        S.n_history = cnt;
        for (int i = 0; i < cnt; ++i) S.history[i] = so.hist[(size_t)p * DFMG_MAX_HISTORY + i];
        S.res0 = cnt ? S.history[0] : 0.0;
        S.res_final = cnt ? S.history[cnt - 1] : 0.0;
        S.rho = (S.cycles > 0 && S.res0 > 0) ? std::pow(S.res_final / S.res0, 1.0 / S.cycles) : 0.0;
        S.status = stopv[p] == 1 ? DFMG_OK : (stopv[p] == 2 ? DFMG_EDIVERGED : DFMG_ENOTCONV);
        S.solve_seconds = secs;
        if (S.status == DFMG_EDIVERGED) worst = DFMG_EDIVERGED;
        else if (S.status == DFMG_ENOTCONV && worst == DFMG_OK) worst = DFMG_ENOTCONV;
    }
    return worst;
}

int solve_status(int status) {
    if (status == DFMG_ENOTCONV) return fail(status, "maximum number of V-cycles reached");
    if (status == DFMG_EDIVERGED) return fail(status, "residual diverged (NaN/Inf or growth)");
    return DFMG_OK;
}


// ||F - K U||_2 of every problem (xoff as in solve_begin; with offsets the
// vectors are first copied into the finest level's internal F and U)
void residual_norms(dfmg_ctx *c, const double *F, const double *U, const int64_t *xoff, double *out) {
    const int L = c->L();
    const int64_t n = c->S().lv[L - 1].n;
    if (xoff) {
        LevelData<double> &v = c->dl[L - 1].d;
        launch_copy_off(n, F, xoff, n, v.F, nullptr, n, c->np, c->s);
        launch_copy_off(n, U, xoff, n, v.U, nullptr, n, c->np, c->s);
        F = v.F;
        U = v.U;
    }
    const int nb = spmv<double>(c, L - 1, F, U, c->rtmp, c->partial, nullptr);
    launch_reduce(nb, c->partial, c->nparts, c->scal, 1.0, c->np, c->s);
    std::vector<double> v(c->np);
    HIPCHK(hipMemcpyAsync(v.data(), c->scal, c->np * sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    for (int p = 0; p < c->np; ++p) out[p] = std::sqrt(v[p]);
}

// ||div u_h||_L2 of every problem, Up[p] = problem p's U on the device
void div_norms(dfmg_ctx *c, const double *const *Up, double *out) {
    const Hierarchy &H = c->S();
    const HostLevel &h = H.lv[H.pb.L - 1];
    for (int p = 0; p < c->np; ++p) {
        DivArgs a{};
        a.d = H.pb.d;
        a.k = H.pb.k;
        a.N = H.pb.N;
        for (int R = 0; R < 4; ++R) {
            a.off[R] = R <= h.nblk ? h.off[R] : 0;
            for (int j = 0; j < 3; ++j) a.nb[R][j] = R < h.nblk ? h.nb[R][j] : 1;
        }
        a.U = Up[p];
        a.dcoef = c->dcoef;
        a.pmass = c->pmass;
        a.dvec = c->dvec;
        a.partial = c->partial;
        launch_div(a, c->s);
        const int nb = blocks_for(h.n_q);
        launch_div_mass(a, nb, c->s);
        launch_reduce(nb, c->partial, 0, c->scal + p, 1.0, 1, c->s);
    }
    std::vector<double> v(c->np);
    HIPCHK(hipMemcpyAsync(v.data(), c->scal, c->np * sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    for (int p = 0; p < c->np; ++p) out[p] = std::sqrt(std::max(0.0, v[p]));
}

}  // namespace

extern "C" {

void dfmg_default_options(dfmg_options *o) {
    if (!o) return;
    o->nu1 = 2;
    o->nu2 = 2;
    o->eta = 0.0;
    o->precision = 0;
    o->smoother = 0;
    o->max_cycles = 200;
    o->use_graph = 1;
    o->cycles_per_check = 1;
    o->share_inverses = 1;
    o->inner_cycles = 1;
    o->multiplicative = 0;
    o->time_stepping = 0;
}

const char *dfmg_last_error(void) { return g_err.c_str(); }

int dfmg_setup(const dfmg_grid *grid, int k, double nu, double sigma, const dfmg_advection *adv,
               const dfmg_options *opt, dfmg_ctx **out) {
    return dfmg_batch_setup(1, grid, k, &nu, &sigma, adv, opt, out);
}

int dfmg_batch_setup(int nprob, const dfmg_grid *grid, int k, const double *nu, const double *sigma,
                     const dfmg_advection *adv, const dfmg_options *opt, dfmg_ctx **out) {
    if (!grid || !out || !nu || !sigma) return fail(DFMG_EINVAL, "null argument");
    if (nprob < 1 || nprob > 65535) return fail(DFMG_EINVAL, "batch size must be in [1, 65535]");
    *out = nullptr;
    return guarded([&] {
        const dfmg_options o = checked_options(opt, grid->dim);
        auto *c = new dfmg_ctx();
        try {
            c->np = nprob;
            c->P.resize(nprob);
            std::vector<std::string> errs(nprob);
            const int nth = std::max(1, std::min<int>(nprob, (int)std::thread::hardware_concurrency()));
            std::vector<std::thread> pool;
            for (int t = 0; t < nth; ++t)
                pool.emplace_back([&, t] {
                    for (int p = t; p < nprob; p += nth) {
                        try {
                            build_hierarchy(make_problem(grid, k, nu[p], sigma[p], adv ? adv + p : nullptr, o),
                                            c->P[p]);
                        } catch (const std::exception &e) {
                            errs[p] = e.what();
                        }
                    }
                });
            for (auto &th : pool) th.join();
            for (int p = 0; p < nprob; ++p)
                if (!errs[p].empty()) throw ArgError("problem " + std::to_string(p) + ": " + errs[p]);
        } catch (...) {
            delete c;
            throw;
        }
        init_ctx(c, o);
        *out = c;
    });
}

int dfmg_batch_size(const dfmg_ctx *c, int *nprob) {
    if (!c || !nprob) return fail(DFMG_EINVAL, "null argument");
    *nprob = c->np;
    return DFMG_OK;
}

void dfmg_destroy(dfmg_ctx *c) {
    if (!c) return;
    for (auto g : c->graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    for (hipEvent_t e : c->ev_flag)
        if (e) (void)hipEventDestroy(e);
    if (c->hflags) (void)hipHostFree(c->hflags);
    if (c->s) (void)hipStreamDestroy(c->s);
    delete c;
}

int dfmg_workspace_bytes(const dfmg_ctx *c, size_t *bytes) {
    if (!c || !bytes) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        Arena A;
        plan(const_cast<dfmg_ctx *>(c), A);
        *bytes = A.used + 256;
    });
}

int dfmg_bind(dfmg_ctx *c, void *ws, size_t bytes, void *stream) {
    if (!c || !ws) return fail(DFMG_EINVAL, "null argument");
    if (((uintptr_t)ws) & 255) return fail(DFMG_EINVAL, "workspace must be 256-byte aligned");
    return guarded([&] {
        if (c->bound) throw StateError("already bound");
        Arena M;
        plan(c, M);
        if (bytes < M.used) throw std::bad_alloc();
        Arena A;
        A.base = (char *)ws;
        plan(c, A);
        c->user = (hipStream_t)stream;
        HIPCHK(hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
        const Hierarchy &H = c->S();
        hipStream_t s = c->s;
        const int np = c->np;
        HIPCHK(hipEventRecord(c->ev_in, c->user));
        HIPCHK(hipStreamWaitEvent(s, c->ev_in, 0));
        for (int l = 0; l < H.pb.L; ++l) {
            const HostLevel &h = H.lv[l];
            DevLevel &v = c->dl[l];
            HIPCHK(hipMemsetAsync(v.d.U, 0, v.n * np * sizeof(double), s));
            HIPCHK(hipMemsetAsync(v.d.F, 0, v.n * np * sizeof(double), s));
            HIPCHK(hipMemsetAsync(v.d.r, 0, v.n * np * sizeof(double), s));
            for (int p = 0; p < np; ++p) up(v.d.val + p * v.sval, c->P[p].lv[l].val, s);
            if (c->mixed()) {
                HIPCHK(hipMemsetAsync(v.f.U, 0, v.n * np * sizeof(float), s));
                HIPCHK(hipMemsetAsync(v.f.F, 0, v.n * np * sizeof(float), s));
                HIPCHK(hipMemsetAsync(v.f.r, 0, v.n * np * sizeof(float), s));
                for (int p = 0; p < np; ++p) {
                    up32(v.f.val + p * v.sval, c->P[p].lv[l].val, s);
                    if (l > 0) up32(v.f.M + p * v.sM, c->P[p].lv[l].M, s);
                }
                if (l > 0) {
                    up32(v.f.P_v, h.P_v, s);
                    up32(v.f.R_v, h.R_v, s);
                    up32(v.f.P_ev, h.P_ev, s);
                    up32(v.f.R_ev, h.R_ev, s);
                }
                HIPCHK(hipMemsetAsync(v.psi, 0, v.npsi * np * sizeof(double), s));
                if (l == 0) {
                    for (int p = 0; p < np; ++p) up(v.Q0 + p * h.Q0.size(), c->P[p].lv[0].Q0, s);
                } else {
                    for (int p = 0; p < np; ++p) {
                        up32(v.Q + p * v.sQ, c->P[p].lv[l].Q, s);
                        up(v.qoff + p * h.n_patch, c->P[p].lv[l].qoff, s);
                        up(v.beta_row + p * v.nbeta, c->P[p].lv[l].beta_row, s);
                    }
                    HIPCHK(hipStreamSynchronize(s));
                    if (v.soa) {
                        // the single potential row of each full small subdomain, interleaved
                        const size_t ns = h.small_list.size();
                        std::vector<double> qs((size_t)kSmallPatch * ns);
                        for (int p = 0; p < np; ++p) {
                            const HostLevel &hp = c->P[p].lv[l];
                            std::fill(qs.begin(), qs.end(), 0.0);
                            for (size_t q = 0; q < ns; ++q) {
                                const int32_t i = h.small_list[q];
                                if (h.pptr[i + 1] - h.pptr[i] != kSmallPatch) continue;  // read from Q instead
                                for (int e = 0; e < kSmallPatch; ++e) qs[(size_t)e * ns + q] = hp.Q[hp.qoff[i] + e];
                            }
                            up32(v.qsoa + p * kSmallPatch * ns, qs, s);  // synchronous
                        }
                    }
                    up(v.Ps_v, h.Ps_v, s);
                    up(v.qptr, h.qptr, s);
                    up(v.beta_patch, h.beta_patch, s);
                    up(v.bigbeta, h.big_beta, s);
                    up(v.qinv_ptr, h.qinv_ptr, s);
                    up(v.qinv_pos, h.qinv_pos, s);
                    up(v.Ps_rp, h.Ps_rp, s);
                    up(v.Ps_ci, h.Ps_ci, s);
                    up(v.qinv_ell, h.qinv_ell, s);
                    up(v.Ps_eci, h.Ps_eci, s);
                    up(v.Ps_ev, h.Ps_ev, s);
                    HIPCHK(hipMemsetAsync(v.beta, 0, v.nbeta * np * sizeof(float), s));
                }
            }
            if (l == 0) {
                for (int p = 0; p < np; ++p) up(v.Kinv + p * h.Kinv.size(), c->P[p].lv[0].Kinv, s);
                continue;
            }
            up(v.pptr, h.pptr, s);
            up(v.pdofs, h.pdofs, s);
            up(v.inv_ptr, h.inv_ptr, s);
            up(v.inv_pos, h.inv_pos, s);
            up(v.col_list, h.col_list, s);
            up(v.small, h.small_list, s);
            up(v.bigent, h.big_ent, s);
            up(v.small_dofs, h.small_dofs, s);
            up(v.inv_pos4, h.inv_pos4, s);
            up(v.inv_ell, h.inv_ell, s);
            up(v.inv4_ell, h.inv4_ell, s);
            if (c->mult()) {
                up(v.mlane, h.mlane, s);
                up(v.mstride, h.mstride, s);
            }
            if (c->mult() && v.d.mval) {
                // the operator rows in lane order, per problem
                std::vector<double> mv((size_t)v.smval);
                for (int p = 0; p < np; ++p) {
                    const HostLevel &hp = c->P[p].lv[l];
                    std::fill(mv.begin(), mv.end(), 0.0);
                    for (size_t ln = 0; ln < h.mlane.size(); ++ln) {
                        const int32_t e = h.mlane[ln];
                        if (e < 0) continue;
                        const int64_t g = h.pdofs[e];
                        int R = 0;
                        while (g >= h.off[R + 1]) ++R;
                        const int64_t li = g - h.off[R];
                        const size_t base = (ln >> 6) * (size_t)v.mslots * 64 + (ln & 63) * kEllVec;
                        for (int sl = 0; sl < h.nslots[R]; ++sl)
                            mv[base + (size_t)(sl / kEllVec) * 64 * kEllVec + sl % kEllVec] = hp.val[hp.ell_index(R, li, sl)];
                    }
                    up(v.d.mval + (size_t)p * v.smval, mv, s);
                    HIPCHK(hipStreamSynchronize(s));  // mv is refilled for the next problem
                }
            }
            up(v.d.P_v, h.P_v, s);
            up(v.d.R_v, h.R_v, s);
            up(v.d.P_ev, h.P_ev, s);
            up(v.d.R_ev, h.R_ev, s);
            up(v.P_eci, h.P_eci, s);
            up(v.R_eci, h.R_eci, s);
            {
                std::vector<int4> bm(h.big_sub.size());
                for (size_t t = 0; t < bm.size(); ++t)
                    bm[t] = make_int4(h.big_mesh[4 * t], h.big_mesh[4 * t + 1], h.big_mesh[4 * t + 2],
                                      h.big_mesh[4 * t + 3]);
                up(v.bmesh, bm, s);
                // per problem: the offsets of each subdomain's inverse and
                // potential map (classes differ between problems)
                const size_t ns = h.small_list.size(), nb = h.big_sub.size();
                std::vector<int4> si(ns * np);
                std::vector<int2> bi(nb * np);
                const bool pot = !h.qptr.empty();
                for (int p = 0; p < np; ++p) {
                    const HostLevel &hp = c->P[p].lv[l];
                    for (size_t q = 0; q < ns; ++q) {
                        const int32_t i = h.small_list[q];
                        si[p * ns + q] = make_int4(h.pptr[i + 1] - h.pptr[i], hp.moff[i], pot ? hp.qoff[i] : 0,
                                                   pot ? h.qptr[i] : 0);
                    }
                    for (size_t t = 0; t < nb; ++t) {
                        const int32_t i = h.big_sub[t];
                        bi[p * nb + t] = make_int2(hp.moff[i], pot ? hp.qoff[i] : 0);
                    }
                }
                up(v.sinfo, si, s);
                up(v.binfo, bi, s);
                HIPCHK(hipStreamSynchronize(s));  // the host tables go out of scope
            }
            up(v.P_rp, h.P_rp, s);
            up(v.P_ci, h.P_ci, s);
            up(v.R_rp, h.R_rp, s);
            up(v.R_ci, h.R_ci, s);
            std::vector<int4> info(v.nent);
            for (int p = 0; p < np; ++p) {
                const HostLevel &hp = c->P[p].lv[l];
                up(v.d.M + p * v.sM, hp.M, s);
                up(v.moff + p * h.n_patch, hp.moff, s);
                for (int64_t q = 0; q < h.n_patch; ++q) {
                    const int nn = h.pptr[q + 1] - h.pptr[q];
                    for (int m = 0; m < nn; ++m) info[h.pptr[q] + m] = make_int4(hp.moff[q] + m * nn, h.pptr[q], nn, 0);
                }
                up(v.ent_info + p * v.nent, info, s);
                HIPCHK(hipStreamSynchronize(s));  // info is reused for the next problem
            }
            if (v.soa) {
                // chunks of W coefficients of a row (16 bytes: W = 2 in FP64, 4 in
                // FP32), chunk e / W of subdomain q at ((e / W) * ns + q) * W
                const size_t ns = h.small_list.size(), kk = (size_t)kSmallPatch * kSmallPatch;
                std::vector<double> ms(kk * ns);
                auto fill = [&](const HostLevel &hp, size_t W) {
                    std::fill(ms.begin(), ms.end(), 0.0);
                    for (size_t q = 0; q < ns; ++q) {
                        const int32_t i = h.small_list[q];
                        if (h.pptr[i + 1] - h.pptr[i] != kSmallPatch) continue;  // read from M instead
                        for (size_t e = 0; e < kk; ++e) ms[((e / W) * ns + q) * W + e % W] = hp.M[hp.moff[i] + e];
                    }
                };
                for (int p = 0; p < np; ++p) {
                    const HostLevel &hp = c->P[p].lv[l];
                    fill(hp, 2);
                    up(v.d.msoa + p * kk * ns, ms, s);
                    HIPCHK(hipStreamSynchronize(s));  // ms is refilled
                    if (c->mixed()) {
                        fill(hp, 4);
                        up32(v.f.msoa + p * kk * ns, ms, s);  // synchronous
                    }
                }
            }
        }
        up(c->eta, c->eta_host, s);
        up(c->eta_fixed, c->eta_host, s);
        up(c->unit, std::vector<double>(np, 1.0), s);
        HIPCHK(hipMemsetAsync(c->fallback, 0, np * sizeof(int), s));
        HIPCHK(hipMemsetAsync(c->rho_plain, 0, np * sizeof(double), s));
        up(c->dcoef, H.dcoef, s);
        up(c->pmass, H.pmass, s);
        up(c->wfine, H.lv[H.pb.L - 1].w, s);
        if (c->opt.time_stepping) {
            up(c->qbval, H.qbval, s);
            up(c->qbder, H.qbder, s);
            up(c->qw, H.qw, s);
            std::vector<double> sg(np);
            for (int p = 0; p < np; ++p) sg[p] = c->P[p].pb.sigma;
            up(c->sigma_dev, sg, s);
            HIPCHK(hipStreamSynchronize(s));
        }
        HIPCHK(hipMemsetAsync(c->counter, 0, kFlagSets * np * sizeof(int), s));
        HIPCHK(hipHostMalloc((void **)&c->hflags, 2 * kFlagSets * np * sizeof(int), hipHostMallocDefault));
        std::memset(c->hflags, 0, 2 * kFlagSets * np * sizeof(int));
        for (auto &e : c->ev_flag) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        upload_small_tables(c);
        HIPCHK(hipStreamSynchronize(s));
        c->bound = true;
    });
}

int dfmg_sizes(const dfmg_ctx *c, int level, int64_t *n_vel, int64_t *n_pres, int64_t *n_patch, int64_t *nnz) {
    if (!c) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level);
        const HostLevel &h = c->S().lv[level];
        if (n_vel) *n_vel = h.n_v;
        if (n_pres) *n_pres = h.n_q;
        if (n_patch) *n_patch = h.n_patch;
        if (nnz) {
            int64_t cnt = 0;
            for (double x : h.val)
                if (x != 0.0) ++cnt;
            *nnz = cnt;
        }
    });
}

int dfmg_set_eta(dfmg_ctx *c, const double *eta, int n) {
    if (!c || !eta) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        const int L = c->L(), m = L - 1;
        if (n != m && n != m * c->np) throw ArgError("need n_levels - 1 dampings, or that many per problem");
        for (int i = 0; i < n; ++i)
            if (!(eta[i] > 0.0 && eta[i] < 1.0)) throw ArgError("damping must lie in (0, 1)");
        for (int p = 0; p < c->np; ++p) {
            const double *e = (n == m) ? eta : eta + (size_t)p * m;
            for (int i = 0; i < m; ++i) c->eta_host[(size_t)p * L + (L - 1 - i)] = e[i];
        }
        c->learned = false;
        if (c->bound) {
            enter(c);
            clear_fallback(c);
            upload_eta(c);
            HIPCHK(hipMemcpyAsync(c->eta_fixed, c->eta_host.data(), c->eta_host.size() * sizeof(double),
                                  hipMemcpyHostToDevice, c->s));
            HIPCHK(hipStreamSynchronize(c->s));
            leave(c);
        }
    });
}

int dfmg_set_smoothing(dfmg_ctx *c, const int *nu1, const int *nu2, int n) {
    if (!c || !nu1 || !nu2) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        const int L = c->L();
        if (n != L - 1) throw ArgError("need n_levels - 1 smoothing counts");
        for (int i = 0; i < n; ++i)
            if (nu1[i] < 0 || nu1[i] > 16 || nu2[i] < 0 || nu2[i] > 16)
                throw ArgError("smoothing counts must lie in [0, 16]");
        for (int i = 0; i < n; ++i) {
            c->nu1l[L - 1 - i] = nu1[i];
            c->nu2l[L - 1 - i] = nu2[i];
        }
        drop_graph(c);
        if (c->bound) {
            enter(c);
            upload_small_tables(c);
            if (c->sched_on) build_schedule(c);
            leave(c);
        }
    });
}

int dfmg_get_smoothing(const dfmg_ctx *c, int *nu1, int *nu2) {
    if (!c || !nu1 || !nu2) return fail(DFMG_EINVAL, "null argument");
    const int L = c->L();
    for (int i = 0; i < L - 1; ++i) {
        nu1[i] = c->nu1l[L - 1 - i];
        nu2[i] = c->nu2l[L - 1 - i];
    }
    return DFMG_OK;
}

int dfmg_vcycle(dfmg_ctx *c, const double *F, double *U, int ncycles) {
    if (!c || !F || !U) return fail(DFMG_EINVAL, "null argument");
    if (ncycles < 0) return fail(DFMG_EINVAL, "ncycles < 0");
    return guarded([&] {
        enter(c);
        const int L = c->L(), np = c->np;
        const int64_t n = c->S().lv[L - 1].n;
        LevelData<double> &v = c->dl[L - 1].d;
        reset_flags(c);
        launch_copy(n, F, n, v.F, n, nullptr, np, c->s);
        launch_copy(n, U, n, v.U, n, nullptr, np, c->s);
        for (int i = 0; i < ncycles; ++i) run_cycle(c, 0);
        launch_copy(n, v.U, n, U, n, nullptr, np, c->s);
        HIPCHK(hipGetLastError());
        leave(c);
    });
}

int dfmg_residual_norm(dfmg_ctx *c, const double *F, const double *U, double *out) {
    if (!c || !F || !U || !out) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        enter(c);
        residual_norms(c, F, U, nullptr, out);
        leave(c);
    });
}

int dfmg_div_norm(dfmg_ctx *c, const double *U, double *out) {
    if (!c || !U || !out) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        enter(c);
        const int64_t n = c->S().lv[c->L() - 1].n;
        std::vector<const double *> Up(c->np);
        for (int p = 0; p < c->np; ++p) Up[p] = U + p * n;
        div_norms(c, Up.data(), out);
        leave(c);
    });
}

// load of one Crank-Nicolson / Adams-Bashforth step into Fout (see dfmg.h)
static void cnab_rhs(dfmg_ctx *c, const double *F2, const double *U, const double *Uold, double *Fout, int conv = 1) {
    if (!c->opt.time_stepping) throw StateError("set options.time_stepping = 1 before dfmg_setup");
    if (conv)
        for (const Hierarchy &Q : c->P)
            if (Q.pb.adv_kind != 0)
                throw ArgError("the Crank-Nicolson / Adams-Bashforth step is a generalized Stokes problem");
    const Hierarchy &H = c->S();
    const HostLevel &h = H.lv[H.pb.L - 1];
    spmv<double>(c, H.pb.L - 1, F2, U, Fout, nullptr, nullptr);  // F2 - K U^n
    CnabArgs a{};
    a.d = H.pb.d;
    a.k = H.pb.k;
    a.N = H.pb.N;
    a.nq = H.pb.k + 3;
    for (int R = 0; R < 4; ++R) a.off[R] = R <= a.d ? h.off[R] : h.n;
    for (int R = 0; R < 3; ++R)
        for (int j = 0; j < 3; ++j) a.nb[R][j] = R < a.d ? h.nb[R][j] : 1;
    a.n = h.n;
    a.svec = h.n;
    a.bval = c->qbval;
    a.bder = c->qbder;
    a.wq = c->qw;
    a.U = U;
    a.Uold = Uold;
    a.sigma = c->sigma_dev;
    a.G = c->qG;
    a.npts = c->npts;
    a.sG = c->npts * a.d;
    a.Fout = Fout;
    a.nprob = c->np;
    a.conv = conv;
    launch_cnab_load(a, c->s);
}

extern "C" int dfmg_go_rhs(dfmg_ctx *c, const double *F2, const double *U, double *Fout) {
    if (!c || !F2 || !U || !Fout) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        enter(c);
        cnab_rhs(c, F2, U, nullptr, Fout, 0);
        HIPCHK(hipGetLastError());
        leave(c);
    });
}

extern "C" int dfmg_cnab_rhs(dfmg_ctx *c, const double *F2, const double *U, const double *Uold, double *Fout) {
    if (!c || !F2 || !U || !Fout) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        enter(c);
        cnab_rhs(c, F2, U, Uold, Fout);
        HIPCHK(hipGetLastError());
        leave(c);
    });
}

int dfmg_solve(dfmg_ctx *c, const double *F, double *U, double tol, dfmg_stats *st) {
    if (!c || !F || !U) return fail(DFMG_EINVAL, "null argument");
    if (!(tol > 0.0)) return fail(DFMG_EINVAL, "tol must be positive");
    int status = DFMG_OK;
    std::vector<dfmg_stats> local;
    int rc = guarded([&] {
        enter(c);
        const auto t0 = std::chrono::steady_clock::now();
        solve_begin(c, F, U, nullptr, tol);
        const int np = c->np, kind = solve_kind(c);
        auto [buf, all] = pipelined_cycles(
            c->opt.max_cycles, c->opt.cycles_per_check,
            [&](int k, int b) {
                for (int i = 0; i < k; ++i) run_cycle(c, kind);
                flags_async(c, b);
            },
            [&](int b) { return flags_wait(c, b); });
        if (!all && kind != 2) {  // (a refinement step already ends with the check of its iterate)
            solve_limit(c);
            buf = 0;
            flags_async(c, buf);
            flags_wait(c, buf);
        }
        const int *counter = c->hflags + buf * kFlagSets * np, *stopv = counter + np;
        SolveOut so;
        solve_end_launch(c, U, nullptr, so);
        HIPCHK(hipStreamSynchronize(c->s));
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        local.assign(np, dfmg_stats{});
        status = solve_stats(c, so, counter, stopv, tol, secs, local.data());
        c->exit_mode = 0;  // launches outside a solve see no stopped problems
        leave(c);
    });
    if (st)
        for (size_t p = 0; p < local.size(); ++p) st[p] = local[p];
    if (rc != DFMG_OK) return rc;
    return solve_status(status);
}

int dfmg_cnab_step(dfmg_ctx *c, const double *F2, const double *Uold, const double *U, double *Unext, double tol,
                   dfmg_stats *st) {
    if (!c || !F2 || !U || !Unext) return fail(DFMG_EINVAL, "null argument");
    const int rc = guarded([&] {
        enter(c);
        cnab_rhs(c, F2, U, Uold, c->fstep);
        const int64_t n = c->S().lv[c->L() - 1].n;
        if (Unext != U) launch_copy(n, U, n, Unext, n, nullptr, c->np, c->s);
        HIPCHK(hipGetLastError());
        leave(c);
    });
    if (rc != DFMG_OK) return rc;
    return dfmg_solve(c, c->fstep, Unext, tol, st);
}

int dfmg_level_residual(dfmg_ctx *c, int level, const double *F, const double *U, double *r) {
    if (!c || !F || !U || !r) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level, 0);
        enter(c);
        spmv<double>(c, level, F, U, r, nullptr, nullptr);
        leave(c);
    });
}

int dfmg_time_kernel(dfmg_ctx *c, int kernel, int level, int reps, double *ms) {
    if (!c || !ms || reps < 1 || kernel < 0 || kernel > 3) return fail(DFMG_EINVAL, "invalid argument");
    return guarded([&] {
        check_level(c, level, kernel >= 2 ? 1 : 0);
        if ((kernel & 1) && !c->mixed()) throw ArgError("FP32 kernels exist with precision 1 only");
        enter(c);
        auto launch = [&] {
            if (kernel == 0) {
                LevelData<double> &v = c->dl[level].d;
                spmv<double>(c, level, v.F, v.U, v.r, nullptr, nullptr);
            } else if (kernel == 1) {
                LevelData<float> &v = c->dl[level].f;
                spmv<float>(c, level, v.F, v.U, v.r, nullptr, nullptr);
            } else if (kernel == 2) {
                LevelData<double> &v = c->dl[level].d;
                if (c->mult()) mult_sweep<double>(c, level, v.F, v.U, nullptr);
                else schwarz<double>(c, level, v.r, v.U, false, nullptr);
            } else {
                LevelData<float> &v = c->dl[level].f;
                schwarz<float>(c, level, v.r, v.U, false, nullptr);
            }
        };
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        launch();  // warm
        HIPCHK(hipEventRecord(e0, c->s));
        for (int i = 0; i < reps; ++i) launch();
        HIPCHK(hipEventRecord(e1, c->s));
        HIPCHK(hipEventSynchronize(e1));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *ms = (double)t / reps;
        leave(c);
    });
}

int dfmg_level_smooth(dfmg_ctx *c, int level, const double *F, double *U, int nsteps) {
    if (!c || !F || !U) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level, 1);
        enter(c);
        for (int i = 0; i < nsteps; ++i) {
            if (c->mult()) {
                mult_sweep<double>(c, level, F, U, nullptr);
                continue;
            }
            spmv<double>(c, level, F, U, c->rtmp, nullptr, nullptr);
            schwarz<double>(c, level, c->rtmp, U, false, nullptr);
        }
        leave(c);
    });
}

int dfmg_level_restrict(dfmg_ctx *c, int level, const double *r, double *G) {
    if (!c || !r || !G) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level, 1);
        enter(c);
        restrict_to<double>(c, level, r, G, nullptr);
        leave(c);
    });
}

int dfmg_level_prolong_add(dfmg_ctx *c, int level, const double *dU, double *U) {
    if (!c || !dU || !U) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level, 1);
        enter(c);
        prolong_add<double>(c, level, dU, U, nullptr);
        leave(c);
    });
}

int dfmg_coarse_solve(dfmg_ctx *c, const double *G, double *dU) {
    if (!c || !G || !dU) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        enter(c);
        coarse<double>(c, G, dU, nullptr);
        leave(c);
    });
}

int dfmg_get_tuning(const dfmg_ctx *c, int *lpr, int *smoother) {
    if (!c || !lpr || !smoother) return fail(DFMG_EINVAL, "null argument");
    for (int l = 0; l < c->L(); ++l) {
        lpr[l] = c->lpr[l];
        smoother[l] = (l >= 1 && l <= c->small_top) ? 5 : c->smoother[l];
    }
    return DFMG_OK;
}

int dfmg_set_tuning(dfmg_ctx *c, const int *lpr, const int *smoother) {
    if (!c || !lpr || !smoother) return fail(DFMG_EINVAL, "null argument");
    const int L = c->L();
    int top = 0;
    while (top + 1 < L && smoother[top + 1] == 5) ++top;
    for (int l = 0; l < L; ++l) {
        if (!(lpr[l] == 1 || lpr[l] == 2 || lpr[l] == 4)) return fail(DFMG_EINVAL, "lpr must be 1, 2 or 4");
        if (c->S().pb.geometry != 0 && lpr[l] != 1) return fail(DFMG_EINVAL, "mapped domains take lpr 1");
        const bool in_small = l >= 1 && l <= top;
        if (!in_small && !(smoother[l] >= 1 && smoother[l] <= 4))
            return fail(DFMG_EINVAL, "smoother must be 1 .. 4, or 5 on levels 1 .. t");
    }
    if (top > L - 2) return fail(DFMG_EINVAL, "the finest level cannot run in the single-workgroup cycle");
    if (top > 0 && c->S().pb.geometry != 0)
        return fail(DFMG_EINVAL, "mapped domains do not run the single-workgroup cycle");
    return guarded([&] {
        for (int l = 0; l < L; ++l) {
            c->lpr[l] = lpr[l];
            if (!(l >= 1 && l <= top)) c->smoother[l] = smoother[l];
        }
        c->small_top = top;
        drop_graph(c);
    });
}

int dfmg_get_tile_shape(const dfmg_ctx *c, int *bs, int *ms, int *tb) {
    if (!c || !bs || !ms || !tb) return fail(DFMG_EINVAL, "null argument");
    for (int l = 0; l < c->L(); ++l) {
        bs[l] = c->tile[l].bs;
        ms[l] = c->tile[l].ms;
        tb[l] = c->tile[l].tb;
    }
    return DFMG_OK;
}

int dfmg_set_tile_shape(dfmg_ctx *c, const int *bs, const int *ms, const int *tb) {
    if (!c || !bs || !ms || !tb) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        const int L = c->L();
        for (int l = 0; l < L; ++l) {
            if (bs[l] != 64 && bs[l] != 128 && bs[l] != 256 && bs[l] != 512)
                throw ArgError("threads per workgroup must be 64, 128, 256 or 512");
            if (ms[l] < 0 || ms[l] > 2) throw ArgError("inverse reading must be 0, 1 or 2");
            if (tb[l] != 32 && tb[l] != 64) throw ArgError("threads per boundary subdomain must be 32 or 64");
        }
        for (int l = 0; l < L; ++l) c->tile[l] = TileShape{bs[l], ms[l], tb[l]};
        drop_graph(c);
    });
}

int dfmg_time_cycle(dfmg_ctx *c, int reps, double *ms_out) {
    if (!c || !ms_out || reps < 1) return fail(DFMG_EINVAL, "invalid argument");
    return guarded([&] {
        enter(c);
        reset_flags(c);
        hipGraph_t g;
        hipGraphExec_t x;
        HIPCHK(hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal));
        if (c->mixed()) cycle_body<float>(c, false, true);
        else cycle_body<double>(c, false, false);
        HIPCHK(hipStreamEndCapture(c->s, &g));
        HIPCHK(hipGraphInstantiate(&x, g, nullptr, nullptr, 0));
        HIPCHK(hipGraphDestroy(g));
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipGraphLaunch(x, c->s));  // warm
        double best = 1e30;
        for (int round = 0; round < 3; ++round) {
            HIPCHK(hipEventRecord(e0, c->s));
            for (int i = 0; i < reps; ++i) HIPCHK(hipGraphLaunch(x, c->s));
            HIPCHK(hipEventRecord(e1, c->s));
            HIPCHK(hipEventSynchronize(e1));
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, e0, e1));
            best = std::min(best, (double)t / reps);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        HIPCHK(hipGraphExecDestroy(x));
        *ms_out = best;
        leave(c);
    });
}

int dfmg_autotune(dfmg_ctx *c, int reps, double *ms_out) {
    if (!c || reps < 1) return fail(DFMG_EINVAL, "invalid argument");
    return guarded([&] {
        enter(c);
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        auto timed = [&](auto &&fn) {
            fn();  // warm
            HIPCHK(hipEventRecord(e0, c->s));
            for (int i = 0; i < reps; ++i) fn();
            HIPCHK(hipEventRecord(e1, c->s));
            HIPCHK(hipEventSynchronize(e1));
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, e0, e1));
            return (double)t / reps;
        };
        const int L = c->L();
        // the variants are timed in the precision the V-cycles run in
        auto tune = [&](auto zero) {
            using T = decltype(zero);
            for (int l = 0; l < L; ++l) {
                LevelData<T> &v = c->dl[l].data<T>();
                double best = 1e30;
                int bl = c->lpr[l];
                for (int lp : {1, 2, 4}) {
                    if (c->S().pb.geometry != 0 && lp != 1) continue;  // mapped: one lane per row
                    c->lpr[l] = lp;
                    const double t = timed([&] { spmv<T>(c, l, v.F, v.U, v.r, nullptr, nullptr); });
                    if (t < best) {
                        best = t;
                        bl = lp;
                    }
                }
                c->lpr[l] = bl;
                if (ms_out) ms_out[2 * l] = best;
                if (l == 0) {
                    if (ms_out) ms_out[1] = 0.0;
                    continue;
                }
                if (c->mult()) {  // the additive forms do not run
                    if (ms_out) ms_out[2 * l + 1] = timed([&] { mult_sweep<T>(c, l, v.F, v.U, nullptr); });
                    launch_fill<T>(c->S().lv[l].n, v.U, c->S().lv[l].n, T(0), nullptr, c->np, c->s);
                    continue;
                }
                double bests = 1e30;
                int bs = c->smoother[l];
                for (int sm : {1, 2, 3, 4}) {
                    c->smoother[l] = sm;
                    const double t = timed([&] { schwarz<T>(c, l, v.r, v.U, false, nullptr); });
                    if (t < bests) {
                        bests = t;
                        bs = sm;
                    }
                }
                c->smoother[l] = bs;
                if (ms_out) ms_out[2 * l + 1] = bests;
                // the timing runs added corrections to U_l: restore zeros (the
                // internal U is reloaded or reset by every cycle)
                launch_fill<T>(c->S().lv[l].n, v.U, c->S().lv[l].n, T(0), nullptr, c->np, c->s);
            }
        };
        if (c->mixed()) tune(0.0f);
        else tune(0.0);
        // how many coarse levels run in the single-workgroup cycle: whole
        // V-cycles timed for every admissible choice (no check, no flags)
        reset_flags(c);
        int best_top = 0;
        double best_t = 1e30;
        // the FP32 cycle tracks potentials, mapped domains couple components: no t
        for (int t = 0; t <= (c->mixed() || c->mult() || c->S().pb.geometry != 0 ? 0 : L - 2); ++t) {
            if (t >= 1 && c->S().lv[t].n > kSmallCycleMax) break;
            c->small_top = t;
            const double ms = timed([&] {
                if (c->mixed()) cycle_body<float>(c, false, true);
                else cycle_body<double>(c, false, false);
            });
            if (ms < best_t) {
                best_t = ms;
                best_top = t;
            }
        }
        c->small_top = best_top;
        // in context: a kernel timed alone (back-to-back launches of itself)
        // can rank the variants otherwise than inside the cycle, where every
        // launch waits for the previous kernel's results.  Whole V-cycles,
        // captured and replayed as the solves run them, for every lanes-per-row
        // variant and smoother form of one level at a time (finest first, the
        // other levels as chosen); a variant replaces the choice when its
        // cycle is faster by more than 0.5% (best of three rounds of reps).
        auto cycle_ms = [&] {
            hipGraph_t g;
            hipGraphExec_t x;
            HIPCHK(hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal));
            if (c->mixed()) cycle_body<float>(c, false, true);
            else cycle_body<double>(c, false, false);
            HIPCHK(hipStreamEndCapture(c->s, &g));
            HIPCHK(hipGraphInstantiate(&x, g, nullptr, nullptr, 0));
            HIPCHK(hipGraphDestroy(g));
            HIPCHK(hipGraphLaunch(x, c->s));  // warm
            double best = 1e30;
            for (int round = 0; round < 3; ++round) {
                HIPCHK(hipEventRecord(e0, c->s));
                for (int i = 0; i < reps; ++i) HIPCHK(hipGraphLaunch(x, c->s));
                HIPCHK(hipEventRecord(e1, c->s));
                HIPCHK(hipEventSynchronize(e1));
                float t = 0.f;
                HIPCHK(hipEventElapsedTime(&t, e0, e1));
                best = std::min(best, (double)t / reps);
            }
            HIPCHK(hipGraphExecDestroy(x));
            return best;
        };
        double cur = cycle_ms();
        for (int l = L - 1; l > c->small_top && l >= 1; --l) {
            int bl = c->lpr[l];
            for (int lp : {1, 2, 4}) {
                if (lp == bl || (c->S().pb.geometry != 0 && lp != 1)) continue;
                c->lpr[l] = lp;
                const double t = cycle_ms();
                if (t < 0.995 * cur) {
                    cur = t;
                    bl = lp;
                }
                c->lpr[l] = bl;
            }
            if (c->mult()) continue;  // no additive forms to choose
            // the FP32 cycle runs forms 3 and 4 only (the others as 4)
            int bs = c->smoother[l];
            const std::vector<int> forms = c->mixed() ? std::vector<int>{3, 4} : std::vector<int>{1, 2, 3, 4};
            for (int sm : forms) {
                if (sm == bs || (c->mixed() && sm == 4 && bs != 3)) continue;
                c->smoother[l] = sm;
                const double t = cycle_ms();
                if (t < 0.995 * cur) {
                    cur = t;
                    bs = sm;
                }
                c->smoother[l] = bs;
            }
            // the tile shape of the form-4 local solves, where form 4 runs:
            // workgroup size, then the reading of shared inverses, then the
            // threads per boundary subdomain
            const bool form4 = c->mixed() ? c->smoother[l] != 3 : c->smoother[l] == 4;
            if (!form4) continue;
            auto try_shape = [&](TileShape cand) {
                const TileShape keep = c->tile[l];
                c->tile[l] = cand;
                const double t = cycle_ms();
                if (t < 0.995 * cur) cur = t;
                else c->tile[l] = keep;
            };
            for (int v : {64, 128, 256, 512})
                if (v != c->tile[l].bs) try_shape(TileShape{v, c->tile[l].ms, c->tile[l].tb});
            for (int v : {0, 1, 2})
                if (v != c->tile[l].ms) try_shape(TileShape{c->tile[l].bs, v, c->tile[l].tb});
            for (int v : {32, 64})
                if (v != c->tile[l].tb) try_shape(TileShape{c->tile[l].bs, c->tile[l].ms, v});
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        drop_graph(c);
        HIPCHK(hipStreamSynchronize(c->s));
        leave(c);
    });
}

int dfmg_mlp_forward(int n, const float *W, const float *X, float *Z, void *stream) {
    if (n < 0 || (n > 0 && (!W || !X || !Z))) return fail(DFMG_EINVAL, "invalid argument");
    return guarded([&] {
        launch_mlp_forward(n, W, X, Z, (hipStream_t)stream);
        HIPCHK(hipGetLastError());
    });
}

int dfmg_mlp_grad(int n, const float *W, const float *X, const float *Y, const float *Mk, float scale, float *work,
                  float *G, float *loss, void *stream) {
    if (n < 1 || !W || !X || !Y || !Mk || !work || !G || !loss) return fail(DFMG_EINVAL, "invalid argument");
    return guarded([&] {
        launch_mlp_grad(n, W, X, Y, Mk, scale, work, work + (int64_t)n * MLP_NPARAM, G, loss, (hipStream_t)stream);
        HIPCHK(hipGetLastError());
    });
}

static_assert(DFMG_MLP_SCRATCH_SAMPLES == MLP_SCRATCH_SAMPLES && DFMG_MLP_NPARAM == MLP_NPARAM,
              "header and library agree on the network's sizes");

int dfmg_mlp_grad_noalloc(int n, const float *W, const float *X, const float *Y, const float *Mk, float scale,
                          float *G, float *loss, void *stream) {
    if (!W || !X || !Y || !Mk || !G || !loss) return fail(DFMG_EINVAL, "invalid argument");
    if (n < 1 || n > MLP_SCRATCH_SAMPLES)
        return fail(DFMG_EINVAL, "n must lie in [1, " + std::to_string(MLP_SCRATCH_SAMPLES) +
                                     "] (the static scratch holds that many samples)");
    return guarded([&] {
        hipStream_t st = (hipStream_t)stream;
        int device = -1;
        if (st) HIPCHK(hipStreamGetDevice(st, &device));
        else HIPCHK(hipGetDevice(&device));
        hipError_t e = hipSuccess;
        float *scr = mlp_scratch(device, &e);
        if (!scr) throw HipError(std::string("scratch address: ") + hipGetErrorString(e));
        launch_mlp_grad_scratch(n, W, X, Y, Mk, scale, scr, G, loss, st);
        HIPCHK(hipGetLastError());
    });
}

int dfmg_mlp_adam(float *W, float *m, float *v, const float *G, int t, float lr, void *stream) {
    if (!W || !m || !v || !G || t < 1) return fail(DFMG_EINVAL, "invalid argument");
    return guarded([&] {
        launch_mlp_adam(W, m, v, G, t, lr, (hipStream_t)stream);
        HIPCHK(hipGetLastError());
    });
}

// network inputs of every problem: log10(nu) / 2, log10(sigma) / 4,
// |a| h / nu, k - 1.5
std::vector<float> network_features(const dfmg_ctx *c) {
    std::vector<float> feat((size_t)MLP_IN * c->np);
    for (int p = 0; p < c->np; ++p) {
        const Problem &pb = c->P[p].pb;
        const double amag = advection_speed(pb);
        feat[p * MLP_IN + 0] = (float)(std::log10(pb.nu) / 2.0);
        feat[p * MLP_IN + 1] = (float)(std::log10(std::max(pb.sigma, 1e-300)) / 4.0);
        feat[p * MLP_IN + 2] = (float)(amag / (pb.N * pb.nu));
        feat[p * MLP_IN + 3] = (float)(pb.k - 1.5);
    }
    return feat;
}

int dfmg_set_learned(dfmg_ctx *c, const float *W, const double *rho) {
    if (!c) return fail(DFMG_EINVAL, "null argument");
    if (W && c->mult()) return fail(DFMG_EINVAL, "learned dampings belong to the additive smoother");
    return guarded([&] {
        enter(c);
        if (!W) {
            c->learned = false;
            clear_fallback(c);
            upload_eta(c);
            c->nu1l.assign(c->L(), c->opt.nu1);
            c->nu2l.assign(c->L(), c->opt.nu2);
            drop_graph(c);
            upload_small_tables(c);
            if (c->sched_on) build_schedule(c);
            leave(c);
            return;
        }
        const std::vector<float> feat = network_features(c);
        // smoothing steps: the network's count outputs, the largest over the
        // batch (its problems share one launch sequence)
        const int L = c->L();
        std::vector<int> steps(L - 1, 1);
        for (int p = 0; p < c->np; ++p) {
            double z[MLP_OUT];
            mlp_forward_host(W, &feat[(size_t)p * MLP_IN], z);
            for (int i = 0; i < L - 1; ++i) {
                const long v = std::lround(z[MLP_ETA + std::min(i, MLP_OUT - MLP_ETA - 1)]);
                steps[i] = std::max(steps[i], (int)std::min(8L, std::max(1L, v)));
            }
        }
        for (int i = 0; i < L - 1; ++i) c->nu1l[L - 1 - i] = c->nu2l[L - 1 - i] = steps[i];
        drop_graph(c);
        upload_small_tables(c);
        up(c->mlpW, W, MLP_NPARAM, c->s);
        up(c->feat, feat, c->s);
        if (rho) up(c->rho_plain, rho, c->np, c->s);
        else clear_fallback(c);
        c->learned = true;
        apply_learned(c);
        if (c->sched_on) build_schedule(c);
        HIPCHK(hipStreamSynchronize(c->s));
        leave(c);
    });
}

int dfmg_set_chebyshev(dfmg_ctx *c, double alpha, int iters) {
    if (!c) return fail(DFMG_EINVAL, "null argument");
    if (alpha < 0.0) alpha = c->S().pb.d == 3 ? kChebAlpha3d : kChebAlpha2d;
    if (!(alpha == 0.0 || (alpha > 1.0 && alpha <= 1e6))) return fail(DFMG_EINVAL, "alpha must be 0 or in (1, 1e6]");
    if (alpha > 0.0 && (iters < 1 || iters > 1000)) return fail(DFMG_EINVAL, "iters must lie in [1, 1000]");
    if (alpha > 0.0 && c->mult()) return fail(DFMG_EINVAL, "the damping schedule belongs to the additive smoother");
    return guarded([&] {
        enter(c);
        drop_graph(c);
        if (alpha == 0.0) {
            c->sched_on = false;
        } else {
            estimate_lmax(c, iters);
            c->alpha.assign((size_t)c->np * c->L(), alpha);
            c->sched_on = true;
            build_schedule(c);
        }
        HIPCHK(hipStreamSynchronize(c->s));
        leave(c);
    });
}

int dfmg_set_chebyshev_alpha(dfmg_ctx *c, const double *alpha, int n) {
    if (!c || !alpha) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        const int L = c->L(), m = L - 1;
        if (n != m && n != m * c->np) throw ArgError("need n_levels - 1 or nprob * (n_levels - 1) ratios");
        for (int i = 0; i < n; ++i)
            if (!(alpha[i] > 1.0 && alpha[i] <= 1e6)) throw ArgError("alpha must lie in (1, 1e6]");
        if (!c->sched_on) throw StateError("no damping schedule in use (call dfmg_set_chebyshev first)");
        enter(c);
        for (int p = 0; p < c->np; ++p)
            for (int i = 0; i < m; ++i) c->alpha[(size_t)p * L + (L - 1 - i)] = alpha[(n == m ? 0 : (size_t)p * m) + i];
        build_schedule(c);
        leave(c);
    });
}

int dfmg_set_learned_chebyshev(dfmg_ctx *c, const float *W, const double *rho, int iters) {
    if (!c) return fail(DFMG_EINVAL, "null argument");
    if (W && c->mult()) return fail(DFMG_EINVAL, "the damping schedule belongs to the additive smoother");
    if (W && (iters < 1 || iters > 1000)) return fail(DFMG_EINVAL, "iters must lie in [1, 1000]");
    return guarded([&] {
        enter(c);
        const int L = c->L(), np = c->np;
        // the per-level dampings stay the fixed ones (the fallback's)
        c->learned = false;
        upload_eta(c);
        drop_graph(c);
        if (!W) {
            clear_fallback(c);
            c->sched_on = false;
            c->nu1l.assign(L, c->opt.nu1);
            c->nu2l.assign(L, c->opt.nu2);
            upload_small_tables(c);
            leave(c);
            return;
        }
        // the network's outputs on the device (the inference kernel), read back
        const std::vector<float> feat = network_features(c);
        up(c->mlpW, W, MLP_NPARAM, c->s);
        up(c->feat, feat, c->s);
        launch_mlp_forward(np, c->mlpW, c->feat, c->mlpZ, c->s);
        HIPCHK(hipGetLastError());
        std::vector<float> z((size_t)np * MLP_OUT);
        HIPCHK(hipMemcpyAsync(z.data(), c->mlpZ, z.size() * sizeof(float), hipMemcpyDeviceToHost, c->s));
        HIPCHK(hipStreamSynchronize(c->s));
        // outputs 0 .. MLP_ETA-1: logit of a / b = 1 / alpha per level (finest
        // first; deeper levels take the last); the others: step counts, the
        // largest over the batch (one launch sequence)
        std::vector<int> steps(L - 1, 1);
        c->alpha.assign((size_t)np * L, 0.0);
        for (int p = 0; p < np; ++p)
            for (int i = 0; i < L - 1; ++i) {
                const float *zp = &z[(size_t)p * MLP_OUT];
                const double q = 1.0 / (1.0 + std::exp(-(double)zp[std::min(i, MLP_ETA - 1)]));
                c->alpha[(size_t)p * L + (L - 1 - i)] = std::min(1e3, std::max(1.5, 1.0 / q));
                const long v = std::lround(zp[MLP_ETA + std::min(i, MLP_OUT - MLP_ETA - 1)]);
                steps[i] = std::max(steps[i], (int)std::min(8L, std::max(1L, v)));
            }
        for (int i = 0; i < L - 1; ++i) c->nu1l[L - 1 - i] = c->nu2l[L - 1 - i] = steps[i];
        upload_small_tables(c);
        if (rho) up(c->rho_plain, rho, np, c->s);
        else clear_fallback(c);
        if (c->lmax.empty()) estimate_lmax(c, iters);
        c->sched_on = true;
        build_schedule(c);
        leave(c);
    });
}

int dfmg_get_alpha(const dfmg_ctx *c, double *out) {
    if (!c || !out) return fail(DFMG_EINVAL, "null argument");
    if (!c->sched_on) return fail(DFMG_ESTATE, "no damping schedule in use");
    const int L = c->L();
    for (int p = 0; p < c->np; ++p)
        for (int i = 0; i < L - 1; ++i) out[(size_t)p * (L - 1) + i] = c->alpha[(size_t)p * L + (L - 1 - i)];
    return DFMG_OK;
}

int dfmg_get_lmax(const dfmg_ctx *c, double *out) {
    if (!c || !out) return fail(DFMG_EINVAL, "null argument");
    if (c->lmax.empty()) return fail(DFMG_ESTATE, "no eigenvalue estimate (call dfmg_set_chebyshev first)");
    const int L = c->L();
    for (int p = 0; p < c->np; ++p)
        for (int i = 0; i < L - 1; ++i) out[(size_t)p * (L - 1) + i] = c->lmax[(size_t)p * L + (L - 1 - i)];
    return DFMG_OK;
}

int dfmg_get_schedule(dfmg_ctx *c, double *out) {
    if (!c || !out) return fail(DFMG_EINVAL, "null argument");
    if (!c->sched_on) return fail(DFMG_ESTATE, "no damping schedule in use");
    return guarded([&] {
        enter(c);
        const int L = c->L();
        std::vector<double> e((size_t)c->np * L * kSchedPerLevel);
        HIPCHK(hipMemcpyAsync(e.data(), c->sched, e.size() * sizeof(double), hipMemcpyDeviceToHost, c->s));
        HIPCHK(hipStreamSynchronize(c->s));
        for (int p = 0; p < c->np; ++p)
            for (int i = 0; i < L - 1; ++i)
                std::copy_n(&e[((size_t)p * L + (L - 1 - i)) * kSchedPerLevel], kSchedPerLevel,
                            out + ((size_t)p * (L - 1) + i) * kSchedPerLevel);
        leave(c);
    });
}

int dfmg_get_eta(dfmg_ctx *c, double *eta) {
    if (!c || !eta) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        enter(c);
        const int L = c->L();
        std::vector<double> e((size_t)L * c->np);
        HIPCHK(hipMemcpyAsync(e.data(), c->eta, e.size() * sizeof(double), hipMemcpyDeviceToHost, c->s));
        HIPCHK(hipStreamSynchronize(c->s));
        for (int p = 0; p < c->np; ++p)
            for (int i = 0; i < L - 1; ++i) eta[(size_t)p * (L - 1) + i] = e[(size_t)p * L + (L - 1 - i)];
        leave(c);
    });
}

int dfmg_export_matrix(const dfmg_ctx *c, int level, int64_t *rowptr, int32_t *col, double *val) {
    if (!c || !rowptr || !col || !val) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level);
        const Hierarchy &H = c->S();
        const HostLevel &h = H.lv[level];
        const int d = H.pb.d;
        BlockGeom G{d, H.pb.k, H.pb.geometry != 0};
        int64_t nz = 0;
        rowptr[0] = 0;
        for (int R = 0; R <= d; ++R) {
            for (int64_t li = 0; li < h.off[R + 1] - h.off[R]; ++li) {
                int is[3];
                int64_t t = li;
                for (int j = 0; j < 3; ++j) {
                    is[j] = (int)(t % h.nb[R][j]);
                    t /= h.nb[R][j];
                }
                const int64_t grow = h.off[R] + li;
                for (int C = 0; C <= d; ++C) {
                    if (!G.coupled(R, C)) continue;
                    int lo[3] = {0, 0, 0}, W[3] = {1, 1, 1};
                    for (int j = 0; j < d; ++j) {
                        lo[j] = G.lo(R, C, j);
                        W[j] = G.width(R, C, j);
                    }
                    for (int o2 = 0; o2 < W[2]; ++o2)
                        for (int o1 = 0; o1 < W[1]; ++o1)
                            for (int o0 = 0; o0 < W[0]; ++o0) {
                                const int o[3] = {o0, o1, o2};
                                int js[3] = {0, 0, 0};
                                bool ok = true;
                                for (int j = 0; j < d; ++j) {
                                    js[j] = is[j] + lo[j] + o[j];
                                    if (js[j] < 0 || js[j] >= h.nb[C][j]) ok = false;
                                }
                                if (!ok) continue;
                                const int64_t gcol =
                                    h.off[C] + js[0] + (int64_t)h.nb[C][0] * (js[1] + (int64_t)h.nb[C][1] * js[2]);
                                const double x = level_entry(H, level, grow, gcol);
                                if (x == 0.0) continue;
                                col[nz] = (int32_t)gcol;
                                val[nz] = x;
                                ++nz;
                            }
                }
                rowptr[grow + 1] = nz;
            }
        }
    });
}

int dfmg_patch_total(const dfmg_ctx *c, int level, int64_t *total) {
    if (!c || !total) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level, 1);
        *total = (int64_t)c->S().lv[level].pdofs.size();
    });
}

int dfmg_export_patches(const dfmg_ctx *c, int level, int64_t *ptr, int32_t *dofs, int32_t *color) {
    if (!c || !ptr || !dofs || !color) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level, 1);
        const HostLevel &h = c->S().lv[level];
        for (size_t i = 0; i < h.pptr.size(); ++i) ptr[i] = h.pptr[i];
        std::memcpy(dofs, h.pdofs.data(), h.pdofs.size() * sizeof(int32_t));
        std::memcpy(color, h.color.data(), h.color.size() * sizeof(int32_t));
    });
}

int dfmg_export_sweep_colours(const dfmg_ctx *c, int level, int32_t *colour) {
    if (!c || !colour) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level, 1);
        const HostLevel &h = c->S().lv[level];
        for (int64_t i = 0; i < h.n_patch; ++i) colour[i] = h.mcolor[i];
    });
}

int dfmg_prolongation_nnz(const dfmg_ctx *c, int level, int64_t *nnz) {
    if (!c || !nnz) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level, 1);
        *nnz = (int64_t)c->S().lv[level].P_ci.size();
    });
}

int dfmg_export_prolongation(const dfmg_ctx *c, int level, int64_t *rowptr, int32_t *col, double *val) {
    if (!c || !rowptr || !col || !val) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level, 1);
        const HostLevel &h = c->S().lv[level];
        for (size_t i = 0; i < h.P_rp.size(); ++i) rowptr[i] = h.P_rp[i];
        std::memcpy(col, h.P_ci.data(), h.P_ci.size() * sizeof(int32_t));
        std::memcpy(val, h.P_v.data(), h.P_v.size() * sizeof(double));
    });
}

int dfmg_manufactured_rhs(const dfmg_ctx *c, double *F) {
    if (!c || !F) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        const int64_t n = c->S().lv[c->L() - 1].n;
        for (int p = 0; p < c->np; ++p) manufactured_rhs(c->P[p], F + p * n);
    });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of problems on different meshes: one single-mesh batch (dfmg_ctx)
// per (dim, n_elem, n_levels, k), each on its own stream.  A solve step forks
// the groups off the batch's stream, runs each group's cycle on its stream
// and joins them; with use_graph the whole fork/join step is captured once as
// one hipGraph with a branch per group and replayed.
// ---------------------------------------------------------------------------

struct dfmg_multi {
    std::vector<dfmg_ctx *> g;
    std::vector<std::vector<int>> member;  // caller indices of each group's problems
    std::vector<int> base;                 // first position of each group in group order
    std::vector<int64_t> off;              // caller offset of each problem's vectors (nprob + 1)
    std::vector<size_t> ws_off;            // workspace offset of each group
    size_t ws_tab = 0, ws_flags = 0, ws_total = 0;
    int64_t *tab = nullptr;                // device: caller offsets in group order
    int *dflags = nullptr;                 // device: counters, stop flags, near flags, group order
    int *hflags = nullptr;                 // pinned host copies of dflags, two buffers
    hipEvent_t ev_flag[2] = {nullptr, nullptr};
    dfmg_options opt{};
    int nprob = 0;
    bool bound = false;
    hipStream_t user = nullptr, s = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // per exit mode, as in dfmg_ctx
    int graph_kind[2] = {-1, -1};
    int exit_mode = 0;
};

namespace {

void mfork(dfmg_multi *m) {
    HIPCHK(hipEventRecord(m->ev_fork, m->s));
    for (dfmg_ctx *c : m->g) HIPCHK(hipStreamWaitEvent(c->s, m->ev_fork, 0));
}
void mjoin(dfmg_multi *m) {
    for (size_t i = 0; i < m->g.size(); ++i) {
        HIPCHK(hipEventRecord(m->ev_join[i], m->g[i]->s));
        HIPCHK(hipStreamWaitEvent(m->s, m->ev_join[i], 0));
    }
}
void menter(dfmg_multi *m) {
    if (!m->bound) throw StateError("workspace not bound (call dfmg_multi_bind first)");
    HIPCHK(hipEventRecord(m->ev_in, m->user));
    HIPCHK(hipStreamWaitEvent(m->s, m->ev_in, 0));
}
void mleave(dfmg_multi *m) {
    HIPCHK(hipEventRecord(m->ev_out, m->s));
    HIPCHK(hipStreamWaitEvent(m->user, m->ev_out, 0));
}

// counters, stop and near flags of every group into dflags (on the batch
// stream)
void pack_flags(dfmg_multi *m) {
    for (size_t i = 0; i < m->g.size(); ++i) {
        dfmg_ctx *c = m->g[i];
        launch_copy_int(c->np, c->counter, m->dflags + m->base[i], m->s);
        launch_copy_int(c->np, c->stop, m->dflags + m->nprob + m->base[i], m->s);
        launch_copy_int(c->np, c->near, m->dflags + 2 * m->nprob + m->base[i], m->s);
    }
}

// one cycle (kind as in run_cycle) of every group, then the flag packing
void multi_body(dfmg_multi *m, int kind) {
    mfork(m);
    for (dfmg_ctx *c : m->g) body(c, kind);
    mjoin(m);
    pack_flags(m);
}

void multi_step(dfmg_multi *m, int kind) {
    const int x = m->exit_mode;
    for (dfmg_ctx *c : m->g) c->exit_mode = x;
    if (!m->opt.use_graph) {
        multi_body(m, kind);
        return;
    }
    if (m->graph[x] && m->graph_kind[x] != kind) {
        HIPCHK(hipGraphExecDestroy(m->graph[x]));
        m->graph[x] = nullptr;
    }
    if (!m->graph[x]) {
        hipGraph_t gr;
        HIPCHK(hipStreamBeginCapture(m->s, hipStreamCaptureModeThreadLocal));
        multi_body(m, kind);
        HIPCHK(hipStreamEndCapture(m->s, &gr));
        HIPCHK(hipGraphInstantiate(&m->graph[x], gr, nullptr, nullptr, 0));
        HIPCHK(hipGraphDestroy(gr));
        m->graph_kind[x] = kind;
    }
    HIPCHK(hipGraphLaunch(m->graph[x], m->s));
}

void multi_drop_graph(dfmg_multi *m) {
    for (auto &g : m->graph)
        if (g) {
            HIPCHK(hipGraphExecDestroy(g));
            g = nullptr;
        }
}

// queue a copy of the packed flags into pinned buffer buf / wait for it
void multi_flags_async(dfmg_multi *m, int buf) {
    HIPCHK(hipMemcpyAsync(m->hflags + buf * kFlagSets * m->nprob, m->dflags, kFlagSets * m->nprob * sizeof(int),
                          hipMemcpyDeviceToHost, m->s));
    HIPCHK(hipEventRecord(m->ev_flag[buf], m->s));
}
int multi_flags_wait(dfmg_multi *m, int buf) {
    HIPCHK(hipEventSynchronize(m->ev_flag[buf]));
    const int st = flag_state(m->hflags + buf * kFlagSets * m->nprob + m->nprob, m->nprob);
    if (st & kAnyStopped) m->exit_mode = 1;
    return st;
}

void multi_plan(dfmg_multi *m) {
    size_t used = 0;
    m->ws_off.clear();
    for (dfmg_ctx *c : m->g) {
        Arena A;
        plan(c, A);
        m->ws_off.push_back(used);
        used += ((A.used + 256 + 255) & ~(size_t)255);
    }
    m->ws_tab = used;
    used += ((m->nprob * sizeof(int64_t) + 255) & ~(size_t)255);
    m->ws_flags = used;
    used += ((kFlagSets * m->nprob * sizeof(int) + 255) & ~(size_t)255);
    m->ws_total = used;
}

}  // namespace

extern "C" {

int dfmg_multi_setup(int nprob, const dfmg_grid *grids, const int *k, const double *nu, const double *sigma,
                     const dfmg_advection *adv, const dfmg_options *opt, dfmg_multi **out) {
    if (!grids || !k || !nu || !sigma || !out) return fail(DFMG_EINVAL, "null argument");
    if (nprob < 1 || nprob > 65535) return fail(DFMG_EINVAL, "batch size must be in [1, 65535]");
    *out = nullptr;
    return guarded([&] {
        auto *m = new dfmg_multi();
        try {
            m->nprob = nprob;
            // groups in order of first appearance
            std::vector<std::array<int, 4>> keys;
            std::vector<int> gid(nprob);
            for (int p = 0; p < nprob; ++p) {
                const std::array<int, 4> key{grids[p].dim, grids[p].n_elem, grids[p].n_levels, k[p]};
                auto it = std::find(keys.begin(), keys.end(), key);
                gid[p] = (int)(it - keys.begin());
                if (it == keys.end()) {
                    keys.push_back(key);
                    m->member.emplace_back();
                }
                m->member[gid[p]].push_back(p);
            }
            m->off.assign(nprob + 1, 0);
            for (size_t i = 0; i < keys.size(); ++i) {
                const auto &mem = m->member[i];
                std::vector<double> gnu, gsig;
                std::vector<dfmg_advection> gadv;
                for (int p : mem) {
                    gnu.push_back(nu[p]);
                    gsig.push_back(sigma[p]);
                    gadv.push_back(adv ? adv[p] : dfmg_advection{0, 0.0});
                }
                dfmg_ctx *c = nullptr;
                const int rc = dfmg_batch_setup((int)mem.size(), &grids[mem[0]], keys[i][3], gnu.data(), gsig.data(),
                                                gadv.data(), opt, &c);
                if (rc != DFMG_OK) throw ArgError("group " + std::to_string(i) + ": " + g_err);
                m->g.push_back(c);
                m->opt = c->opt;
                const int64_t n = c->S().lv[c->L() - 1].n;
                for (int p : mem) m->off[p + 1] = n;
            }
            for (int p = 0; p < nprob; ++p) m->off[p + 1] += m->off[p];
            int b = 0;
            for (const auto &mem : m->member) {
                m->base.push_back(b);
                b += (int)mem.size();
            }
        } catch (...) {
            dfmg_multi_destroy(m);
            throw;
        }
        *out = m;
    });
}

void dfmg_multi_destroy(dfmg_multi *m) {
    if (!m) return;
    for (auto g : m->graph)
        if (g) (void)hipGraphExecDestroy(g);
    for (dfmg_ctx *c : m->g) dfmg_destroy(c);
    for (hipEvent_t e : m->ev_join) (void)hipEventDestroy(e);
    if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
    if (m->ev_in) (void)hipEventDestroy(m->ev_in);
    if (m->ev_out) (void)hipEventDestroy(m->ev_out);
    if (m->s) (void)hipStreamDestroy(m->s);
    if (m->hflags) (void)hipHostFree(m->hflags);
    for (hipEvent_t e : m->ev_flag)
        if (e) (void)hipEventDestroy(e);
    delete m;
}

int dfmg_multi_layout(const dfmg_multi *m, int64_t *offset, int *n_groups) {
    if (!m) return fail(DFMG_EINVAL, "null argument");
    if (offset) std::copy(m->off.begin(), m->off.end(), offset);
    if (n_groups) *n_groups = (int)m->g.size();
    return DFMG_OK;
}

int dfmg_multi_workspace_bytes(const dfmg_multi *m, size_t *bytes) {
    if (!m || !bytes) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        multi_plan(const_cast<dfmg_multi *>(m));
        *bytes = m->ws_total;
    });
}

int dfmg_multi_bind(dfmg_multi *m, void *ws, size_t bytes, void *stream) {
    if (!m || !ws) return fail(DFMG_EINVAL, "null argument");
    if (((uintptr_t)ws) & 255) return fail(DFMG_EINVAL, "workspace must be 256-byte aligned");
    return guarded([&] {
        if (m->bound) throw StateError("already bound");
        multi_plan(m);
        if (bytes < m->ws_total) throw std::bad_alloc();
        char *base = (char *)ws;
        for (size_t i = 0; i < m->g.size(); ++i) {
            size_t b = 0;
            if (dfmg_workspace_bytes(m->g[i], &b) != DFMG_OK) throw ArgError(g_err);
            if (dfmg_bind(m->g[i], base + m->ws_off[i], b, stream) != DFMG_OK) throw HipError(g_err);
        }
        m->tab = (int64_t *)(base + m->ws_tab);
        m->dflags = (int *)(base + m->ws_flags);
        m->user = (hipStream_t)stream;
        HIPCHK(hipStreamCreateWithFlags(&m->s, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&m->ev_in, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&m->ev_out, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming));
        m->ev_join.assign(m->g.size(), nullptr);
        for (auto &e : m->ev_join) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIPCHK(hipHostMalloc((void **)&m->hflags, 2 * kFlagSets * m->nprob * sizeof(int), hipHostMallocDefault));
        std::memset(m->hflags, 0, 2 * kFlagSets * m->nprob * sizeof(int));
        for (auto &e : m->ev_flag) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        std::vector<int64_t> tab;
        for (const auto &mem : m->member)
            for (int p : mem) tab.push_back(m->off[p]);
        up(m->tab, tab, m->s);
        HIPCHK(hipMemsetAsync(m->dflags, 0, kFlagSets * m->nprob * sizeof(int), m->s));
        HIPCHK(hipStreamSynchronize(m->s));
        m->bound = true;
    });
}

int dfmg_multi_autotune(dfmg_multi *m, int reps) {
    if (!m || reps < 1) return fail(DFMG_EINVAL, "invalid argument");
    return guarded([&] {
        if (!m->bound) throw StateError("workspace not bound (call dfmg_multi_bind first)");
        std::vector<double> ms;
        for (dfmg_ctx *c : m->g) {
            ms.assign(2 * c->L(), 0.0);
            if (dfmg_autotune(c, reps, ms.data()) != DFMG_OK) throw HipError(g_err);
        }
        multi_drop_graph(m);
    });
}

int dfmg_multi_set_learned(dfmg_multi *m, const float *W, const double *rho) {
    if (!m) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        if (!m->bound) throw StateError("workspace not bound (call dfmg_multi_bind first)");
        for (size_t i = 0; i < m->g.size(); ++i) {
            std::vector<double> r;
            if (rho)
                for (int p : m->member[i]) r.push_back(rho[p]);
            if (dfmg_set_learned(m->g[i], W, rho ? r.data() : nullptr) != DFMG_OK) throw HipError(g_err);
        }
        multi_drop_graph(m);  // the step counts are part of the captured launches
    });
}

int dfmg_multi_set_chebyshev(dfmg_multi *m, double alpha, int iters) {
    if (!m) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        if (!m->bound) throw StateError("workspace not bound (call dfmg_multi_bind first)");
        for (size_t i = 0; i < m->g.size(); ++i)
            if (dfmg_set_chebyshev(m->g[i], alpha, iters) != DFMG_OK) throw ArgError(g_err);
        multi_drop_graph(m);
    });
}

int dfmg_multi_set_learned_chebyshev(dfmg_multi *m, const float *W, const double *rho, int iters) {
    if (!m) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        if (!m->bound) throw StateError("workspace not bound (call dfmg_multi_bind first)");
        for (size_t i = 0; i < m->g.size(); ++i) {
            std::vector<double> r;
            if (rho)
                for (int p : m->member[i]) r.push_back(rho[p]);
            if (dfmg_set_learned_chebyshev(m->g[i], W, rho ? r.data() : nullptr, iters) != DFMG_OK)
                throw HipError(g_err);
        }
        multi_drop_graph(m);
    });
}

int dfmg_multi_manufactured_rhs(const dfmg_multi *m, double *F) {
    if (!m || !F) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        for (size_t i = 0; i < m->g.size(); ++i)
            for (size_t j = 0; j < m->member[i].size(); ++j)
                manufactured_rhs(m->g[i]->P[j], F + m->off[m->member[i][j]]);
    });
}

int dfmg_multi_solve(dfmg_multi *m, const double *F, double *U, double tol, dfmg_stats *st) {
    if (!m || !F || !U) return fail(DFMG_EINVAL, "null argument");
    if (!(tol > 0.0)) return fail(DFMG_EINVAL, "tol must be positive");
    int status = DFMG_OK;
    std::vector<dfmg_stats> local;
    int rc = guarded([&] {
        menter(m);
        const auto t0 = std::chrono::steady_clock::now();
        const size_t G = m->g.size();
        mfork(m);
        for (size_t i = 0; i < G; ++i) solve_begin(m->g[i], F, U, m->tab + m->base[i], tol);
        m->exit_mode = 0;
        mjoin(m);
        const int kind = solve_kind(m->g[0]);
        auto [buf, all] = pipelined_cycles(
            m->opt.max_cycles, m->opt.cycles_per_check,
            [&](int k, int b) {
                for (int i = 0; i < k; ++i) multi_step(m, kind);
                multi_flags_async(m, b);
            },
            [&](int b) { return multi_flags_wait(m, b); });
        if (!all && kind != 2) {  // (a refinement step already ends with the check of its iterate)
            mfork(m);
            for (dfmg_ctx *c : m->g) solve_limit(c);
            mjoin(m);
            pack_flags(m);
            buf = 0;
            multi_flags_async(m, buf);
            multi_flags_wait(m, buf);
        }
        const int *fl = m->hflags + buf * kFlagSets * m->nprob;
        std::vector<SolveOut> so(G);
        mfork(m);
        for (size_t i = 0; i < G; ++i) solve_end_launch(m->g[i], U, m->tab + m->base[i], so[i]);
        mjoin(m);
        HIPCHK(hipStreamSynchronize(m->s));
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        local.assign(m->nprob, dfmg_stats{});
        std::vector<dfmg_stats> gs;
        int worst = DFMG_OK;
        for (size_t i = 0; i < G; ++i) {
            gs.assign(m->g[i]->np, dfmg_stats{});
            const int w = solve_stats(m->g[i], so[i], fl + m->base[i], fl + m->nprob + m->base[i], tol, secs,
                                      gs.data());
            if (w == DFMG_EDIVERGED || (w == DFMG_ENOTCONV && worst == DFMG_OK)) worst = w;
            for (size_t j = 0; j < gs.size(); ++j) local[m->member[i][j]] = gs[j];
        }
        status = worst;
        m->exit_mode = 0;
        for (dfmg_ctx *c : m->g) c->exit_mode = 0;
        mleave(m);
    });
    if (st)
        for (size_t p = 0; p < local.size(); ++p) st[p] = local[p];
    if (rc != DFMG_OK) return rc;
    return solve_status(status);
}

int dfmg_multi_residual_norm(dfmg_multi *m, const double *F, const double *U, double *out) {
    if (!m || !F || !U || !out) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        menter(m);
        std::vector<double> v;
        for (size_t i = 0; i < m->g.size(); ++i) {
            dfmg_ctx *c = m->g[i];
            v.assign(c->np, 0.0);
            enter(c);
            residual_norms(c, F, U, m->tab + m->base[i], v.data());
            leave(c);
            for (int j = 0; j < c->np; ++j) out[m->member[i][j]] = v[j];
        }
        mleave(m);
    });
}

int dfmg_multi_div_norm(dfmg_multi *m, const double *U, double *out) {
    if (!m || !U || !out) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        menter(m);
        std::vector<double> v;
        std::vector<const double *> Up;
        for (size_t i = 0; i < m->g.size(); ++i) {
            dfmg_ctx *c = m->g[i];
            v.assign(c->np, 0.0);
            Up.clear();
            for (int p : m->member[i]) Up.push_back(U + m->off[p]);
            enter(c);
            div_norms(c, Up.data(), v.data());
            leave(c);
            for (int j = 0; j < c->np; ++j) out[m->member[i][j]] = v[j];
        }
        mleave(m);
    });
}

}  // extern "C"
