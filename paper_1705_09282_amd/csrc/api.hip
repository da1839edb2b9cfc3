// C-ABI of the library: context, workspace binding, V-cycle orchestration,
// solve loop, diagnostics and exports.  See include/dfmg.h.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/dfmg.h"
#include "kernels.hpp"
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

// Typed values and vectors of one level: FP64 for the plain path, FP32 for
// the V-cycle inside the iterative refinement.
template <class T>
struct LevelData {
    T *val = nullptr, *U = nullptr, *F = nullptr, *r = nullptr, *M = nullptr, *delta = nullptr;
    T *P_v = nullptr, *R_v = nullptr;
};

struct DevLevel {
    LevelData<double> d;
    LevelData<float> f;
    int32_t *pptr = nullptr, *pdofs = nullptr, *moff = nullptr, *inv_ptr = nullptr, *inv_pos = nullptr;
    int4 *ent_info = nullptr;
    int32_t *col_list = nullptr;
    int32_t *P_rp = nullptr, *P_ci = nullptr, *R_rp = nullptr, *R_ci = nullptr;
    double *Kinv = nullptr;
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
    Hierarchy H;
    dfmg_options opt{};
    bool bound = false;
    hipStream_t user = nullptr, s = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<DevLevel> dl;
    double *eta = nullptr;       // per level
    double *partial = nullptr;   // per-block partial sums
    int nparts = 0;
    double *hist = nullptr;
    int *counter = nullptr, *stop = nullptr;
    double *thresh2 = nullptr, *scal = nullptr;
    double *dvec = nullptr, *dcoef = nullptr, *pmass = nullptr, *rtmp = nullptr, *wfine = nullptr;
    double *psi = nullptr;       // refinement: streamfunction increment
    hipGraphExec_t graph = nullptr;
    int graph_kind = -1;         // 0: FP64 cycle, 1: FP64 cycle with check, 2: refinement step
    std::vector<int> smoother;   // per level: 1 gather, 2 colour
    std::vector<int> lpr;        // per level: lanes per row of the residual kernel
    std::vector<double> eta_host;
    bool mixed() const { return opt.precision == 1; }
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
void take_level(Arena &A, const HostLevel &h, LevelData<T> &v, bool coarse) {
    v.U = A.take<T>(h.n);
    v.F = A.take<T>(h.n);
    v.r = A.take<T>(h.n);
    v.val = A.take<T>(h.val.size());
    if (coarse) return;
    v.M = A.take<T>(h.M.size());
    v.delta = A.take<T>(h.pdofs.size());
    v.P_v = A.take<T>(h.P_v.size());
    v.R_v = A.take<T>(h.R_v.size());
}

void plan(dfmg_ctx *c, Arena &A) {
    const Hierarchy &H = c->H;
    const int L = H.pb.L;
    c->dl.assign(L, DevLevel());
    int maxblocks = 1;
    int64_t nmax = 0;
    for (int l = 0; l < L; ++l) {
        const HostLevel &h = H.lv[l];
        DevLevel &v = c->dl[l];
        take_level(A, h, v.d, l == 0);
        if (c->mixed()) take_level(A, h, v.f, l == 0);
        nmax = std::max(nmax, h.n);
        maxblocks = std::max(maxblocks, spmv_blocks(h.n, 4));
        if (l == 0) {
            v.Kinv = A.take<double>(h.Kinv.size());
            continue;
        }
        v.pptr = A.take<int32_t>(h.pptr.size());
        v.pdofs = A.take<int32_t>(h.pdofs.size());
        v.moff = A.take<int32_t>(h.moff.size());
        v.inv_ptr = A.take<int32_t>(h.inv_ptr.size());
        v.inv_pos = A.take<int32_t>(h.inv_pos.size());
        v.ent_info = A.take<int4>(h.pdofs.size());
        v.col_list = A.take<int32_t>(h.col_list.size());
        v.P_rp = A.take<int32_t>(h.P_rp.size());
        v.P_ci = A.take<int32_t>(h.P_ci.size());
        v.R_rp = A.take<int32_t>(h.R_rp.size());
        v.R_ci = A.take<int32_t>(h.R_ci.size());
    }
    c->nparts = padded_grid(maxblocks);
    c->eta = A.take<double>(L);
    c->partial = A.take<double>(c->nparts);
    c->hist = A.take<double>(DFMG_MAX_HISTORY);
    c->counter = A.take<int>(1);
    c->stop = A.take<int>(1);
    c->thresh2 = A.take<double>(1);
    c->scal = A.take<double>(4);
    c->dvec = A.take<double>(H.lv[L - 1].n_q);
    c->dcoef = A.take<double>(H.dcoef.size());
    c->pmass = A.take<double>(H.pmass.size());
    c->rtmp = A.take<double>(nmax);
    c->wfine = A.take<double>(H.lv[L - 1].n_q);
    if (c->mixed()) c->psi = A.take<double>((size_t)(H.pb.N + H.pb.k - 1) * (H.pb.N + H.pb.k - 1));
}

template <class T>
void up(T *dst, const std::vector<T> &src, hipStream_t s) {
    if (!src.empty()) HIPCHK(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// FP32 copy of a host array, uploaded synchronously (the staging buffer is local)
void up32(float *dst, const std::vector<double> &src, hipStream_t s) {
    if (src.empty()) return;
    std::vector<float> tmp(src.begin(), src.end());
    HIPCHK(hipMemcpyAsync(dst, tmp.data(), tmp.size() * sizeof(float), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
}

template <class T>
SpmvArgsT<T> spmv_args(dfmg_ctx *c, int l, const T *F, const T *U, T *r, double *partial, const int *stop) {
    const HostLevel &h = c->H.lv[l];
    SpmvArgsT<T> a{};
    a.val = c->dl[l].data<T>().val;
    for (int R = 0; R < 4; ++R) a.val_off[R] = R < h.nblk ? h.val_off[R] : 0;
    for (int R = 0; R < 5; ++R) a.off[R] = R <= h.nblk ? h.off[R] : h.n;
    for (int R = 0; R < 4; ++R)
        for (int j = 0; j < 3; ++j) a.nb[R][j] = R < h.nblk ? h.nb[R][j] : 1;
    a.n = (int)h.n;
    a.nblocks = spmv_blocks(h.n, c->lpr[l]);
    a.F = F;
    a.U = U;
    a.r = r;
    a.partial = partial;
    a.stop = stop;
    return a;
}

// r = F - K_l U; returns the number of per-block partial sums written
template <class T>
int spmv(dfmg_ctx *c, int l, const T *F, const T *U, T *r, double *partial, const int *stop) {
    const SpmvArgsT<T> a = spmv_args<T>(c, l, F, U, r, partial, stop);
    launch_spmv<T>(c->H.pb.d, c->H.pb.k, c->lpr[l], a, c->s);
    return a.nblocks;
}

// eta * sum_i E_i^T M_i E_i r added to (or assigned into) U on level l.
template <class T>
void schwarz(dfmg_ctx *c, int l, const T *r, T *U, bool assign, const int *stop) {
    const HostLevel &h = c->H.lv[l];
    DevLevel &v = c->dl[l];
    PatchArgsT<T> a{};
    a.n = (int)h.n;
    a.nent = (int)h.pdofs.size();
    a.inv_ptr = v.inv_ptr;
    a.inv_pos = v.inv_pos;
    a.pptr = v.pptr;
    a.pdofs = v.pdofs;
    a.moff = v.moff;
    a.ent_info = v.ent_info;
    a.delta = v.data<T>().delta;
    a.M = v.data<T>().M;
    a.r = r;
    a.U = U;
    a.eta = c->eta + l;
    a.assign = assign ? 1 : 0;
    a.stop = stop;
    if (c->smoother[l] == 2) {
        if (assign) launch_fill<T>(h.n, U, T(0), stop, c->s);
        for (size_t col = 0; col + 1 < h.col_ptr.size(); ++col)
            launch_schwarz_colour<T>(a, v.col_list + h.col_ptr[col], h.col_ptr[col + 1] - h.col_ptr[col], c->s);
    } else {
        launch_schwarz_gather<T>(a, c->s);
    }
}

template <class T>
void restrict_to(dfmg_ctx *c, int l, const T *r, T *G, const int *stop) {
    const HostLevel &hc = c->H.lv[l - 1];
    DevLevel &v = c->dl[l];
    launch_csr<T>((int)hc.n, v.R_rp, v.R_ci, v.data<T>().R_v, r, G, 0, stop, c->s);
}

template <class T>
void prolong_add(dfmg_ctx *c, int l, const T *dU, T *U, const int *stop) {
    const HostLevel &h = c->H.lv[l];
    DevLevel &v = c->dl[l];
    launch_csr<T>((int)h.n, v.P_rp, v.P_ci, v.data<T>().P_v, dU, U, 1, stop, c->s);
}

// exact coarse solve (FP64 bordered inverse, FP64 accumulation)
template <class T>
void coarse(dfmg_ctx *c, const T *G, T *dU, const int *stop) {
    const int n = (int)c->H.lv[0].n;
    launch_gemv<T>(n, n, c->dl[0].Kinv, G, dU, stop, c->s);
}

// One V-cycle (Algorithm 1) on the finest level's internal U, F of type T.
// norm: the first residual of the finest level also feeds the convergence
// check.  fine_zero: the finest U is known to be zero (its first smoothing
// step then needs no residual).
template <class T>
void cycle_body(dfmg_ctx *c, bool norm, bool fine_zero) {
    const int L = c->H.pb.L, nu1 = c->opt.nu1, nu2 = c->opt.nu2;
    const int *stop = c->stop;
    if (L == 1) {
        LevelData<T> &v = c->dl[0].data<T>();
        if (norm) {
            const int np = spmv<T>(c, 0, v.F, v.U, v.r, c->partial, stop);
            launch_check(np, c->partial, c->hist, c->counter, c->stop, c->thresh2, DFMG_MAX_HISTORY, c->s);
        }
        coarse<T>(c, v.F, v.U, stop);  // exact solve of K U = F
        return;
    }
    for (int l = L - 1; l >= 1; --l) {
        LevelData<T> &v = c->dl[l].data<T>();
        const HostLevel &h = c->H.lv[l];
        bool zero = (l < L - 1) || fine_zero;
        bool first_res = (l == L - 1) && norm;
        for (int s = 0; s < nu1; ++s) {
            if (zero && !first_res) {
                schwarz<T>(c, l, v.F, v.U, true, stop);  // U = 0: residual is F
                zero = false;
                continue;
            }
            const int np = spmv<T>(c, l, v.F, v.U, v.r, first_res ? c->partial : nullptr, stop);
            if (first_res) {
                launch_check(np, c->partial, c->hist, c->counter, c->stop, c->thresh2, DFMG_MAX_HISTORY, c->s);
                first_res = false;
            }
            schwarz<T>(c, l, v.r, v.U, zero, stop);
            zero = false;
        }
        if (zero && !first_res) {
            launch_fill<T>(h.n, v.U, T(0), stop, c->s);
            restrict_to<T>(c, l, v.F, c->dl[l - 1].data<T>().F, stop);
        } else {
            const int np = spmv<T>(c, l, v.F, v.U, v.r, first_res ? c->partial : nullptr, stop);
            if (first_res)
                launch_check(np, c->partial, c->hist, c->counter, c->stop, c->thresh2, DFMG_MAX_HISTORY, c->s);
            restrict_to<T>(c, l, v.r, c->dl[l - 1].data<T>().F, stop);
        }
    }
    coarse<T>(c, c->dl[0].data<T>().F, c->dl[0].data<T>().U, stop);
    for (int l = 1; l < L; ++l) {
        LevelData<T> &v = c->dl[l].data<T>();
        prolong_add<T>(c, l, c->dl[l - 1].data<T>().U, v.U, stop);
        for (int s = 0; s < nu2; ++s) {
            spmv<T>(c, l, v.F, v.U, v.r, nullptr, stop);
            schwarz<T>(c, l, v.r, v.U, false, stop);
        }
    }
}

// One step of the FP64 iterative refinement: r = F - K U in FP64 (with the
// convergence check), inner_cycles FP32 V-cycles on K dU = r from dU = 0,
// then U += [curl psi; dU_p] in FP64 with psi recovered from dU_x.
void refine_body(dfmg_ctx *c) {
    const int L = c->H.pb.L;
    const HostLevel &h = c->H.lv[L - 1];
    DevLevel &v = c->dl[L - 1];
    const int np = spmv<double>(c, L - 1, v.d.F, v.d.U, v.d.r, c->partial, c->stop);
    launch_check(np, c->partial, c->hist, c->counter, c->stop, c->thresh2, DFMG_MAX_HISTORY, c->s);
    launch_cast(h.n, v.d.r, v.f.F, c->stop, c->s);
    for (int i = 0; i < c->opt.inner_cycles; ++i) cycle_body<float>(c, false, i == 0);
    RefineArgs a{};
    a.N = c->H.pb.N;
    a.k = c->H.pb.k;
    a.off_uy = h.off[1];
    a.off_p = h.off[2];
    a.n = h.n;
    a.X = v.f.U;
    a.dcoef = c->dcoef;
    a.psi = c->psi;
    a.U = v.d.U;
    a.stop = c->stop;
    launch_refine_update_2d(a, c->s);
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
    if (c->graph && c->graph_kind != kind) {
        HIPCHK(hipGraphExecDestroy(c->graph));
        c->graph = nullptr;
    }
    if (!c->graph) {
        hipGraph_t g;
        HIPCHK(hipStreamBeginCapture(c->s, hipStreamCaptureModeThreadLocal));
        body(c, kind);
        HIPCHK(hipStreamEndCapture(c->s, &g));
        HIPCHK(hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0));
        HIPCHK(hipGraphDestroy(g));
        c->graph_kind = kind;
    }
    HIPCHK(hipGraphLaunch(c->graph, c->s));
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

double read_scalar(dfmg_ctx *c, const double *dev) {
    double v = 0.0;
    HIPCHK(hipMemcpyAsync(&v, dev, sizeof(double), hipMemcpyDeviceToHost, c->s));
    HIPCHK(hipStreamSynchronize(c->s));
    return v;
}

void check_level(const dfmg_ctx *c, int level, int minlevel = 0) {
    if (level < minlevel || level >= c->H.pb.L) throw ArgError("level out of range");
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
}

const char *dfmg_last_error(void) { return g_err.c_str(); }

int dfmg_setup(const dfmg_grid *grid, int k, double nu, double sigma, const dfmg_advection *adv,
               const dfmg_options *opt, dfmg_ctx **out) {
    if (!grid || !out) return fail(DFMG_EINVAL, "null argument");
    *out = nullptr;
    return guarded([&] {
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
        }
        dfmg_options o;
        dfmg_default_options(&o);
        if (opt) o = *opt;
        if (o.nu1 < 0 || o.nu2 < 0 || o.max_cycles < 1 || o.cycles_per_check < 1)
            throw ArgError("invalid options");
        if (o.max_cycles > DFMG_MAX_HISTORY - 2) throw ArgError("max_cycles too large");
        if (o.precision != 0 && o.precision != 1) throw ArgError("precision must be 0 or 1");
        if (o.precision == 1 && pb.d != 2) throw ArgError("FP32 refinement is implemented for dim 2");
        if (o.inner_cycles < 1) throw ArgError("inner_cycles must be >= 1");
        if (o.smoother < 0 || o.smoother > 2) throw ArgError("smoother must be 0, 1 or 2");
        if (o.eta >= 1.0) throw ArgError("eta must be < 1");
        pb.share_inverses = o.share_inverses != 0;
        auto *c = new dfmg_ctx();
        try {
            build_hierarchy(pb, c->H);
        } catch (...) {
            delete c;
            throw;
        }
        c->opt = o;
        const double eta0 = o.eta > 0 ? o.eta : c->H.default_eta;
        c->eta_host.assign(pb.L, eta0);
        c->eta_host[0] = 0.0;
        c->smoother.assign(pb.L, o.smoother == 2 ? 2 : 1);
        c->lpr.assign(pb.L, 1);
        for (int l = 0; l < pb.L; ++l) {
            const int64_t n = c->H.lv[l].n;
            c->lpr[l] = n < 20000 ? 4 : (n < 100000 ? 2 : 1);
        }
        *out = c;
    });
}

void dfmg_destroy(dfmg_ctx *c) {
    if (!c) return;
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
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
        Arena M;
        plan(c, M);
        if (bytes < M.used) throw std::bad_alloc();
        if (c->bound) throw StateError("already bound");
        Arena A;
        A.base = (char *)ws;
        plan(c, A);
        c->user = (hipStream_t)stream;
        HIPCHK(hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
        const Hierarchy &H = c->H;
        hipStream_t s = c->s;
        HIPCHK(hipEventRecord(c->ev_in, c->user));
        HIPCHK(hipStreamWaitEvent(s, c->ev_in, 0));
        for (int l = 0; l < H.pb.L; ++l) {
            const HostLevel &h = H.lv[l];
            DevLevel &v = c->dl[l];
            HIPCHK(hipMemsetAsync(v.d.U, 0, h.n * sizeof(double), s));
            HIPCHK(hipMemsetAsync(v.d.F, 0, h.n * sizeof(double), s));
            HIPCHK(hipMemsetAsync(v.d.r, 0, h.n * sizeof(double), s));
            up(v.d.val, h.val, s);
            if (c->mixed()) {
                HIPCHK(hipMemsetAsync(v.f.U, 0, h.n * sizeof(float), s));
                HIPCHK(hipMemsetAsync(v.f.F, 0, h.n * sizeof(float), s));
                HIPCHK(hipMemsetAsync(v.f.r, 0, h.n * sizeof(float), s));
                up32(v.f.val, h.val, s);
                if (l > 0) {
                    up32(v.f.M, h.M, s);
                    up32(v.f.P_v, h.P_v, s);
                    up32(v.f.R_v, h.R_v, s);
                }
            }
            if (l == 0) {
                up(v.Kinv, h.Kinv, s);
                continue;
            }
            up(v.pptr, h.pptr, s);
            up(v.pdofs, h.pdofs, s);
            up(v.moff, h.moff, s);
            up(v.inv_ptr, h.inv_ptr, s);
            up(v.inv_pos, h.inv_pos, s);
            {
                std::vector<int4> info(h.pdofs.size());
                for (int64_t p = 0; p < h.n_patch; ++p) {
                    const int nn = h.pptr[p + 1] - h.pptr[p];
                    for (int m = 0; m < nn; ++m)
                        info[h.pptr[p] + m] = make_int4(h.moff[p] + m * nn, h.pptr[p], nn, 0);
                }
                up(v.ent_info, info, s);
                HIPCHK(hipStreamSynchronize(s));  // info is a local host buffer
            }
            up(v.col_list, h.col_list, s);
            up(v.d.M, h.M, s);
            up(v.P_rp, h.P_rp, s);
            up(v.P_ci, h.P_ci, s);
            up(v.d.P_v, h.P_v, s);
            up(v.R_rp, h.R_rp, s);
            up(v.R_ci, h.R_ci, s);
            up(v.d.R_v, h.R_v, s);
        }
        up(c->eta, c->eta_host, s);
        up(c->dcoef, H.dcoef, s);
        up(c->pmass, H.pmass, s);
        up(c->wfine, H.lv[H.pb.L - 1].w, s);
        HIPCHK(hipMemsetAsync(c->stop, 0, sizeof(int), s));
        HIPCHK(hipMemsetAsync(c->counter, 0, sizeof(int), s));
        HIPCHK(hipStreamSynchronize(s));
        c->bound = true;
    });
}

int dfmg_sizes(const dfmg_ctx *c, int level, int64_t *n_vel, int64_t *n_pres, int64_t *n_patch, int64_t *nnz) {
    if (!c) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level);
        const HostLevel &h = c->H.lv[level];
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
        const int L = c->H.pb.L;
        if (n != L - 1) throw ArgError("need n_levels - 1 dampings");
        for (int i = 0; i < n; ++i)
            if (!(eta[i] > 0.0 && eta[i] < 1.0)) throw ArgError("damping must lie in (0, 1)");
        for (int i = 0; i < n; ++i) c->eta_host[L - 1 - i] = eta[i];
        if (c->bound) {
            enter(c);
            HIPCHK(hipMemcpyAsync(c->eta, c->eta_host.data(), L * sizeof(double), hipMemcpyHostToDevice, c->s));
            HIPCHK(hipStreamSynchronize(c->s));
            leave(c);
        }
    });
}

int dfmg_vcycle(dfmg_ctx *c, const double *F, double *U, int ncycles) {
    if (!c || !F || !U) return fail(DFMG_EINVAL, "null argument");
    if (ncycles < 0) return fail(DFMG_EINVAL, "ncycles < 0");
    return guarded([&] {
        enter(c);
        const int L = c->H.pb.L;
        const int64_t n = c->H.lv[L - 1].n;
        LevelData<double> &v = c->dl[L - 1].d;
        launch_fill_int(1, c->stop, 0, c->s);
        launch_copy(n, F, v.F, nullptr, c->s);
        launch_copy(n, U, v.U, nullptr, c->s);
        for (int i = 0; i < ncycles; ++i) run_cycle(c, 0);
        launch_copy(n, v.U, U, nullptr, c->s);
        HIPCHK(hipGetLastError());
        leave(c);
    });
}

int dfmg_residual_norm(dfmg_ctx *c, const double *F, const double *U, double *out) {
    if (!c || !F || !U || !out) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        enter(c);
        const int L = c->H.pb.L;
        const int nb = spmv<double>(c, L - 1, F, U, c->rtmp, c->partial, nullptr);
        launch_reduce(nb, c->partial, c->scal, 1.0, c->s);
        *out = std::sqrt(read_scalar(c, c->scal));
        leave(c);
    });
}

int dfmg_div_norm(dfmg_ctx *c, const double *U, double *out) {
    if (!c || !U || !out) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        enter(c);
        const Hierarchy &H = c->H;
        const HostLevel &h = H.lv[H.pb.L - 1];
        DivArgs a{};
        a.d = H.pb.d;
        a.k = H.pb.k;
        a.N = H.pb.N;
        for (int R = 0; R < 4; ++R) {
            a.off[R] = R <= h.nblk ? h.off[R] : 0;
            for (int j = 0; j < 3; ++j) a.nb[R][j] = R < h.nblk ? h.nb[R][j] : 1;
        }
        a.U = U;
        a.dcoef = c->dcoef;
        a.pmass = c->pmass;
        a.dvec = c->dvec;
        a.partial = c->partial;
        launch_div(a, c->s);
        const int nb = blocks_for(h.n_q);
        launch_div_mass(a, nb, c->s);
        launch_reduce(nb, c->partial, c->scal, 1.0, c->s);
        const double v = read_scalar(c, c->scal);
        *out = std::sqrt(std::max(0.0, v));
        leave(c);
    });
}

int dfmg_solve(dfmg_ctx *c, const double *F, double *U, double tol, dfmg_stats *st) {
    if (!c || !F || !U) return fail(DFMG_EINVAL, "null argument");
    if (!(tol > 0.0)) return fail(DFMG_EINVAL, "tol must be positive");
    int status = DFMG_OK;
    dfmg_stats local{};
    int rc = guarded([&] {
        enter(c);
        const auto t0 = std::chrono::steady_clock::now();
        const int L = c->H.pb.L;
        const HostLevel &h = c->H.lv[L - 1];
        const int64_t n = h.n;
        LevelData<double> &v = c->dl[L - 1].d;
        const int nb = blocks_for(n);
        const int kind = c->mixed() ? 2 : 1;
        launch_fill_int(1, c->stop, 0, c->s);
        launch_fill_int(1, c->counter, 0, c->s);
        launch_copy(n, F, v.F, nullptr, c->s);
        launch_copy(n, U, v.U, nullptr, c->s);
        launch_dot_partial((int)n, v.F, v.F, c->partial, nb, c->s);
        launch_reduce(nb, c->partial, c->thresh2, tol * tol, c->s);
        const int maxc = c->opt.max_cycles;
        int launched = 0, counter = 0, stopv = 0;
        while (launched < maxc) {
            const int chunk = std::min(c->opt.cycles_per_check, maxc - launched);
            for (int i = 0; i < chunk; ++i) run_cycle(c, kind);
            launched += chunk;
            int hv[2];
            HIPCHK(hipMemcpyAsync(&hv[0], c->counter, sizeof(int), hipMemcpyDeviceToHost, c->s));
            HIPCHK(hipMemcpyAsync(&hv[1], c->stop, sizeof(int), hipMemcpyDeviceToHost, c->s));
            HIPCHK(hipStreamSynchronize(c->s));
            counter = hv[0];
            stopv = hv[1];
            if (stopv) break;
        }
        if (!stopv) {
            // limit reached: measure the residual of the last iterate
            const int np = spmv<double>(c, L - 1, v.F, v.U, v.r, c->partial, nullptr);
            launch_check(np, c->partial, c->hist, c->counter, c->stop, c->thresh2, DFMG_MAX_HISTORY, c->s);
            int hv[2];
            HIPCHK(hipMemcpyAsync(&hv[0], c->counter, sizeof(int), hipMemcpyDeviceToHost, c->s));
            HIPCHK(hipMemcpyAsync(&hv[1], c->stop, sizeof(int), hipMemcpyDeviceToHost, c->s));
            HIPCHK(hipStreamSynchronize(c->s));
            counter = hv[0];
            stopv = hv[1];
        }
        // zero-mean pressure: p <- p - (w^T p) 1 (partition of unity, |Omega| = 1)
        launch_dot_partial((int)h.n_q, v.U + h.n_v, c->wfine, c->partial, blocks_for(h.n_q), c->s);
        launch_reduce(blocks_for(h.n_q), c->partial, c->scal, 1.0, c->s);
        launch_sub_scalar((int)h.n_q, v.U + h.n_v, c->scal, c->s);
        launch_copy(n, v.U, U, nullptr, c->s);
        local.cycles = counter - 1;
        local.converged = stopv == 1;
        std::vector<double> hist(std::min(counter, DFMG_MAX_HISTORY));
        HIPCHK(hipMemcpyAsync(hist.data(), c->hist, hist.size() * sizeof(double), hipMemcpyDeviceToHost, c->s));
        HIPCHK(hipMemcpyAsync(&local.fnorm, c->thresh2, sizeof(double), hipMemcpyDeviceToHost, c->s));
        HIPCHK(hipStreamSynchronize(c->s));
        local.fnorm = std::sqrt(local.fnorm) / tol;
        local.n_history = (int)hist.size();
        for (size_t i = 0; i < hist.size(); ++i) local.history[i] = hist[i];
        local.res0 = hist.empty() ? 0.0 : hist[0];
        local.res_final = hist.empty() ? 0.0 : hist.back();
        local.rho = (local.cycles > 0 && local.res0 > 0) ? std::pow(local.res_final / local.res0, 1.0 / local.cycles)
                                                          : 0.0;
        status = stopv == 1 ? DFMG_OK : (stopv == 2 ? DFMG_EDIVERGED : DFMG_ENOTCONV);
        local.status = status;
        local.solve_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        leave(c);
    });
    if (st) *st = local;
    if (rc != DFMG_OK) return rc;
    if (status == DFMG_ENOTCONV) return fail(status, "maximum number of V-cycles reached");
    if (status == DFMG_EDIVERGED) return fail(status, "residual diverged (NaN/Inf or growth)");
    return DFMG_OK;
}

int dfmg_level_residual(dfmg_ctx *c, int level, const double *F, const double *U, double *r) {
    if (!c || !F || !U || !r) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level, 1);
        enter(c);
        spmv<double>(c, level, F, U, r, nullptr, nullptr);
        leave(c);
    });
}

int dfmg_time_residual(dfmg_ctx *c, int level, const double *F, const double *U, double *r, int reps,
                       double *ms) {
    if (!c || !F || !U || !r || !ms || reps < 1) return fail(DFMG_EINVAL, "invalid argument");
    return guarded([&] {
        check_level(c, level, 0);
        enter(c);
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        spmv<double>(c, level, F, U, r, nullptr, nullptr);  // warm
        HIPCHK(hipEventRecord(e0, c->s));
        for (int i = 0; i < reps; ++i) spmv<double>(c, level, F, U, r, nullptr, nullptr);
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
    for (int l = 0; l < c->H.pb.L; ++l) {
        lpr[l] = c->lpr[l];
        smoother[l] = c->smoother[l];
    }
    return DFMG_OK;
}

int dfmg_set_tuning(dfmg_ctx *c, const int *lpr, const int *smoother) {
    if (!c || !lpr || !smoother) return fail(DFMG_EINVAL, "null argument");
    for (int l = 0; l < c->H.pb.L; ++l)
        if (!(lpr[l] == 1 || lpr[l] == 2 || lpr[l] == 4) || !(smoother[l] == 1 || smoother[l] == 2))
            return fail(DFMG_EINVAL, "lpr must be 1, 2 or 4 and smoother 1 or 2");
    return guarded([&] {
        for (int l = 0; l < c->H.pb.L; ++l) {
            c->lpr[l] = lpr[l];
            c->smoother[l] = smoother[l];
        }
        if (c->graph) {
            HIPCHK(hipGraphExecDestroy(c->graph));
            c->graph = nullptr;
        }
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
        const int L = c->H.pb.L;
        // the variants are timed in the precision the V-cycles run in
        auto tune = [&](auto zero) {
            using T = decltype(zero);
            for (int l = 0; l < L; ++l) {
                LevelData<T> &v = c->dl[l].data<T>();
                double best = 1e30;
                int bl = c->lpr[l];
                for (int lp : {1, 2, 4}) {
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
                double bests = 1e30;
                int bs = c->smoother[l];
                for (int sm : {1, 2}) {
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
                launch_fill<T>(c->H.lv[l].n, v.U, T(0), nullptr, c->s);
            }
        };
        if (c->mixed()) tune(0.0f);
        else tune(0.0);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (c->graph) {
            HIPCHK(hipGraphExecDestroy(c->graph));
            c->graph = nullptr;
        }
        HIPCHK(hipStreamSynchronize(c->s));
        leave(c);
    });
}

int dfmg_export_matrix(const dfmg_ctx *c, int level, int64_t *rowptr, int32_t *col, double *val) {
    if (!c || !rowptr || !col || !val) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level);
        const HostLevel &h = c->H.lv[level];
        const int d = c->H.pb.d;
        BlockGeom G{d, c->H.pb.k};
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
                                const double x = level_entry(c->H, level, grow, gcol);
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
        *total = (int64_t)c->H.lv[level].pdofs.size();
    });
}

int dfmg_export_patches(const dfmg_ctx *c, int level, int64_t *ptr, int32_t *dofs, int32_t *color) {
    if (!c || !ptr || !dofs || !color) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level, 1);
        const HostLevel &h = c->H.lv[level];
        for (size_t i = 0; i < h.pptr.size(); ++i) ptr[i] = h.pptr[i];
        std::memcpy(dofs, h.pdofs.data(), h.pdofs.size() * sizeof(int32_t));
        std::memcpy(color, h.color.data(), h.color.size() * sizeof(int32_t));
    });
}

int dfmg_prolongation_nnz(const dfmg_ctx *c, int level, int64_t *nnz) {
    if (!c || !nnz) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level, 1);
        *nnz = (int64_t)c->H.lv[level].P_ci.size();
    });
}

int dfmg_export_prolongation(const dfmg_ctx *c, int level, int64_t *rowptr, int32_t *col, double *val) {
    if (!c || !rowptr || !col || !val) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] {
        check_level(c, level, 1);
        const HostLevel &h = c->H.lv[level];
        for (size_t i = 0; i < h.P_rp.size(); ++i) rowptr[i] = h.P_rp[i];
        std::memcpy(col, h.P_ci.data(), h.P_ci.size() * sizeof(int32_t));
        std::memcpy(val, h.P_v.data(), h.P_v.size() * sizeof(double));
    });
}

int dfmg_manufactured_rhs(const dfmg_ctx *c, double *F) {
    if (!c || !F) return fail(DFMG_EINVAL, "null argument");
    return guarded([&] { manufactured_rhs(c->H, F); });
}

}  // extern "C"
