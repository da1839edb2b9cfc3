// Host-side hierarchy construction.  See setup.hpp for the storage layout.
#include "setup.hpp"

#include <algorithm>
#include <cmath>
#include <exception>
#include <stdexcept>
#include <thread>
#include <utility>

namespace dfmg {

// Host threads for the setup loops: every hardware thread, at most 16.
static int setup_threads() {
    const unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(h == 0 ? 1u : h, 16u));
}

// Runs body(i) for i in [0, n) on up to setup_threads() threads, contiguous
// chunks of at least `grain` items (small loops stay on the calling thread,
// where starting threads would cost more than the work).
template <class F>
static void parallel_for(int64_t n, F body, int64_t grain = 1) {
    const int nt = (int)std::min<int64_t>(setup_threads(), std::max<int64_t>(n / std::max<int64_t>(grain, 1), 1));
    if (nt <= 1) {
        for (int64_t i = 0; i < n; ++i) body(i, 0);
        return;
    }
    std::vector<std::thread> pool;
    std::vector<std::exception_ptr> err(nt);
    for (int t = 0; t < nt; ++t)
        pool.emplace_back([&, t] {
            try {
                for (int64_t i = n * t / nt; i < n * (t + 1) / nt; ++i) body(i, t);
            } catch (...) {
                err[t] = std::current_exception();
            }
        });
    for (auto &th : pool) th.join();
    for (auto &e : err)
        if (e) std::rethrow_exception(e);
}

// ---------------------------------------------------------------- B-splines

std::vector<double> open_knots(int N, int q) {
    std::vector<double> kn;
    kn.reserve(N + 2 * q + 1);
    for (int i = 0; i <= q; ++i) kn.push_back(0.0);
    for (int e = 1; e < N; ++e) kn.push_back((double)e / N);
    for (int i = 0; i <= q; ++i) kn.push_back(1.0);
    return kn;
}

// Triangular evaluation of the Cox-de Boor recursion restricted to span s.
void span_basis(const std::vector<double> &kn, int q, int s, double x, double *val, double *der) {
    double cur[8], prev[8], lower[8];
    cur[0] = 1.0;
    for (int p = 1; p <= q; ++p) {
        for (int m = 0; m < p; ++m) prev[m] = cur[m];  // degree p-1, functions s-p+1+m
        if (p == q)
            for (int m = 0; m < p; ++m) lower[m] = prev[m];
        for (int m = 0; m <= p; ++m) {
            const int i = s - p + m;
            double v = 0.0;
            if (m >= 1) {
                const double d1 = kn[i + p] - kn[i];
                if (d1 > 0) v += (x - kn[i]) / d1 * prev[m - 1];
            }
            if (m <= p - 1) {
                const double d2 = kn[i + p + 1] - kn[i + 1];
                if (d2 > 0) v += (kn[i + p + 1] - x) / d2 * prev[m];
            }
            cur[m] = v;
        }
    }
    for (int m = 0; m <= q; ++m) val[m] = cur[m];
    if (!der) return;
    if (q == 0) {
        der[0] = 0.0;
        return;
    }
    for (int m = 0; m <= q; ++m) {
        const int i = s - q + m;
        double v = 0.0;
        if (m >= 1) {
            const double d1 = kn[i + q] - kn[i];
            if (d1 > 0) v += q / d1 * lower[m - 1];
        }
        if (m <= q - 1) {
            const double d2 = kn[i + q + 1] - kn[i + 1];
            if (d2 > 0) v -= q / d2 * lower[m];
        }
        der[m] = v;
    }
}

void gauss_legendre(int n, std::vector<double> &t, std::vector<double> &w) {
    t.resize(n);
    w.resize(n);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double p0 = 1.0, p1 = z, dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            p0 = 1.0;
            p1 = z;
            for (int j = 2; j <= n; ++j) {
                const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            dp = (n == 1) ? 1.0 : n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        p0 = 1.0;
        p1 = z;
        for (int j = 2; j <= n; ++j) {
            const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        dp = (n == 1) ? 1.0 : n * (z * p1 - p0) / (z * z - 1.0);
        t[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Sparse row: (column, value) pairs.
using SRow = std::vector<std::pair<int, double>>;

static SRow combine(double a, const SRow &x, double b, const SRow &y) {
    SRow out;
    size_t i = 0, j = 0;
    while (i < x.size() || j < y.size()) {
        if (j >= y.size() || (i < x.size() && x[i].first < y[j].first)) {
            out.push_back({x[i].first, a * x[i].second});
            ++i;
        } else if (i >= x.size() || y[j].first < x[i].first) {
            out.push_back({y[j].first, b * y[j].second});
            ++j;
        } else {
            out.push_back({x[i].first, a * x[i].second + b * y[j].second});
            ++i;
            ++j;
        }
    }
    return out;
}

// Boehm's algorithm: inserting knot t into span s (kn[s] <= t < kn[s+1]) maps
// control points P to Q with Q_i = P_i (i <= s-q), Q_i = P_{i-1} (i > s) and
// Q_i = a_i P_i + (1 - a_i) P_{i-1}, a_i = (t - kn[i]) / (kn[i+q] - kn[i]),
// otherwise.  Composing the insertions of all midpoints gives the map A from
// coarse to fine coefficients; the basis relation is its transpose.
Mat1 refinement_matrix(int Nc, int q) {
    std::vector<double> kn = open_knots(Nc, q);
    const int nc = Nc + q;
    std::vector<SRow> A(nc);
    for (int i = 0; i < nc; ++i) A[i] = {{i, 1.0}};
    for (int m = 0; m < Nc; ++m) {
        const double t = (2.0 * m + 1.0) / (2.0 * Nc);
        int s = q;
        while (!(kn[s] <= t && t < kn[s + 1])) ++s;
        const int n = (int)kn.size() - q - 1;
        std::vector<SRow> B(n + 1);
        for (int i = 0; i <= n; ++i) {
            if (i <= s - q) {
                B[i] = A[i];
            } else if (i >= s + 1) {
                B[i] = A[i - 1];
            } else {
                const double al = (t - kn[i]) / (kn[i + q] - kn[i]);
                B[i] = combine(al, A[i], 1.0 - al, A[i - 1]);
            }
        }
        A.swap(B);
        kn.insert(kn.begin() + s + 1, t);
    }
    const int nf = 2 * Nc + q;
    Mat1 T;
    T.init(nc, nf);
    for (int j = 0; j < nf; ++j)
        for (auto &e : A[j])
            if (std::fabs(e.second) > 1e-14) T(e.first, j) = e.second;
    return T;
}

// Xc = Tr X Tc^T
static Mat1 rap(const Mat1 &Tr, const Mat1 &X, const Mat1 &Tc) {
    std::vector<SRow> rr(Tr.nr), rc(Tc.nr);
    for (int i = 0; i < Tr.nr; ++i)
        for (int a = 0; a < Tr.nc; ++a)
            if (Tr(i, a) != 0.0) rr[i].push_back({a, Tr(i, a)});
    for (int i = 0; i < Tc.nr; ++i)
        for (int a = 0; a < Tc.nc; ++a)
            if (Tc(i, a) != 0.0) rc[i].push_back({a, Tc(i, a)});
    Mat1 Y;
    Y.init(X.nr, Tc.nr);
    for (int j = 0; j < Tc.nr; ++j)
        for (auto &e : rc[j])
            for (int a = 0; a < X.nr; ++a) {
                const double x = X(a, e.first);
                if (x != 0.0) Y(a, j) += x * e.second;
            }
    Mat1 Xc;
    Xc.init(Tr.nr, Tc.nr);
    for (int i = 0; i < Tr.nr; ++i)
        for (auto &e : rr[i])
            for (int j = 0; j < Tc.nr; ++j) {
                const double y = Y(e.first, j);
                if (y != 0.0) Xc(i, j) += e.second * y;
            }
    return Xc;
}

// ---------------------------------------------------------- 1D factor matrices

static void fine_factors(const Problem &pb, Factors &F) {
    const int N = pb.N, k = pb.k, nq = k + 3;
    const double h = 1.0 / N, CI = 4.0 * k;
    std::vector<double> t, wt;
    gauss_legendre(nq, t, wt);
    F.N = N;
    double v[8], dv[8], v0[8];
    for (int a = 0; a < 2; ++a) {
        const int q = k + a, n = N + q;
        const auto kn = open_knots(N, q);
        F.mass[a].init(n, n);
        F.stiff[a].init(n, n);
        F.dcol[a].init(n, n);
        F.xmass[a].init(n, n);
        F.nit[a].init(n, n);
        for (int e = 0; e < N; ++e)
            for (int g = 0; g < nq; ++g) {
                const double x = (e + 0.5 * (t[g] + 1.0)) * h, wq = 0.5 * h * wt[g];
                span_basis(kn, q, e + q, x, v, dv);
                for (int m1 = 0; m1 <= q; ++m1)
                    for (int m2 = 0; m2 <= q; ++m2) {
                        const int i = e + m1, j = e + m2;
                        F.mass[a](i, j) += wq * v[m1] * v[m2];
                        F.stiff[a](i, j) += wq * dv[m1] * dv[m2];
                        F.dcol[a](i, j) += wq * v[m1] * dv[m2];
                        F.xmass[a](i, j) += wq * (x - 0.5) * v[m1] * v[m2];
                    }
            }
        // Nitsche boundary terms at both ends: -n (N_i N_j' + N_i' N_j) + C_I/h N_i N_j
        for (int side = 0; side < 2; ++side) {
            const double x = side, nrm = side ? 1.0 : -1.0;
            const int s = side ? q + N - 1 : q;
            span_basis(kn, q, s, x, v, dv);
            for (int m1 = 0; m1 <= q; ++m1)
                for (int m2 = 0; m2 <= q; ++m2)
                    F.nit[a](s - q + m1, s - q + m2) +=
                        -nrm * (v[m1] * dv[m2] + dv[m1] * v[m2]) + CI / h * v[m1] * v[m2];
        }
    }
    if (pb.adv_kind == 2) {
        // weights s = sin^2(pi x) and s' = pi sin(2 pi x) of the manufactured
        // velocity's factors, by the same quadrature
        for (int a = 0; a < 2; ++a) {
            const int q = k + a, n = N + q;
            const auto kn = open_knots(N, q);
            for (int wi = 0; wi < 2; ++wi) {
                F.wmass[a][wi].init(n, n);
                F.wdcol[a][wi].init(n, n);
            }
            for (int e = 0; e < N; ++e)
                for (int g = 0; g < nq; ++g) {
                    const double x = (e + 0.5 * (t[g] + 1.0)) * h, wq = 0.5 * h * wt[g];
                    const double wv[2] = {std::sin(M_PI * x) * std::sin(M_PI * x), M_PI * std::sin(2.0 * M_PI * x)};
                    span_basis(kn, q, e + q, x, v, dv);
                    for (int wi = 0; wi < 2; ++wi)
                        for (int m1 = 0; m1 <= q; ++m1)
                            for (int m2 = 0; m2 <= q; ++m2) {
                                F.wmass[a][wi](e + m1, e + m2) += wq * wv[wi] * v[m1] * v[m2];
                                F.wdcol[a][wi](e + m1, e + m2) += wq * wv[wi] * v[m1] * dv[m2];
                            }
                }
        }
    }
    const auto kn1 = open_knots(N, k + 1), kn0 = open_knots(N, k);
    F.grad.init(N + k + 1, N + k);
    for (int e = 0; e < N; ++e)
        for (int g = 0; g < nq; ++g) {
            const double x = (e + 0.5 * (t[g] + 1.0)) * h, wq = 0.5 * h * wt[g];
            span_basis(kn1, k + 1, e + k + 1, x, v, dv);
            span_basis(kn0, k, e + k, x, v0, nullptr);
            for (int m1 = 0; m1 <= k + 1; ++m1)
                for (int m2 = 0; m2 <= k; ++m2) F.grad(e + m1, e + m2) += wq * dv[m1] * v0[m2];
        }
}

static void coarse_factors(const Factors &Ff, int k, Factors &Fc) {
    const int Nc = Ff.N / 2;
    Fc.N = Nc;
    Mat1 T[2] = {refinement_matrix(Nc, k), refinement_matrix(Nc, k + 1)};
    for (int a = 0; a < 2; ++a) {
        Fc.mass[a] = rap(T[a], Ff.mass[a], T[a]);
        Fc.stiff[a] = rap(T[a], Ff.stiff[a], T[a]);
        Fc.dcol[a] = rap(T[a], Ff.dcol[a], T[a]);
        Fc.xmass[a] = rap(T[a], Ff.xmass[a], T[a]);
        Fc.nit[a] = rap(T[a], Ff.nit[a], T[a]);
        for (int wi = 0; wi < 2; ++wi)
            if (Ff.wmass[a][wi].nr) {
                Fc.wmass[a][wi] = rap(T[a], Ff.wmass[a][wi], T[a]);
                Fc.wdcol[a][wi] = rap(T[a], Ff.wdcol[a][wi], T[a]);
            }
    }
    Fc.grad = rap(T[1], Ff.grad, T[0]);
}

// ----------------------------------------------------------- operator terms

// The manufactured velocity u = curl psi (2D psi = s(x) s(y); 3D psi = (g, 0,
// g), g = s(x) s(y) s(z), s(t) = sin^2(pi t)): component c is a sum of
// coef * prod_j s^(n_j)(x_j).
struct VelTerm {
    double c;
    int n[3];
};
static const std::vector<std::vector<VelTerm>> &velocity_terms(int d) {
    static const std::vector<std::vector<VelTerm>> u2 = {{{1.0, {0, 1, 0}}}, {{-1.0, {1, 0, 0}}}};
    static const std::vector<std::vector<VelTerm>> u3 = {
        {{1.0, {0, 1, 0}}}, {{1.0, {0, 0, 1}}, {-1.0, {1, 0, 0}}}, {{-1.0, {0, 1, 0}}}};
    return d == 2 ? u2 : u3;
}

struct FRef {
    const Mat1 *m = nullptr;
    bool tr = false;
    double get(int i, int j) const { return tr ? (*m)(j, i) : (*m)(i, j); }
};
struct Term {
    double coef;
    FRef f[3];
};

static std::vector<Term> make_terms(const Problem &pb, const Factors &F, int R, int C) {
    const int d = pb.d;
    std::vector<Term> T;
    auto idx = [&](int comp, int dir) { return (comp < d && dir == comp) ? 1 : 0; };
    if (R < d && C == R) {
        const int c = R;
        Term t{pb.sigma, {}};
        for (int j = 0; j < d; ++j) t.f[j] = {&F.mass[idx(c, j)], false};
        T.push_back(t);
        for (int e = 0; e < d; ++e) {
            Term s{pb.nu, {}}, n{pb.nu, {}};
            for (int j = 0; j < d; ++j) {
                s.f[j] = {j == e ? &F.stiff[idx(c, j)] : &F.mass[idx(c, j)], false};
                n.f[j] = {j == e ? &F.nit[idx(c, j)] : &F.mass[idx(c, j)], false};
            }
            T.push_back(s);
            T.push_back(n);
        }
        if (pb.adv_kind == 1) {
            // a = c (-(y - 1/2), x - 1/2[, 0]):  (v_c, a_x d_x u_c) + (v_c, a_y d_y u_c)
            Term ax{-pb.adv_c, {}}, ay{pb.adv_c, {}};
            ax.f[0] = {&F.dcol[idx(c, 0)], false};
            ax.f[1] = {&F.xmass[idx(c, 1)], false};
            ay.f[0] = {&F.xmass[idx(c, 0)], false};
            ay.f[1] = {&F.dcol[idx(c, 1)], false};
            if (d == 3) ax.f[2] = ay.f[2] = {&F.mass[idx(c, 2)], false};
            T.push_back(ax);
            T.push_back(ay);
        } else if (pb.adv_kind == 2) {
            // a = c u, u_j = sum of coef * prod_dir s^(n_dir)(x_dir), n in {0, 1}:
            // (v_c, a_j d_j u_c) = c coef x (weighted derivative integral in
            // direction j) x (weighted mass integrals in the others)
            for (int j = 0; j < d; ++j)
                for (const VelTerm &vt : velocity_terms(d)[j]) {
                    Term a{pb.adv_c * vt.c, {}};
                    for (int e = 0; e < d; ++e)
                        a.f[e] = {e == j ? &F.wdcol[idx(c, e)][vt.n[e]] : &F.wmass[idx(c, e)][vt.n[e]], false};
                    T.push_back(a);
                }
        }
    } else if (R < d && C == d) {
        Term t{-1.0, {}};  // -B
        for (int j = 0; j < d; ++j) t.f[j] = {j == R ? &F.grad : &F.mass[0], false};
        T.push_back(t);
    } else if (R == d && C < d) {
        Term t{1.0, {}};  // B^T
        for (int j = 0; j < d; ++j) t.f[j] = {j == C ? &F.grad : &F.mass[0], j == C};
        T.push_back(t);
    }
    return T;
}

// ------------------------------------------------------------ level storage

static void level_geometry(const Problem &pb, int N, HostLevel &L) {
    const int d = pb.d, k = pb.k;
    BlockGeom G{d, k};
    L.N = N;
    L.nblk = d + 1;
    L.off[0] = 0;
    for (int R = 0; R <= d; ++R) {
        int64_t rows = 1;
        for (int j = 0; j < 3; ++j) {
            L.nb[R][j] = (j < d) ? N + k - G.s(R, j) : 1;
            rows *= L.nb[R][j];
        }
        L.off[R + 1] = L.off[R] + rows;
    }
    L.n = L.off[d + 1];
    L.n_v = L.off[d];
    L.n_q = L.n - L.n_v;
}

// first stored column index of a row's box in one direction (see HostLevel)
static int box_start(bool win, int i, int lo, int W, int n) {
    return win ? std::min(std::max(i + lo, 0), n - W) : i + lo;
}

// Allocates the stencil-ELL values of a level and, on the unit square / cube,
// fills them from the Kronecker terms (a mapped domain's values come from
// assemble_mapped).
static void fill_matrix(const Problem &pb, const Factors &F, HostLevel &L) {
    const int d = pb.d;
    BlockGeom G{d, pb.k, pb.geometry != 0};
    // window layout when every box fits inside the grid in every direction
    L.win = true;
    for (int R = 0; R <= d; ++R)
        for (int C = 0; C <= d; ++C)
            if (G.coupled(R, C))
                for (int j = 0; j < d; ++j)
                    if (L.nb[C][j] < G.width(R, C, j)) L.win = false;
    int64_t tot = 0;
    for (int R = 0; R <= d; ++R) {
        int ns = 0;
        for (int C = 0; C <= d; ++C)
            if (G.coupled(R, C)) {
                int w = 1;
                for (int j = 0; j < d; ++j) w *= G.width(R, C, j);
                ns += w;
            }
        ns = (ns + kEllVec - 1) / kEllVec * kEllVec;
        L.nslots[R] = ns;
        L.val_off[R] = tot;
        tot += (L.off[R + 1] - L.off[R] + 63) / 64 * 64 * ns;  // slices of 64 rows
    }
    L.val_off[d + 1] = tot;
    L.val.assign(tot, 0.0);
    if (pb.geometry != 0) return;
    for (int R = 0; R <= d; ++R) {
        const int64_t rows = L.off[R + 1] - L.off[R];
        int slot0 = 0;
        int cs[4];
        const int ncs = G.order(R, cs);
        for (int ci = 0; ci < ncs; ++ci) {
            const int C = cs[ci];
            const auto terms = make_terms(pb, F, R, C);
            int W[3] = {1, 1, 1}, lo[3] = {0, 0, 0};
            for (int j = 0; j < d; ++j) {
                W[j] = G.width(R, C, j);
                lo[j] = G.lo(R, C, j);
            }
            // rows on the setup threads (each writes only its own slots)
            parallel_for(rows, [&](int64_t li, int) {
                int is[3], base[3] = {0, 0, 0};
                int64_t t = li;
                for (int j = 0; j < 3; ++j) {
                    is[j] = (int)(t % L.nb[R][j]);
                    t /= L.nb[R][j];
                    if (j < d) base[j] = box_start(L.win, is[j], lo[j], W[j], L.nb[C][j]);
                }
                int slot = slot0;
                for (int o2 = 0; o2 < W[2]; ++o2)
                    for (int o1 = 0; o1 < W[1]; ++o1)
                        for (int o0 = 0; o0 < W[0]; ++o0, ++slot) {
                            const int o[3] = {o0, o1, o2};
                            bool ok = true;
                            int itrue[3], jtrue[3];
                            for (int j = 0; j < d; ++j) {
                                const int js = base[j] + o[j];
                                if (js < 0 || js >= L.nb[C][j]) ok = false;
                                itrue[j] = is[j] + G.s(R, j);
                                jtrue[j] = js + G.s(C, j);
                            }
                            if (!ok) continue;
                            double v = 0.0;
                            for (auto &tm : terms) {
                                double p = tm.coef;
                                for (int j = 0; j < d; ++j) p *= tm.f[j].get(itrue[j], jtrue[j]);
                                v += p;
                            }
                            L.val[L.ell_index(R, li, slot)] = v;
                        }
            }, 2048);
            int w = 1;
            for (int j = 0; j < d; ++j) w *= W[j];
            slot0 += w;
        }
    }
}

static int block_of(const HostLevel &L, int64_t g) {
    int R = 0;
    while (R + 1 < L.nblk && g >= L.off[R + 1]) ++R;
    return R;
}

static double entry(const Problem &pb, const HostLevel &L, int64_t grow, int64_t gcol) {
    const int d = pb.d;
    BlockGeom G{d, pb.k, pb.geometry != 0};
    const int R = block_of(L, grow), C = block_of(L, gcol);
    if (!G.coupled(R, C)) return 0.0;
    int64_t a = grow - L.off[R], b = gcol - L.off[C];
    int slot = G.slot_base(R, C);
    int o[3] = {0, 0, 0}, W[3] = {1, 1, 1};
    for (int j = 0; j < 3; ++j) {
        const int is = (int)(a % L.nb[R][j]), js = (int)(b % L.nb[C][j]);
        a /= L.nb[R][j];
        b /= L.nb[C][j];
        if (j < d) {
            W[j] = G.width(R, C, j);
            o[j] = js - box_start(L.win, is, G.lo(R, C, j), W[j], L.nb[C][j]);
            if (o[j] < 0 || o[j] >= W[j]) return 0.0;
        }
    }
    slot += (o[2] * W[1] + o[1]) * W[0] + o[0];
    return L.val[L.ell_index(R, grow - L.off[R], slot)];
}

double level_entry(const Hierarchy &H, int level, int64_t grow, int64_t gcol) {
    return entry(H.pb, H.lv[level], grow, gcol);
}

// ------------------------------------------------------------- dense solves

// Inverse of an n x n matrix by Gaussian elimination with partial pivoting.
static void invert(int n, std::vector<double> &A, std::vector<double> &Ainv) {
    Ainv.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Ainv[(size_t)i * n + i] = 1.0;
    double scale = 0.0;
    for (double x : A) scale = std::max(scale, std::fabs(x));
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)p * n + c])) p = r;
        if (std::fabs(A[(size_t)p * n + c]) <= 1e-13 * scale) throw std::runtime_error("singular local system");
        if (p != c)
            for (int j = 0; j < n; ++j) {
                std::swap(A[(size_t)p * n + j], A[(size_t)c * n + j]);
                std::swap(Ainv[(size_t)p * n + j], Ainv[(size_t)c * n + j]);
            }
        const double inv = 1.0 / A[(size_t)c * n + c];
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = A[(size_t)r * n + c] * inv;
            if (f == 0.0) continue;
            for (int j = 0; j < n; ++j) {
                A[(size_t)r * n + j] -= f * A[(size_t)c * n + j];
                Ainv[(size_t)r * n + j] -= f * Ainv[(size_t)c * n + j];
            }
        }
    }
    for (int r = 0; r < n; ++r) {
        const double inv = 1.0 / A[(size_t)r * n + r];
        for (int j = 0; j < n; ++j) Ainv[(size_t)r * n + j] *= inv;
    }
}

// Bordered local system [[K_sub, e], [e^T, 0]], e = integrals of the local
// pressure functions (zero on velocity rows): row-major (n+1) x (n+1).
static void bordered_system(const Problem &pb, const HostLevel &L, const int32_t *dofs, int n,
                            std::vector<double> &A) {
    const int m = n + 1;
    A.assign((size_t)m * m, 0.0);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) A[(size_t)a * m + b] = entry(pb, L, dofs[a], dofs[b]);
    for (int a = 0; a < n; ++a) {
        const double e = dofs[a] >= L.n_v ? L.w[dofs[a] - L.n_v] : 0.0;
        A[(size_t)a * m + n] = e;
        A[(size_t)n * m + a] = e;
    }
}

// Leading n x n block of inv([[K_sub, e], [e^T, 0]]).
static void bordered_inverse(const Problem &pb, const HostLevel &L, const int32_t *dofs, int n, double *out) {
    const int m = n + 1;
    std::vector<double> A, Ai;
    bordered_system(pb, L, dofs, n, A);
    invert(m, A, Ai);
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) out[(size_t)a * n + b] = Ai[(size_t)a * m + b];
}

// ---------------------------------------------------------------- subdomains

static void build_patches(const Problem &pb, HostLevel &L, bool share) {
    const int d = pb.d, k = pb.k, N = L.N;
    BlockGeom G{d, k};
    // potential blocks: degree and true index range per direction
    struct PB {
        int q[3], lo[3], hi[3];
    };
    std::vector<PB> pots;
    if (d == 2) {
        PB p{};
        for (int j = 0; j < 3; ++j) {
            p.q[j] = (j < d) ? k + 1 : 0;
            p.lo[j] = (j < d) ? 1 : 0;
            p.hi[j] = (j < d) ? N + k : 1;
        }
        pots.push_back(p);
    } else {
        for (int o = 0; o < 3; ++o) {
            PB p{};
            for (int j = 0; j < 3; ++j) {
                p.q[j] = (j == o) ? k : k + 1;
                p.lo[j] = (j == o) ? 0 : 1;
                p.hi[j] = (j == o) ? N + k : N + k;
            }
            pots.push_back(p);
        }
    }
    L.pptr.assign(1, 0);
    L.pdofs.clear();
    L.color.clear();
    L.mcolor.clear();
    L.ppot.clear();
    for (int o = 0; o < (int)pots.size(); ++o) {
        const PB &p = pots[o];
        for (int a2 = p.lo[2]; a2 < p.hi[2]; ++a2)
            for (int a1 = p.lo[1]; a1 < p.hi[1]; ++a1)
                for (int a0 = p.lo[0]; a0 < p.hi[0]; ++a0) {
                    const int a[3] = {a0, a1, a2};
                    int e0[3] = {0, 0, 0}, e1[3] = {0, 0, 0};
                    for (int j = 0; j < d; ++j) {
                        e0[j] = std::max(0, a[j] - p.q[j]);
                        e1[j] = std::min(N - 1, a[j]);
                    }
                    for (int b = 0; b <= d; ++b) {
                        int r0[3] = {0, 0, 0}, r1[3] = {0, 0, 0};  // stored index range, inclusive
                        bool empty = false;
                        for (int j = 0; j < 3; ++j) {
                            if (j >= d) continue;
                            const int q = G.q(b, j), s = G.s(b, j);
                            const int lo = s, hi = N + k + (q - k) - s;  // true kept range [lo, hi)
                            int first = -1, last = -2;
                            for (int i = std::max(lo, e0[j]); i < std::min(hi, e1[j] + q + 1); ++i) {
                                const bool in = std::max(0, i - q) >= e0[j] && std::min(N - 1, i) <= e1[j];
                                if (in) {
                                    if (first < 0) first = i;
                                    last = i;
                                }
                            }
                            if (first < 0) {
                                empty = true;
                                break;
                            }
                            r0[j] = first - s;
                            r1[j] = last - s;
                        }
                        if (empty) continue;
                        for (int i2 = r0[2]; i2 <= r1[2]; ++i2)
                            for (int i1 = r0[1]; i1 <= r1[1]; ++i1)
                                for (int i0 = r0[0]; i0 <= r1[0]; ++i0)
                                    L.pdofs.push_back((int32_t)(L.off[b] + i0 +
                                                                (int64_t)L.nb[b][0] * (i1 + (int64_t)L.nb[b][1] * i2)));
                    }
                    L.pptr.push_back((int32_t)L.pdofs.size());
                    L.ppot.insert(L.ppot.end(), {o, a[0], a[1], a[2]});
                    int col = o;
                    for (int j = 0; j < d; ++j) col = col * (k + 1) + a[j] % (k + 1);
                    L.color.push_back(col);
                    // coupling-free colour: boxes of one colour and orientation
                    // are k+2 elements apart in some direction, so no basis
                    // function inside one overlaps one inside another
                    int mc = o;
                    for (int j = 0; j < d; ++j) mc = mc * (k + 2) + a[j] % (k + 2);
                    L.mcolor.push_back(mc);
                }
    }
    L.n_patch = (int64_t)L.pptr.size() - 1;
    L.moff.resize(L.n_patch);
    L.max_patch = 0;
    for (int64_t i = 0; i < L.n_patch; ++i) L.max_patch = std::max(L.max_patch, L.pptr[i + 1] - L.pptr[i]);
    L.M.clear();
    const int nthr = setup_threads();
    if (!share) {
        // one inverse per subdomain, stored in subdomain order; the subdomains
        // on the setup threads, each writing its own range
        std::vector<int64_t> off(L.n_patch + 1, 0);
        for (int64_t i = 0; i < L.n_patch; ++i) {
            const int64_t n = L.pptr[i + 1] - L.pptr[i];
            off[i + 1] = off[i] + n * n;
        }
        if (off[L.n_patch] > (int64_t)INT32_MAX) throw std::runtime_error("local inverse store exceeds 2^31 entries");
        L.M.assign((size_t)off[L.n_patch], 0.0);
        std::vector<std::vector<double>> As(nthr), Ais(nthr);
        parallel_for(L.n_patch, [&](int64_t i, int t) {
            const int n = L.pptr[i + 1] - L.pptr[i];
            bordered_system(pb, L, &L.pdofs[L.pptr[i]], n, As[t]);
            invert(n + 1, As[t], Ais[t]);
            double *out = L.M.data() + off[i];
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b) out[(size_t)a * n + b] = Ais[t][(size_t)a * (n + 1) + b];
            L.moff[i] = (int32_t)off[i];
        }, 128);
        L.n_class = L.n_patch;
    } else {
        // local inverses; subdomains whose bordered local systems agree to
        // rounding (translates of one another on a uniform grid with constant
        // coefficients) share one stored inverse.  The local systems and their
        // hashes are built on the setup threads, a chunk of subdomains at a
        // time; the classes are then found in subdomain order.
        struct Cls {
            int n;
            int32_t off;
            std::vector<double> A;
        };
        std::vector<Cls> classes;
        std::vector<std::vector<int>> bucket(1 << 16);
        std::vector<double> Ainv;
        const int64_t chunk = 8192;
        std::vector<std::vector<double>> As(chunk);
        std::vector<uint64_t> hs(chunk);
        std::vector<double> sc(chunk);
        for (int64_t c0 = 0; c0 < L.n_patch; c0 += chunk) {
            const int64_t c1 = std::min(L.n_patch, c0 + chunk);
            parallel_for(c1 - c0, [&](int64_t u, int) {
                const int64_t i = c0 + u;
                const int n = L.pptr[i + 1] - L.pptr[i];
                std::vector<double> &A = As[u];
                bordered_system(pb, L, &L.pdofs[L.pptr[i]], n, A);
                double scale = 0.0;
                for (double x : A) scale = std::max(scale, std::fabs(x));
                // hash of a coarse quantization: equal matrices land in one bucket
                uint64_t hsh = (uint64_t)n * 1469598103934665603ull;
                for (double x : A) hsh = (hsh ^ (uint64_t)(int64_t)std::llround(x / scale * 4096.0)) * 1099511628211ull;
                hs[u] = hsh;
                sc[u] = scale;
            }, 256);
            for (int64_t i = c0; i < c1; ++i) {
                const int64_t u = i - c0;
                const int n = L.pptr[i + 1] - L.pptr[i];
                std::vector<double> &A = As[u];
                const double scale = sc[u];
                const uint64_t hsh = hs[u];
                int found = -1;
                for (int c : bucket[hsh & 0xffff]) {
                    const Cls &C = classes[c];
                    if (C.n != n) continue;
                    double dmax = 0.0;
                    for (size_t t = 0; t < A.size(); ++t) dmax = std::max(dmax, std::fabs(A[t] - C.A[t]));
                    if (dmax <= 1e-14 * scale) {
                        found = c;
                        break;
                    }
                }
                if (found < 0) {
                    Cls C;
                    C.n = n;
                    C.off = (int32_t)L.M.size();
                    C.A = A;
                    invert(n + 1, A, Ainv);  // A is overwritten by the elimination
                    for (int a = 0; a < n; ++a)
                        for (int b = 0; b < n; ++b) L.M.push_back(Ainv[(size_t)a * (n + 1) + b]);
                    if (L.M.size() > (size_t)INT32_MAX) throw std::runtime_error("local inverse store exceeds 2^31 entries");
                    found = (int)classes.size();
                    bucket[hsh & 0xffff].push_back(found);
                    classes.push_back(std::move(C));
                }
                L.moff[i] = classes[found].off;
            }
        }
        L.n_class = (int64_t)classes.size();
    }
    // inverse map: for each DOF the delta positions of its (patch, row)
    // entries, patch ascending
    L.inv_ptr.assign(L.n + 1, 0);
    for (int32_t g : L.pdofs) L.inv_ptr[g + 1]++;
    for (int64_t g = 0; g < L.n; ++g) L.inv_ptr[g + 1] += L.inv_ptr[g];
    L.inv_pos.assign(L.pdofs.size(), 0);
    std::vector<int32_t> fillp(L.inv_ptr.begin(), L.inv_ptr.end() - 1);
    for (int64_t i = 0; i < L.n_patch; ++i)
        for (int32_t t = L.pptr[i]; t < L.pptr[i + 1]; ++t) L.inv_pos[fillp[L.pdofs[t]]++] = t;
    L.small_list.clear();
    L.big_ent.clear();
    for (int64_t i = 0; i < L.n_patch; ++i) {
        if (L.pptr[i + 1] - L.pptr[i] <= kSmallPatch) L.small_list.push_back((int32_t)i);
        else
            for (int32_t t = L.pptr[i]; t < L.pptr[i + 1]; ++t) L.big_ent.push_back(t);
    }
    // colour lists
    int ncol = 0;
    for (int c : L.color) ncol = std::max(ncol, c + 1);
    L.col_ptr.assign(ncol + 1, 0);
    for (int c : L.color) L.col_ptr[c + 1]++;
    for (int c = 0; c < ncol; ++c) L.col_ptr[c + 1] += L.col_ptr[c];
    L.col_list.assign(L.n_patch, 0);
    std::vector<int32_t> fc(L.col_ptr.begin(), L.col_ptr.end() - 1);
    for (int64_t i = 0; i < L.n_patch; ++i) L.col_list[fc[L.color[i]]++] = (int32_t)i;
}

// Lane table of the multiplicative sweep: per coupling-free colour (in
// colour order), its subdomains in ascending order packed into workgroups of
// kMultLanes threads (kMultLanesBig if a subdomain is larger), thread = one
// entry (subdomain, local row); a
// subdomain's entries take consecutive threads of one workgroup, a subdomain
// that does not fit the rest of a workgroup starts the next one, unused
// threads hold -1.
static void build_sweep_lanes(HostLevel &L) {
    int ncol = 0;
    for (int c : L.mcolor) ncol = std::max(ncol, c + 1);
    std::vector<std::vector<int32_t>> members(ncol);
    for (int64_t i = 0; i < L.n_patch; ++i) members[L.mcolor[i]].push_back((int32_t)i);
    L.mwave_ptr.assign(1, 0);
    L.mlane.clear();
    L.mstride.clear();
    const int B = L.max_patch <= kMultLanes ? kMultLanes : kMultLanesBig;
    if (L.max_patch > B) throw std::runtime_error("multiplicative Schwarz needs subdomains of at most 1024 DOFs");
    L.mwidth = B;
    // the most common subdomain size (the interior one): those subdomains go
    // interleaved, B / n of them per workgroup, so that the threads of a
    // wavefront hold the same local row of many subdomains, i.e. rows of one
    // block, and evaluate one row form
    std::vector<int64_t> count(B + 1, 0);
    for (int64_t i = 0; i < L.n_patch; ++i) count[L.pptr[i + 1] - L.pptr[i]]++;
    int nu = 0;
    for (int n = 1; n <= B; ++n)
        if (count[n] > (nu ? count[nu] : 0)) nu = n;
    const int S = nu > 0 && B % nu == 0 && B / nu >= 2 ? B / nu : 0;
    for (int c = 0; c < ncol; ++c) {
        std::vector<int32_t> inter, rest;
        for (int32_t p : members[c]) (S && L.pptr[p + 1] - L.pptr[p] == nu ? inter : rest).push_back(p);
        for (size_t q0 = 0; q0 < inter.size(); q0 += S) {
            const int Sw = (int)std::min<size_t>(S, inter.size() - q0);
            const size_t w0 = L.mlane.size();
            L.mlane.insert(L.mlane.end(), B, -1);
            for (int s = 0; s < Sw; ++s)
                for (int m = 0; m < nu; ++m) L.mlane[w0 + (size_t)m * Sw + s] = L.pptr[inter[q0 + s]] + m;
            L.mstride.push_back(Sw);
        }
        int fill = B;  // forces a new workgroup for the first consecutive subdomain
        for (int32_t p : rest) {
            const int n = L.pptr[p + 1] - L.pptr[p];
            if (fill + n > B) {
                L.mlane.insert(L.mlane.end(), B, -1);
                L.mstride.push_back(1);
                fill = 0;
            }
            const size_t w0 = L.mlane.size() - B;
            for (int m = 0; m < n; ++m) L.mlane[w0 + fill + m] = L.pptr[p] + m;
            fill += n;
        }
        L.mwave_ptr.push_back((int32_t)(L.mlane.size() / B));
    }
}


// ------------------------------------------- potential form (2D, FP32 cycle)

// derivative coefficients of the degree-q splines on N elements:
// (N_a)' = c_a N^{q-1}_{a-1} - c_{a+1} N^{q-1}_a with c_a = q / (xi_{a+q} - xi_a)
static std::vector<double> deriv_coef(int N, int q) {
    const auto kn = open_knots(N, q);
    std::vector<double> c(N + q, 0.0);
    for (int j = 0; j < N + q; ++j) {
        const double den = kn[j + q] - kn[j];
        c[j] = den > 0 ? q / den : 0.0;
    }
    return c;
}

// Entries of the 2D curl u = (d_y psi, -d_x psi) in the velocity row g:
// pairs (potential index, coefficient); potentials on the boundary are zero
// and skipped.
static void curl_row(const HostLevel &L, int k, const std::vector<double> &c, int64_t g,
                     std::vector<std::pair<int, double>> &out) {
    const int m = L.N + k - 1, nq = L.N + k;
    out.clear();
    auto add = [&](int pa, int pb, double v) {
        if (pa >= 1 && pa <= m && pb >= 1 && pb <= m) out.push_back({(pa - 1) + m * (pb - 1), v});
    };
    if (g < L.off[1]) {  // u_x(a, j) stored at (a - 1) + m j
        const int a = (int)(g % m) + 1, j = (int)(g / m);
        add(a, j + 1, c[j + 1]);
        add(a, j, -c[j + 1]);
    } else {  // u_y(i, b) stored at off[1] + i + nq (b - 1)
        const int64_t l = g - L.off[1];
        const int i = (int)(l % nq), b = (int)(l / nq) + 1;
        add(i + 1, b, -c[i + 1]);
        add(i, b, c[i + 1]);
    }
}

// Q = (C^T C)^{-1} C^T X for C (r x p, full column rank) and X (r x n),
// row-major, result p x n
static void left_solve(int r, int p, int n, const std::vector<double> &C, const double *X, std::vector<double> &Q) {
    std::vector<double> G((size_t)p * p, 0.0), Gi;
    for (int a = 0; a < p; ++a)
        for (int b = 0; b < p; ++b) {
            double s = 0.0;
            for (int t = 0; t < r; ++t) s += C[(size_t)t * p + a] * C[(size_t)t * p + b];
            G[(size_t)a * p + b] = s;
        }
    invert(p, G, Gi);
    std::vector<double> CtX((size_t)p * n, 0.0);
    for (int a = 0; a < p; ++a)
        for (int t = 0; t < r; ++t) {
            const double ca = C[(size_t)t * p + a];
            if (ca == 0.0) continue;
            for (int j = 0; j < n; ++j) CtX[(size_t)a * n + j] += ca * X[(size_t)t * n + j];
        }
    Q.assign((size_t)p * n, 0.0);
    for (int a = 0; a < p; ++a)
        for (int b = 0; b < p; ++b) {
            const double g = Gi[(size_t)a * p + b];
            for (int j = 0; j < n; ++j) Q[(size_t)a * n + j] += g * CtX[(size_t)b * n + j];
        }
}

// the inverse map of the local potentials (for each potential its beta
// entries, subdomain ascending) and the split into subdomains with a single
// local potential (one thread each) and the others
static void finish_potential_maps(HostLevel &L) {
    // for each potential the beta entries landing on it, subdomain ascending
    L.qinv_ptr.assign(L.n_psi + 1, 0);
    for (int32_t b : L.qpsi) L.qinv_ptr[b + 1]++;
    for (int64_t b = 0; b < L.n_psi; ++b) L.qinv_ptr[b + 1] += L.qinv_ptr[b];
    L.qinv_pos.assign(L.qpsi.size(), 0);
    std::vector<int32_t> fp(L.qinv_ptr.begin(), L.qinv_ptr.end() - 1);
    for (int64_t e = 0; e < (int64_t)L.qpsi.size(); ++e) L.qinv_pos[fp[L.qpsi[e]]++] = (int32_t)e;
    // one thread per small subdomain computes its single beta entry; every
    // other subdomain's entries go one per thread
    std::vector<int32_t> small;
    L.big_beta.clear();
    std::vector<char> is_small(L.n_patch, 0);
    for (int32_t p : L.small_list) {
        if (L.qptr[p + 1] - L.qptr[p] == 1) {
            small.push_back(p);
            is_small[p] = 1;
        } else {
            for (int32_t t = L.pptr[p]; t < L.pptr[p + 1]; ++t) L.big_ent.push_back(t);
        }
    }
    L.small_list = small;
    std::sort(L.big_ent.begin(), L.big_ent.end());
    for (int64_t i = 0; i < L.n_patch; ++i)
        if (!is_small[i])
            for (int32_t e = L.qptr[i]; e < L.qptr[i + 1]; ++e) L.big_beta.push_back(e);
}

static void build_potential_maps(const Problem &pb, HostLevel &L) {
    const int k = pb.k, q = k + 1, N = L.N, m = N + k - 1;
    L.n_psi = (int64_t)m * m;
    const auto c = deriv_coef(N, q);
    auto e0 = [&](int a) { return std::max(0, a - q); };
    auto e1 = [&](int a) { return std::min(N - 1, a); };
    L.qptr.assign(1, 0);
    L.qpsi.clear();
    L.qoff.clear();
    L.Q.clear();
    L.beta_row.clear();
    L.beta_patch.clear();
    std::vector<int> loc;
    std::vector<double> C, Qi;
    std::vector<std::pair<int, double>> row;
    std::vector<std::vector<int32_t>> qbucket(1 << 16);
    std::vector<std::pair<int64_t, int64_t>> qclass;  // (size, offset)
    for (int64_t i = 0; i < L.n_patch; ++i) {
        const int a0 = (int)(i % m) + 1, a1 = (int)(i / m) + 1;
        loc.clear();
        for (int b1 = std::max(1, a1 - q); b1 <= std::min(m, a1 + q); ++b1) {
            if (e0(b1) < e0(a1) || e1(b1) > e1(a1)) continue;
            for (int b0 = std::max(1, a0 - q); b0 <= std::min(m, a0 + q); ++b0) {
                if (e0(b0) < e0(a0) || e1(b0) > e1(a0)) continue;
                loc.push_back((b0 - 1) + m * (b1 - 1));
            }
        }
        const int np = (int)loc.size(), n = L.pptr[i + 1] - L.pptr[i];
        const int32_t *dofs = &L.pdofs[L.pptr[i]];
        int nv = 0;
        while (nv < n && dofs[nv] < L.n_v) ++nv;
        C.assign((size_t)nv * np, 0.0);
        for (int r = 0; r < nv; ++r) {
            curl_row(L, k, c, dofs[r], row);
            for (auto &e : row) {
                const auto it = std::find(loc.begin(), loc.end(), e.first);
                if (it != loc.end()) C[(size_t)r * np + (it - loc.begin())] += e.second;
            }
        }
        left_solve(nv, np, n, C, &L.M[L.moff[i]], Qi);
        // subdomains with equal maps (translates with a shared inverse) share
        // one stored copy
        double scale = 0.0;
        for (double x : Qi) scale = std::max(scale, std::fabs(x));
        uint64_t hsh = (uint64_t)(np * 64 + n) * 1469598103934665603ull;
        for (double x : Qi)
            hsh = (hsh ^ (uint64_t)(int64_t)std::llround(x / (scale > 0 ? scale : 1.0) * 4096.0)) * 1099511628211ull;
        int32_t off = -1;
        for (int32_t cand : qbucket[hsh & 0xffff]) {
            const auto &ci = qclass[cand];
            if (ci.first != (int64_t)Qi.size()) continue;
            double dmax = 0.0;
            for (size_t t = 0; t < Qi.size(); ++t) dmax = std::max(dmax, std::fabs(Qi[t] - L.Q[ci.second + t]));
            if (dmax <= 1e-14 * scale) {
                off = (int32_t)ci.second;
                break;
            }
        }
        if (off < 0) {
            off = (int32_t)L.Q.size();
            qbucket[hsh & 0xffff].push_back((int32_t)qclass.size());
            qclass.push_back({(int64_t)Qi.size(), (int64_t)off});
            L.Q.insert(L.Q.end(), Qi.begin(), Qi.end());
            if (L.Q.size() > (size_t)INT32_MAX) throw std::runtime_error("potential map store exceeds 2^31 entries");
        }
        L.qoff.push_back(off);
        for (int a = 0; a < np; ++a) {
            L.beta_row.push_back((int32_t)(off + (size_t)a * n));
            L.beta_patch.push_back((int32_t)i);
        }
        L.qpsi.insert(L.qpsi.end(), loc.begin(), loc.end());
        L.qptr.push_back((int32_t)L.qpsi.size());
    }
    finish_potential_maps(L);
}

// potential prolongation: Kronecker product of the 1D refinement of the
// degree-(k+1) splines without their end functions
static void build_potential_prolongation(const Problem &pb, const HostLevel &C, HostLevel &F) {
    const int k = pb.k;
    const Mat1 T = refinement_matrix(C.N, k + 1);
    const int mc = C.N + k - 1, mf = F.N + k - 1;
    std::vector<std::vector<std::pair<int, double>>> list(mf);
    for (int is = 0; is < mf; ++is)
        for (int jc = 0; jc < mc; ++jc) {
            const double v = T(jc + 1, is + 1);
            if (v != 0.0) list[is].push_back({jc, v});
        }
    F.Ps_rp.assign(1, 0);
    F.Ps_ci.clear();
    F.Ps_v.clear();
    for (int i1 = 0; i1 < mf; ++i1)
        for (int i0 = 0; i0 < mf; ++i0) {
            for (auto &y : list[i1])
                for (auto &x : list[i0]) {
                    F.Ps_ci.push_back((int32_t)(x.first + (int64_t)mc * y.first));
                    F.Ps_v.push_back(x.second * y.second);
                }
            F.Ps_rp.push_back((int32_t)F.Ps_ci.size());
        }
}

// coarse level: Q0 = (C^T C)^{-1} C^T Kinv[velocity rows]
static void build_coarse_potentials(const Problem &pb, HostLevel &L) {
    const int k = pb.k, m = L.N + k - 1;
    L.n_psi = (int64_t)m * m;
    const auto c = deriv_coef(L.N, k + 1);
    const int nv = (int)L.n_v, np = (int)L.n_psi, n = (int)L.n;
    std::vector<double> C((size_t)nv * np, 0.0);
    std::vector<std::pair<int, double>> row;
    for (int r = 0; r < nv; ++r) {
        curl_row(L, k, c, r, row);
        for (auto &e : row) C[(size_t)r * np + e.first] += e.second;
    }
    left_solve(nv, np, n, C, L.Kinv.data(), L.Q0);
}

// ---------------------------------------------- potential form (3D, FP32 cycle)
//
// Vector potential component o has degree k in direction o (all N + k
// functions kept) and k + 1 in the others (the two end functions removed:
// psi x n = 0); stored component after component, x fastest over the kept
// box.  u = curl psi:
//   u_x = d_y psi_z - d_z psi_y,  u_y = d_z psi_x - d_x psi_z,  u_z = d_x psi_y - d_y psi_x,
// with the derivative of a degree-(k+1) spline in degree-k splines as in
// deriv_coef.  Local maps use the pseudo-inverse of the local curl: near the
// boundary a subdomain's local potentials can contain gradients (the kernel
// of the curl), and the minimum-norm potentials of a local velocity
// correction are as good as any (only their curl enters the velocity).

struct PotBox {
    int lo[3], hi[3];
    int64_t off;
};

static void pot_boxes(int N, int k, PotBox b[3]) {
    int64_t off = 0;
    for (int o = 0; o < 3; ++o) {
        int64_t n = 1;
        for (int j = 0; j < 3; ++j) {
            b[o].lo[j] = j == o ? 0 : 1;
            b[o].hi[j] = N + k;
            n *= b[o].hi[j] - b[o].lo[j];
        }
        b[o].off = off;
        off += n;
    }
}

// storage index of potential (o, true index t), -1 outside the kept box
static int64_t pot_index(const PotBox &b, int t0, int t1, int t2) {
    const int t[3] = {t0, t1, t2};
    int64_t idx = 0, stride = 1;
    for (int j = 0; j < 3; ++j) {
        if (t[j] < b.lo[j] || t[j] >= b.hi[j]) return -1;
        idx += (int64_t)(t[j] - b.lo[j]) * stride;
        stride *= b.hi[j] - b.lo[j];
    }
    return b.off + idx;
}

// Entries of u = curl psi in velocity row g (3D): (potential index, coefficient)
static void curl_row3(const HostLevel &L, int k, const std::vector<double> &c, int64_t g,
                      std::vector<std::pair<int, double>> &out) {
    PotBox B[3];
    pot_boxes(L.N, k, B);
    out.clear();
    int R = 0;
    while (g >= L.off[R + 1]) ++R;
    int64_t l = g - L.off[R];
    int t[3];
    for (int j = 0; j < 3; ++j) {
        t[j] = (int)(l % L.nb[R][j]) + (j == R ? 1 : 0);
        l /= L.nb[R][j];
    }
    auto add = [&](int o, int a0, int a1, int a2, double v) {
        const int64_t i = pot_index(B[o], a0, a1, a2);
        if (i >= 0) out.push_back({(int)i, v});
    };
    // derivative in direction dir of component o at t: c (psi(t + e_dir) - psi(t))
    auto dpsi = [&](int o, int dir, double sign) {
        const double cc = sign * c[t[dir] + 1];
        int u[3] = {t[0], t[1], t[2]};
        u[dir] += 1;
        add(o, u[0], u[1], u[2], cc);
        add(o, t[0], t[1], t[2], -cc);
    };
    if (R == 0) {
        dpsi(2, 1, 1.0);
        dpsi(1, 2, -1.0);
    } else if (R == 1) {
        dpsi(0, 2, 1.0);
        dpsi(2, 0, -1.0);
    } else {
        dpsi(1, 0, 1.0);
        dpsi(0, 1, -1.0);
    }
}

// Pseudo-inverse of the symmetric positive semidefinite p x p matrix G
// (row-major) by cyclic Jacobi rotations: G = V diag(w) V^T, eigenvalues
// below 1e-12 max(w) are treated as zero.
static void sym_pinv(int p, std::vector<double> G, std::vector<double> &Gp) {
    std::vector<double> V((size_t)p * p, 0.0);
    for (int i = 0; i < p; ++i) V[(size_t)i * p + i] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < p; ++i)
            for (int j = 0; j < p; ++j)
                (i == j ? diag : off) += G[(size_t)i * p + j] * G[(size_t)i * p + j];
        if (off <= 1e-30 * diag) break;
        for (int a = 0; a < p - 1; ++a)
            for (int b = a + 1; b < p; ++b) {
                const double gab = G[(size_t)a * p + b];
                if (gab == 0.0) continue;
                const double gaa = G[(size_t)a * p + a], gbb = G[(size_t)b * p + b];
                const double th = 0.5 * (gbb - gaa) / gab;
                const double tt = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double cs = 1.0 / std::sqrt(tt * tt + 1.0), sn = tt * cs;
                for (int r = 0; r < p; ++r) {  // columns a, b
                    const double x = G[(size_t)r * p + a], y = G[(size_t)r * p + b];
                    G[(size_t)r * p + a] = cs * x - sn * y;
                    G[(size_t)r * p + b] = sn * x + cs * y;
                }
                for (int r = 0; r < p; ++r) {  // rows a, b
                    const double x = G[(size_t)a * p + r], y = G[(size_t)b * p + r];
                    G[(size_t)a * p + r] = cs * x - sn * y;
                    G[(size_t)b * p + r] = sn * x + cs * y;
                }
                for (int r = 0; r < p; ++r) {
                    const double x = V[(size_t)r * p + a], y = V[(size_t)r * p + b];
                    V[(size_t)r * p + a] = cs * x - sn * y;
                    V[(size_t)r * p + b] = sn * x + cs * y;
                }
            }
    }
    double wmax = 0.0;
    for (int i = 0; i < p; ++i) wmax = std::max(wmax, std::fabs(G[(size_t)i * p + i]));
    Gp.assign((size_t)p * p, 0.0);
    for (int e = 0; e < p; ++e) {
        const double w = G[(size_t)e * p + e];
        if (!(w > 1e-12 * wmax)) continue;
        for (int i = 0; i < p; ++i)
            for (int j = 0; j < p; ++j) Gp[(size_t)i * p + j] += V[(size_t)i * p + e] * V[(size_t)j * p + e] / w;
    }
}

// Q = (C^T C)^+ C^T X for C (r x p) and X (r x n), row-major, result p x n:
// the minimum-norm potentials whose curl is each column of X (which lies in
// the range of C)
static void pinv_solve(int r, int p, int n, const std::vector<double> &C, const double *X, std::vector<double> &Q) {
    std::vector<double> G((size_t)p * p, 0.0), Gp;
    for (int a = 0; a < p; ++a)
        for (int b = 0; b < p; ++b) {
            double s = 0.0;
            for (int t = 0; t < r; ++t) s += C[(size_t)t * p + a] * C[(size_t)t * p + b];
            G[(size_t)a * p + b] = s;
        }
    sym_pinv(p, G, Gp);
    std::vector<double> CtX((size_t)p * n, 0.0);
    for (int a = 0; a < p; ++a)
        for (int t = 0; t < r; ++t) {
            const double ca = C[(size_t)t * p + a];
            if (ca == 0.0) continue;
            for (int j = 0; j < n; ++j) CtX[(size_t)a * n + j] += ca * X[(size_t)t * n + j];
        }
    Q.assign((size_t)p * n, 0.0);
    for (int a = 0; a < p; ++a)
        for (int b = 0; b < p; ++b) {
            const double g = Gp[(size_t)a * p + b];
            if (g == 0.0) continue;
            for (int j = 0; j < n; ++j) Q[(size_t)a * n + j] += g * CtX[(size_t)b * n + j];
        }
}

// The velocity response X (r x n, velocity rows of a solution operator) to
// a load without pressure part (its first r columns) is divergence-free, so
// it must be a curl: C Q reproduces those columns (exactness of the local and
// global complexes).  A failure means a wrong curl or potential map.
static void check_curl_map(int r, int p, int n, const std::vector<double> &C, const std::vector<double> &Q,
                           const double *X, const char *what) {
    double scale = 0.0, err = 0.0;
    for (int t = 0; t < r; ++t)
        for (int j = 0; j < r; ++j) {
            double v = 0.0;
            for (int a = 0; a < p; ++a) v += C[(size_t)t * p + a] * Q[(size_t)a * n + j];
            scale = std::max(scale, std::fabs(X[(size_t)t * n + j]));
            err = std::max(err, std::fabs(v - X[(size_t)t * n + j]));
        }
    if (err > 1e-9 * std::max(scale, 1e-300))
        throw std::runtime_error(std::string(what) + ": velocity rows are not curls of the potentials (rel. err " +
                                 std::to_string(err / scale) + ")");
}

// local potentials of every 3D subdomain (the vector-potential functions of
// any component whose supports lie in it) and their maps Q_i
static void build_potential_maps_3d(const Problem &pb, HostLevel &L) {
    const int k = pb.k, N = L.N;
    PotBox B[3];
    pot_boxes(N, k, B);
    {
        int64_t n2 = 1;
        for (int j = 0; j < 3; ++j) n2 *= B[2].hi[j] - B[2].lo[j];
        L.n_psi = B[2].off + n2;
    }
    const auto c = deriv_coef(N, k + 1);
    auto qd = [&](int o, int j) { return j == o ? k : k + 1; };
    L.qptr.assign(1, 0);
    L.qpsi.clear();
    L.qoff.clear();
    L.Q.clear();
    L.beta_row.clear();
    L.beta_patch.clear();
    std::vector<std::vector<std::pair<int64_t, int64_t>>> qbucket(1 << 16);  // (size, offset) per hash
    // per subdomain: its potentials, the local curl C and the map Q_i built on
    // the setup threads, a chunk of subdomains at a time; the maps are then
    // stored (and shared where equal) in subdomain order
    const int64_t chunk = 4096;
    const int nthr = setup_threads();
    std::vector<std::vector<int>> locs(chunk);
    std::vector<std::vector<double>> Qis(chunk), Cs(nthr);
    std::vector<std::vector<std::pair<int, double>>> rows(nthr);
    std::vector<uint64_t> hs(chunk);
    std::vector<double> sc(chunk);
    for (int64_t c0 = 0; c0 < L.n_patch; c0 += chunk) {
        const int64_t c1 = std::min(L.n_patch, c0 + chunk);
        parallel_for(c1 - c0, [&](int64_t u, int t) {
            const int64_t i = c0 + u;
            const int o = L.ppot[4 * i], a[3] = {L.ppot[4 * i + 1], L.ppot[4 * i + 2], L.ppot[4 * i + 3]};
            int e0[3], e1[3];
            for (int j = 0; j < 3; ++j) {
                e0[j] = std::max(0, a[j] - qd(o, j));
                e1[j] = std::min(N - 1, a[j]);
            }
            std::vector<int> &loc = locs[u];
            loc.clear();
            for (int o2 = 0; o2 < 3; ++o2)
                for (int b2 = e0[2]; b2 <= e1[2] + qd(o2, 2); ++b2)
                    for (int b1 = e0[1]; b1 <= e1[1] + qd(o2, 1); ++b1)
                        for (int b0 = e0[0]; b0 <= e1[0] + qd(o2, 0); ++b0) {
                            const int b[3] = {b0, b1, b2};
                            bool in = true;
                            for (int j = 0; j < 3 && in; ++j)
                                in = std::max(0, b[j] - qd(o2, j)) >= e0[j] && std::min(N - 1, b[j]) <= e1[j];
                            if (!in) continue;
                            const int64_t idx = pot_index(B[o2], b0, b1, b2);
                            if (idx >= 0) loc.push_back((int)idx);
                        }
            const int np = (int)loc.size(), n = L.pptr[i + 1] - L.pptr[i];
            const int32_t *dofs = &L.pdofs[L.pptr[i]];
            int nv = 0;
            while (nv < n && dofs[nv] < L.n_v) ++nv;
            std::vector<double> &C = Cs[t];
            C.assign((size_t)nv * np, 0.0);
            for (int r = 0; r < nv; ++r) {
                curl_row3(L, k, c, dofs[r], rows[t]);
                for (auto &e : rows[t]) {
                    const auto it = std::find(loc.begin(), loc.end(), e.first);
                    if (it != loc.end()) C[(size_t)r * np + (it - loc.begin())] += e.second;
                }
            }
            std::vector<double> &Qi = Qis[u];
            pinv_solve(nv, np, n, C, &L.M[L.moff[i]], Qi);
            check_curl_map(nv, np, n, C, Qi, &L.M[L.moff[i]], "3D local potential map");
            double scale = 0.0;
            for (double x : Qi) scale = std::max(scale, std::fabs(x));
            uint64_t hsh = (uint64_t)(np * 64 + n) * 1469598103934665603ull;
            for (double x : Qi)
                hsh = (hsh ^ (uint64_t)(int64_t)std::llround(x / (scale > 0 ? scale : 1.0) * 4096.0)) * 1099511628211ull;
            hs[u] = hsh;
            sc[u] = scale;
        }, 16);
        for (int64_t i = c0; i < c1; ++i) {
            const int64_t u = i - c0;
            const std::vector<int> &loc = locs[u];
            const std::vector<double> &Qi = Qis[u];
            const int np = (int)loc.size(), n = L.pptr[i + 1] - L.pptr[i];
            const double scale = sc[u];
            const uint64_t hsh = hs[u];
            int32_t off = -1;
            for (const auto &ci : qbucket[hsh & 0xffff]) {
                if (ci.first != (int64_t)Qi.size()) continue;
                double dmax = 0.0;
                for (size_t t = 0; t < Qi.size(); ++t) dmax = std::max(dmax, std::fabs(Qi[t] - L.Q[ci.second + t]));
                if (dmax <= 1e-14 * scale) {
                    off = (int32_t)ci.second;
                    break;
                }
            }
            if (off < 0) {
                off = (int32_t)L.Q.size();
                qbucket[hsh & 0xffff].push_back({(int64_t)Qi.size(), (int64_t)off});
                L.Q.insert(L.Q.end(), Qi.begin(), Qi.end());
                if (L.Q.size() > (size_t)INT32_MAX) throw std::runtime_error("potential map store exceeds 2^31 entries");
            }
            L.qoff.push_back(off);
            for (int t = 0; t < np; ++t) {
                L.beta_row.push_back((int32_t)(off + (size_t)t * n));
                L.beta_patch.push_back((int32_t)i);
            }
            L.qpsi.insert(L.qpsi.end(), loc.begin(), loc.end());
            L.qptr.push_back((int32_t)L.qpsi.size());
        }
    }
    finish_potential_maps(L);
}

// 3D potential prolongation: per component the Kronecker product of the 1D
// refinements (degree k in direction o, all functions; degree k+1 without
// the end functions in the others)
static void build_potential_prolongation_3d(const Problem &pb, const HostLevel &C, HostLevel &F) {
    const int k = pb.k;
    const Mat1 T[2] = {refinement_matrix(C.N, k), refinement_matrix(C.N, k + 1)};
    PotBox Bc[3], Bf[3];
    pot_boxes(C.N, k, Bc);
    pot_boxes(F.N, k, Bf);
    F.Ps_rp.assign(1, 0);
    F.Ps_ci.clear();
    F.Ps_v.clear();
    for (int o = 0; o < 3; ++o) {
        // per direction: fine true index -> (coarse true index, coefficient)
        std::vector<std::vector<std::pair<int, double>>> list[3];
        for (int j = 0; j < 3; ++j) {
            const Mat1 &Tj = T[j == o ? 0 : 1];
            list[j].assign(Bf[o].hi[j], {});
            for (int tf = Bf[o].lo[j]; tf < Bf[o].hi[j]; ++tf)
                for (int tc = Bc[o].lo[j]; tc < Bc[o].hi[j]; ++tc) {
                    const double v = Tj(tc, tf);
                    if (v != 0.0) list[j][tf].push_back({tc, v});
                }
        }
        for (int t2 = Bf[o].lo[2]; t2 < Bf[o].hi[2]; ++t2)
            for (int t1 = Bf[o].lo[1]; t1 < Bf[o].hi[1]; ++t1)
                for (int t0 = Bf[o].lo[0]; t0 < Bf[o].hi[0]; ++t0) {
                    for (auto &z : list[2][t2])
                        for (auto &y : list[1][t1])
                            for (auto &x : list[0][t0]) {
                                F.Ps_ci.push_back((int32_t)pot_index(Bc[o], x.first, y.first, z.first));
                                F.Ps_v.push_back(x.second * y.second * z.second);
                            }
                    F.Ps_rp.push_back((int32_t)F.Ps_ci.size());
                }
    }
}

// 3D coarse level: Q0 = (C^T C)^+ C^T Kinv[velocity rows]
static void build_coarse_potentials_3d(const Problem &pb, HostLevel &L) {
    const int k = pb.k;
    PotBox B[3];
    pot_boxes(L.N, k, B);
    int64_t n2 = 1;
    for (int j = 0; j < 3; ++j) n2 *= B[2].hi[j] - B[2].lo[j];
    L.n_psi = B[2].off + n2;
    if (L.n_psi > 2000) throw std::runtime_error("3D FP32 refinement needs a coarsest grid of at most 2000 potentials");
    const auto c = deriv_coef(L.N, k + 1);
    const int nv = (int)L.n_v, np = (int)L.n_psi, n = (int)L.n;
    std::vector<double> C((size_t)nv * np, 0.0);
    std::vector<std::pair<int, double>> row;
    for (int r = 0; r < nv; ++r) {
        curl_row3(L, k, c, r, row);
        for (auto &e : row) C[(size_t)r * np + e.first] += e.second;
    }
    pinv_solve(nv, np, n, C, L.Kinv.data(), L.Q0);
    check_curl_map(nv, np, n, C, L.Q0, L.Kinv.data(), "3D coarse potential map");
}

// Fixed-width form of a CSR map with `rows` rows (see kEllMax): returns the
// width, 0 (nothing stored) when a row is longer than kEllMax.  val may be
// null (index maps).
static int to_ell(const std::vector<int32_t> &rp, const std::vector<int32_t> &ci, const std::vector<double> *val,
                  std::vector<int32_t> &eci, std::vector<double> *ev) {
    const int64_t rows = (int64_t)rp.size() - 1;
    int w = 0;
    for (int64_t i = 0; i < rows; ++i) w = std::max(w, rp[i + 1] - rp[i]);
    eci.clear();
    if (ev) ev->clear();
    if (w > kEllMax || rows <= 0) return 0;
    eci.assign((size_t)w * rows, -1);
    if (ev) ev->assign((size_t)w * rows, 0.0);
    for (int64_t i = 0; i < rows; ++i)
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            const size_t at = (size_t)(e - rp[i]) * rows + i;
            eci[at] = ci[e];
            if (ev) (*ev)[at] = (*val)[e];
        }
    return w;
}

// layout of smoother form 4 (see HostLevel), after the small list is final
static void finalize_small(HostLevel &L) {
    const int64_t ns = (int64_t)L.small_list.size();
    L.small_dofs.assign((size_t)kSmallPatch * ns, 0);
    std::vector<int64_t> pos(L.pdofs.size(), -1);
    for (int64_t q = 0; q < ns; ++q) {
        const int32_t p = L.small_list[q], base = L.pptr[p], nn = L.pptr[p + 1] - base;
        for (int c = 0; c < kSmallPatch; ++c) L.small_dofs[(size_t)c * ns + q] = L.pdofs[base + std::min(c, nn - 1)];
        for (int m = 0; m < nn; ++m) pos[base + m] = m * ns + q;
    }
    L.inv_pos4.resize(L.inv_pos.size());
    for (size_t e = 0; e < L.inv_pos.size(); ++e) {
        const int32_t t = L.inv_pos[e];
        const int64_t v = pos[t] >= 0 ? pos[t] : kSmallPatch * ns + t;
        if (v > INT32_MAX) throw std::runtime_error("correction buffer exceeds 2^31 entries");
        L.inv_pos4[e] = (int32_t)v;
    }
    std::vector<char> small(L.n_patch, 0);
    for (int32_t p : L.small_list) small[p] = 1;
    L.big_sub.clear();
    L.big_mesh.clear();
    L.max_big = 0;
    const bool pot = !L.qptr.empty();
    for (int32_t p = 0; p < (int32_t)L.n_patch; ++p) {
        if (small[p]) continue;
        const int nn = L.pptr[p + 1] - L.pptr[p];
        L.big_sub.push_back(p);
        L.big_mesh.insert(L.big_mesh.end(),
                          {L.pptr[p], nn, pot ? L.qptr[p] : 0, pot ? L.qptr[p + 1] - L.qptr[p] : 0});
        L.max_big = std::max(L.max_big, nn);
    }
    L.inv_w = to_ell(L.inv_ptr, L.inv_pos, nullptr, L.inv_ell, nullptr);
    if (L.inv_w) to_ell(L.inv_ptr, L.inv_pos4, nullptr, L.inv4_ell, nullptr);
    L.qinv_w = pot ? to_ell(L.qinv_ptr, L.qinv_pos, nullptr, L.qinv_ell, nullptr) : 0;
    L.P_w = to_ell(L.P_rp, L.P_ci, &L.P_v, L.P_eci, &L.P_ev);
    L.R_w = to_ell(L.R_rp, L.R_ci, &L.R_v, L.R_eci, &L.R_ev);
    L.Ps_w = pot ? to_ell(L.Ps_rp, L.Ps_ci, &L.Ps_v, L.Ps_eci, &L.Ps_ev) : 0;
}

// -------------------------------------------------------------- prolongation

static void build_prolongation(const Problem &pb, const HostLevel &C, HostLevel &F) {
    const int d = pb.d, k = pb.k;
    BlockGeom G{d, k};
    Mat1 T[2] = {refinement_matrix(C.N, k), refinement_matrix(C.N, k + 1)};
    F.P_rp.assign(1, 0);
    F.P_ci.clear();
    F.P_v.clear();
    for (int b = 0; b <= d; ++b) {
        // per direction: for each fine stored index, list of (coarse stored index, value)
        std::vector<std::vector<std::pair<int, double>>> lists[3];
        for (int j = 0; j < 3; ++j) {
            lists[j].resize(F.nb[b][j]);
            if (j >= d) {
                lists[j][0] = {{0, 1.0}};
                continue;
            }
            const int q = G.q(b, j), s = G.s(b, j);
            const Mat1 &Tq = T[q - k];
            for (int is = 0; is < F.nb[b][j]; ++is)
                for (int jc = 0; jc < C.nb[b][j]; ++jc) {
                    const double v = Tq(jc + s, is + s);
                    if (v != 0.0) lists[j][is].push_back({jc, v});
                }
        }
        for (int i2 = 0; i2 < F.nb[b][2]; ++i2)
            for (int i1 = 0; i1 < F.nb[b][1]; ++i1)
                for (int i0 = 0; i0 < F.nb[b][0]; ++i0) {
                    for (auto &z : lists[2][i2])
                        for (auto &y : lists[1][i1])
                            for (auto &x : lists[0][i0]) {
                                F.P_ci.push_back((int32_t)(C.off[b] + x.first +
                                                           (int64_t)C.nb[b][0] * (y.first + (int64_t)C.nb[b][1] * z.first)));
                                F.P_v.push_back(x.second * y.second * z.second);
                            }
                    F.P_rp.push_back((int32_t)F.P_ci.size());
                }
    }
    // transpose
    F.R_rp.assign(C.n + 1, 0);
    for (int32_t c : F.P_ci) F.R_rp[c + 1]++;
    for (int64_t i = 0; i < C.n; ++i) F.R_rp[i + 1] += F.R_rp[i];
    F.R_ci.assign(F.P_ci.size(), 0);
    F.R_v.assign(F.P_ci.size(), 0.0);
    std::vector<int32_t> fp(F.R_rp.begin(), F.R_rp.end() - 1);
    for (int64_t r = 0; r < F.n; ++r)
        for (int32_t e = F.P_rp[r]; e < F.P_rp[r + 1]; ++e) {
            const int32_t c = F.P_ci[e];
            F.R_ci[fp[c]] = (int32_t)r;
            F.R_v[fp[c]] = F.P_v[e];
            fp[c]++;
        }
}

static void pressure_integrals(const Problem &pb, HostLevel &L) {
    const int d = pb.d, k = pb.k;
    const auto kn = open_knots(L.N, k);
    const int n1 = L.N + k;
    std::vector<double> w1(n1);
    for (int j = 0; j < n1; ++j) w1[j] = (kn[j + k + 1] - kn[j]) / (k + 1);
    L.w.assign(L.n_q, 0.0);
    for (int64_t g = 0; g < L.n_q; ++g) {
        int64_t t = g;
        double v = 1.0;
        for (int j = 0; j < d; ++j) {
            v *= w1[t % n1];
            t /= n1;
        }
        L.w[g] = v;
    }
}


// slot of column (block C, stored index col) in row (block R, stored index
// row) of the stencil-ELL layout, -1 outside the stored box
static int stencil_slot(const HostLevel &L, const BlockGeom &G, int R, int C, int64_t row, int64_t col) {
    if (!G.coupled(R, C)) return -1;
    const int d = G.d;
    int slot = G.slot_base(R, C);
    int o[3] = {0, 0, 0}, W[3] = {1, 1, 1};
    for (int j = 0; j < 3; ++j) {
        const int is = (int)(row % L.nb[R][j]), js = (int)(col % L.nb[C][j]);
        row /= L.nb[R][j];
        col /= L.nb[C][j];
        if (j < d) {
            W[j] = G.width(R, C, j);
            o[j] = js - box_start(L.win, is, G.lo(R, C, j), W[j], L.nb[C][j]);
            if (o[j] < 0 || o[j] >= W[j]) return -1;
        }
    }
    return slot + (o[2] * W[1] + o[1]) * W[0] + o[0];
}

// Runs body(e0, e1, e2, thread) for every element of the N^d grid, colour by
// colour with colour (e mod (k+2)) per direction, the elements of a colour on
// the setup threads.  Two elements of one colour are k+2 apart in some
// direction and share no basis function (a function's support spans at most
// k+2 elements per direction), so bodies that add into the rows of their
// element's functions never collide, and every entry sums its elements in
// colour order whatever the thread count.
template <class F>
static void for_each_element_coloured(int d, int N, int k, F body) {
    const int stride = k + 2, ncol2 = d == 3 ? stride : 1;
    for (int c2 = 0; c2 < ncol2; ++c2)
        for (int c1 = 0; c1 < stride; ++c1)
            for (int c0 = 0; c0 < stride; ++c0) {
                const int n0 = (N - c0 + stride - 1) / stride, n1 = (N - c1 + stride - 1) / stride;
                const int n2 = d == 3 ? (N - c2 + stride - 1) / stride : 1;
                parallel_for((int64_t)n0 * n1 * n2, [&](int64_t i, int th) {
                    const int i0 = (int)(i % n0), i1 = (int)((i / n0) % n1), i2 = (int)(i / ((int64_t)n0 * n1));
                    body(c0 + stride * i0, c1 + stride * i1, c2 + stride * i2, th);
                }, 64);
            }
}

// ------------------------------------------- sparse Galerkin products (host)

// rows of a level operator (or of one of its terms) in CSR form, global
// indices of the level
struct Csr {
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> v;
};

// Rows 0 .. nrows-1 of the Galerkin product R A P on the coarser level
// (ncoarse DOFs), A in CSR over the finer level Fl, whose transfers R and P
// it uses; columns sorted.  Chunks of rows on the setup threads, each row
// summed in the same order whatever the chunking.
static Csr galerkin_rows(const HostLevel &Fl, const Csr &A, int64_t nrows, int64_t ncoarse) {
    const int nch = (int)std::max<int64_t>(1, std::min<int64_t>(setup_threads(), nrows / 2048));
    std::vector<Csr> part(nch);
    parallel_for(nch, [&](int64_t ch, int) {
        Csr &out = part[ch];
        std::vector<double> dense(ncoarse, 0.0);
        std::vector<char> mark(ncoarse, 0);
        std::vector<int32_t> touched;
        for (int64_t I = nrows * ch / nch; I < nrows * (ch + 1) / nch; ++I) {
            touched.clear();
            for (int32_t e1 = Fl.R_rp[I]; e1 < Fl.R_rp[I + 1]; ++e1) {
                const int32_t i = Fl.R_ci[e1];
                const double rv = Fl.R_v[e1];
                for (int64_t e2 = A.rp[i]; e2 < A.rp[i + 1]; ++e2) {
                    const int32_t j = A.ci[e2];
                    const double cv = rv * A.v[e2];
                    for (int32_t e3 = Fl.P_rp[j]; e3 < Fl.P_rp[j + 1]; ++e3) {
                        const int32_t J = Fl.P_ci[e3];
                        if (!mark[J]) {
                            mark[J] = 1;
                            touched.push_back(J);
                        }
                        dense[J] += cv * Fl.P_v[e3];
                    }
                }
            }
            std::sort(touched.begin(), touched.end());
            for (int32_t J : touched) {
                out.ci.push_back(J);
                out.v.push_back(dense[J]);
                dense[J] = 0.0;
                mark[J] = 0;
            }
            out.rp.push_back((int64_t)out.ci.size());  // row ends, local to the chunk
        }
    });
    Csr out;
    out.rp.assign(1, 0);
    for (auto &pc : part) {
        const int64_t base = (int64_t)out.ci.size();
        for (int64_t e : pc.rp) out.rp.push_back(base + e);
        out.ci.insert(out.ci.end(), pc.ci.begin(), pc.ci.end());
        out.v.insert(out.v.end(), pc.v.begin(), pc.v.end());
    }
    return out;
}

// Adds CSR rows 0 .. nrows-1 to the stored values of Lv (every entry must lie
// in the stored pattern).
static void csr_to_level(HostLevel &Lv, const BlockGeom &G, const Csr &Cm, int64_t nrows) {
    for (int64_t r = 0; r < nrows; ++r) {
        int R = 0;
        while (r >= Lv.off[R + 1]) ++R;
        for (int64_t e = Cm.rp[r]; e < Cm.rp[r + 1]; ++e) {
            const int64_t col = Cm.ci[e];
            int C = 0;
            while (col >= Lv.off[C + 1]) ++C;
            const int slot = stencil_slot(Lv, G, R, C, r - Lv.off[R], col - Lv.off[C]);
            if (slot < 0) throw std::runtime_error("Galerkin entry outside the stored pattern");
            Lv.val[Lv.ell_index(R, r - Lv.off[R], slot)] += Cm.v[e];
        }
    }
}

// Every stored non-zero of a level, CSR (columns in storage order per row).
static Csr level_csr(const HostLevel &L, const BlockGeom &G) {
    const int d = G.d;
    Csr out;
    out.rp.assign(1, 0);
    for (int R = 0; R <= d; ++R) {
        int cs[4];
        const int ncs = G.order(R, cs);
        const int64_t rows = L.off[R + 1] - L.off[R];
        for (int64_t li = 0; li < rows; ++li) {
            int is[3] = {0, 0, 0};
            int64_t tt = li;
            for (int j = 0; j < 3; ++j) {
                is[j] = (int)(tt % L.nb[R][j]);
                tt /= L.nb[R][j];
            }
            for (int ci = 0; ci < ncs; ++ci) {
                const int C = cs[ci];
                int W[3] = {1, 1, 1}, base[3] = {0, 0, 0};
                for (int j = 0; j < d; ++j) {
                    W[j] = G.width(R, C, j);
                    base[j] = box_start(L.win, is[j], G.lo(R, C, j), W[j], L.nb[C][j]);
                }
                int slot = G.slot_base(R, C);
                for (int o2 = 0; o2 < W[2]; ++o2)
                    for (int o1 = 0; o1 < W[1]; ++o1)
                        for (int o0 = 0; o0 < W[0]; ++o0, ++slot) {
                            const int o[3] = {o0, o1, o2};
                            int64_t col = 0, stride = 1;
                            bool ok = true;
                            for (int j = 0; j < d; ++j) {
                                const int js = base[j] + o[j];
                                if (js < 0 || js >= L.nb[C][j]) ok = false;
                                col += (int64_t)js * stride;
                                stride *= L.nb[C][j];
                            }
                            const double v = L.val[L.ell_index(R, li, slot)];
                            if (!ok || v == 0.0) continue;
                            out.ci.push_back((int32_t)(L.off[C] + col));
                            out.v.push_back(v);
                        }
            }
            out.rp.push_back((int64_t)out.ci.size());
        }
    }
    return out;
}

// ------------------------------------- advection by a field of the velocity space

// Advection by c times a field a of the finest velocity space (kind 3): the
// blocks (v_R, a . grad u_R) assembled by Gauss quadrature (k+3 points per
// direction per element) on the finest grid, and on the coarser grids their
// Galerkin products R C P through the prolongations (the operator's other
// terms keep their Kronecker factors; the Galerkin product is linear).  The
// terms are added to the stored values of every level.
static void add_field_advection(const Problem &pb, Hierarchy &H) {
    const int d = pb.d, k = pb.k, N = pb.N, nq = k + 3, L = pb.L;
    HostLevel &F = H.lv[L - 1];
    if ((int64_t)pb.adv_field.size() != F.n_v) throw std::runtime_error("advection field needs n_v coefficients");
    std::vector<double> t, wt;
    gauss_legendre(nq, t, wt);
    const double h = 1.0 / N;
    const auto kn0 = open_knots(N, k), kn1 = open_knots(N, k + 1);
    BlockGeom G{d, k};
    // the degree-k and degree-(k+1) functions and derivatives non-zero on each
    // element, at its quadrature points (the same in every direction)
    const int w0 = k + 1, w1 = k + 2;
    std::vector<double> tv0((size_t)N * nq * w0), td0(tv0.size()), tv1((size_t)N * nq * w1), td1(tv1.size());
    for (int e = 0; e < N; ++e)
        for (int g = 0; g < nq; ++g) {
            const double x = (e + 0.5 * (t[g] + 1.0)) * h;
            const size_t at = (size_t)e * nq + g;
            span_basis(kn0, k, e + k, x, &tv0[at * w0], &td0[at * w0]);
            span_basis(kn1, k + 1, e + k + 1, x, &tv1[at * w1], &td1[at * w1]);
        }
    // fine level: element matrices over the quadrature points, scattered
    // once per element into an array of the stencil-ELL shape
    std::vector<double> adv(F.val.size(), 0.0);
    const int G2 = d == 3 ? nq : 1;
    struct Fn {
        int64_t gidx;
        int m[3];
        int st[3];  // tensor index of the function in its block
    };
    // slot geometry of the same-component blocks (c, c)
    int Wc[3][3], loc_[3][3], sbase[3];
    for (int c = 0; c < d; ++c) {
        sbase[c] = G.slot_base(c, c);
        for (int jj = 0; jj < 3; ++jj) {
            Wc[c][jj] = jj < d ? G.width(c, c, jj) : 1;
            loc_[c][jj] = jj < d ? G.lo(c, c, jj) : 0;
        }
    }
    // elements colour by colour (see for_each_element_coloured): the threads
    // of a colour add to disjoint rows of adv
    for_each_element_coloured(d, N, k, [&](int e0, int e1, int e2, int) {
        double val[3][2][8], der[3][2][8];
        const int e[3] = {e0, e1, e2};
        // the functions of each velocity component non-zero on the element
        std::vector<Fn> fns[3];
        for (int c = 0; c < d; ++c) {
            int q[3] = {0, 0, 0};
            for (int jj = 0; jj < d; ++jj) q[jj] = G.q(c, jj);
            const int m2max = d == 3 ? q[2] : 0;
            for (int m2 = 0; m2 <= m2max; ++m2)
                for (int m1 = 0; m1 <= q[1]; ++m1)
                    for (int m0 = 0; m0 <= q[0]; ++m0) {
                        Fn f{0, {m0, m1, m2}, {0, 0, 0}};
                        int64_t idx = 0, stride = 1;
                        bool ok = true;
                        for (int jj = 0; jj < d; ++jj) {
                            const int st = e[jj] + f.m[jj] - G.s(c, jj);
                            if (st < 0 || st >= F.nb[c][jj]) ok = false;
                            f.st[jj] = st;
                            idx += (int64_t)st * stride;
                            stride *= F.nb[c][jj];
                        }
                        if (!ok) continue;
                        f.gidx = F.off[c] + idx;
                        fns[c].push_back(f);
                    }
        }
        std::vector<double> E[3];
        for (int c = 0; c < d; ++c) E[c].assign(fns[c].size() * fns[c].size(), 0.0);
        std::vector<double> fv[3], fdv[3];
        for (int c = 0; c < d; ++c) {  // every used entry is written at each point
            fv[c].assign(fns[c].size(), 0.0);
            fdv[c].assign(fns[c].size() * 3, 0.0);
        }
        for (int g2 = 0; g2 < G2; ++g2)
            for (int g1 = 0; g1 < nq; ++g1)
                for (int g0 = 0; g0 < nq; ++g0) {
                    const int g[3] = {g0, g1, g2};
                    double wq = 1.0;
                    for (int jj = 0; jj < d; ++jj) {
                        wq *= 0.5 * h * wt[g[jj]];
                        const size_t at = (size_t)e[jj] * nq + g[jj];
                        std::copy(&tv0[at * w0], &tv0[at * w0] + w0, val[jj][0]);
                        std::copy(&td0[at * w0], &td0[at * w0] + w0, der[jj][0]);
                        std::copy(&tv1[at * w1], &tv1[at * w1] + w1, val[jj][1]);
                        std::copy(&td1[at * w1], &td1[at * w1] + w1, der[jj][1]);
                    }
                    double a[3] = {0, 0, 0};
                    for (int c = 0; c < d; ++c) {
                        const size_t nf = fns[c].size();
                        for (size_t fi = 0; fi < nf; ++fi) {
                            const Fn &f = fns[c][fi];
                            double v = 1.0;
                            for (int jj = 0; jj < d; ++jj) v *= val[jj][G.q(c, jj) - k][f.m[jj]];
                            fv[c][fi] = v;
                            for (int dd = 0; dd < d; ++dd) {
                                double pp = 1.0;
                                for (int jj = 0; jj < d; ++jj)
                                    pp *= (jj == dd ? der : val)[jj][G.q(c, jj) - k][f.m[jj]];
                                fdv[c][fi * 3 + dd] = pp;
                            }
                            a[c] += pb.adv_field[f.gidx] * v;
                        }
                    }
                    for (int c = 0; c < d; ++c) a[c] *= pb.adv_c;
                    for (int c = 0; c < d; ++c) {
                        const size_t nf = fns[c].size();
                        for (size_t bj = 0; bj < nf; ++bj) {
                            double adv_b = 0.0;
                            for (int dd = 0; dd < d; ++dd) adv_b += a[dd] * fdv[c][bj * 3 + dd];
                            adv_b *= wq;
                            for (size_t ai = 0; ai < nf; ++ai) E[c][ai * nf + bj] += fv[c][ai] * adv_b;
                        }
                    }
                }
        for (int c = 0; c < d; ++c) {
            const size_t nf = fns[c].size();
            for (size_t ai = 0; ai < nf; ++ai) {
                const int64_t row = fns[c][ai].gidx - F.off[c];
                int base[3] = {0, 0, 0};
                for (int jj = 0; jj < d; ++jj)
                    base[jj] = box_start(F.win, fns[c][ai].st[jj], loc_[c][jj], Wc[c][jj], F.nb[c][jj]);
                for (size_t bj = 0; bj < nf; ++bj) {
                    // the slot of column function bj in row ai's box (as stencil_slot)
                    int o[3] = {0, 0, 0};
                    for (int jj = 0; jj < d; ++jj) {
                        o[jj] = fns[c][bj].st[jj] - base[jj];
                        if (o[jj] < 0 || o[jj] >= Wc[c][jj])
                            throw std::runtime_error("advection entry outside the stored pattern");
                    }
                    const int slot = sbase[c] + (o[2] * Wc[c][1] + o[1]) * Wc[c][0] + o[0];
                    adv[F.ell_index(c, row, slot)] += E[c][ai * nf + bj];
                }
            }
        }
    });
    // CSR of the fine advection (velocity rows, same-component columns, the
    // non-zeros of each row in slot order): counts per row, then the entries,
    // both passes with the rows on the setup threads
    const int64_t nvrow = F.off[d];
    auto scan_row = [&](int64_t r, auto &&emit) {
        int c = 0;
        while (r >= F.off[c + 1]) ++c;
        const int64_t li = r - F.off[c];
        int is[3] = {0, 0, 0}, base[3] = {0, 0, 0};
        int64_t tt = li;
        for (int jj = 0; jj < 3; ++jj) {
            is[jj] = (int)(tt % F.nb[c][jj]);
            tt /= F.nb[c][jj];
            if (jj < d) base[jj] = box_start(F.win, is[jj], loc_[c][jj], Wc[c][jj], F.nb[c][jj]);
        }
        int slot = 0;  // block (c, c) comes first in a velocity row
        for (int o2 = 0; o2 < Wc[c][2]; ++o2)
            for (int o1 = 0; o1 < Wc[c][1]; ++o1)
                for (int o0 = 0; o0 < Wc[c][0]; ++o0, ++slot) {
                    const int o[3] = {o0, o1, o2};
                    int64_t col = 0, stride = 1;
                    bool ok = true;
                    for (int jj = 0; jj < d; ++jj) {
                        const int js = base[jj] + o[jj];
                        if (js < 0 || js >= F.nb[c][jj]) ok = false;
                        col += (int64_t)js * stride;
                        stride *= F.nb[c][jj];
                    }
                    const double v = adv[F.ell_index(c, li, slot)];
                    if (!ok || v == 0.0) continue;
                    emit(F.off[c] + col, v);
                }
    };
    Csr cur;
    cur.rp.assign(nvrow + 1, 0);
    parallel_for(nvrow, [&](int64_t r, int) {
        int64_t m = 0;
        scan_row(r, [&](int64_t, double) { ++m; });
        cur.rp[r + 1] = m;
    }, 4096);
    for (int64_t r = 0; r < nvrow; ++r) cur.rp[r + 1] += cur.rp[r];
    cur.ci.assign(cur.rp[nvrow], 0);
    cur.v.assign(cur.rp[nvrow], 0.0);
    parallel_for(nvrow, [&](int64_t r, int) {
        int64_t at = cur.rp[r];
        scan_row(r, [&](int64_t col, double v) {
            cur.ci[at] = (int32_t)col;
            cur.v[at] = v;
            ++at;
        });
    }, 4096);
    for (size_t x = 0; x < adv.size(); ++x) F.val[x] += adv[x];
    adv.clear();
    adv.shrink_to_fit();
    // coarser levels: R C P (velocity rows only: R and P are block diagonal)
    for (int l = L - 1; l >= 1; --l) {
        Csr next = galerkin_rows(H.lv[l], cur, H.lv[l - 1].n_v, H.lv[l - 1].n);
        csr_to_level(H.lv[l - 1], G, next, H.lv[l - 1].n_v);
        cur = std::move(next);
    }
}

// ------------------------------------------------------------ mapped domains
//
// The quarter annulus x = r(xi_1) (cos theta(xi_2), sin theta(xi_2)), r =
// r_in + (r_out - r_in) xi_1, extruded to x_3 = depth xi_3 in 3D.  The
// quarter circle is the quadratic rational Bezier arc with weights 1,
// 1/sqrt(2), 1; a rational quadratic parametrization of a circle differs
// from the half-angle one by a Moebius map of the parameter, and the arc's
// symmetry about t = 1/2 fixes it: tan((theta - pi/4) / 2) = (2t - 1) tan(pi/8).
struct MapPoint {
    double J[3][3];      // J[i][m] = d x_i / d xi_m
    double dJ[3][3][3];  // dJ[q][i][m] = d^2 x_i / d xi_q d xi_m
};

static void annulus_point(const Problem &pb, const double *xi, MapPoint &m) {
    const double dr = pb.r_out - pb.r_in, r = pb.r_in + dr * xi[0];
    const double a = std::tan(M_PI / 8.0), u = (2.0 * xi[1] - 1.0) * a;
    const double th = M_PI / 4.0 + 2.0 * std::atan(u);
    const double t1 = 4.0 * a / (1.0 + u * u);
    const double t2 = -16.0 * a * a * u / ((1.0 + u * u) * (1.0 + u * u));
    const double er[2] = {std::cos(th), std::sin(th)}, et[2] = {-std::sin(th), std::cos(th)};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            m.J[i][j] = 0.0;
            for (int q = 0; q < 3; ++q) m.dJ[q][i][j] = 0.0;
        }
    for (int i = 0; i < 2; ++i) {
        m.J[i][0] = dr * er[i];
        m.J[i][1] = r * t1 * et[i];
        m.dJ[0][i][1] = dr * t1 * et[i];
        m.dJ[1][i][0] = dr * t1 * et[i];
        m.dJ[1][i][1] = r * (t2 * et[i] - t1 * t1 * er[i]);
    }
    m.J[2][2] = pb.depth;
}

static double det3(int d, const double (*J)[3]) {
    if (d == 2) return J[0][0] * J[1][1] - J[0][1] * J[1][0];
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

static void inv3(int d, const double (*J)[3], double det, double (*Ji)[3]) {
    if (d == 2) {
        Ji[0][0] = J[1][1] / det;
        Ji[0][1] = -J[0][1] / det;
        Ji[1][0] = -J[1][0] / det;
        Ji[1][1] = J[0][0] / det;
        return;
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int i1 = (j + 1) % 3, i2 = (j + 2) % 3, j1 = (i + 1) % 3, j2 = (i + 2) % 3;
            Ji[i][j] = (J[i1][j1] * J[i2][j2] - J[i1][j2] * J[i2][j1]) / det;  // cofactor transpose
        }
}

// Per point, the factors that give the physical value and gradient of a
// velocity basis function of component c (the contravariant Piola map v o F =
// J N e_c / det J): value_i = beta[c][i] N, gradient_ij = acoef[c][i][j] N +
// beta[c][i] (grad_x N)_j with (grad_x N)_j = sum_q d_q N Jinv[q][j].
struct Piola {
    double det, Jinv[3][3], beta[3][3], acoef[3][3][3];
};

static void piola_point(int d, const MapPoint &m, Piola &P) {
    P.det = det3(d, m.J);
    inv3(d, m.J, P.det, P.Jinv);
    double ddet[3] = {0, 0, 0};  // d det / d xi_q = det tr(Jinv dJ_q)
    for (int q = 0; q < d; ++q) {
        double tr = 0.0;
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) tr += P.Jinv[a][b] * m.dJ[q][b][a];
        ddet[q] = P.det * tr;
    }
    for (int c = 0; c < d; ++c)
        for (int i = 0; i < d; ++i) {
            P.beta[c][i] = m.J[i][c] / P.det;
            double al[3];
            for (int q = 0; q < d; ++q) al[q] = m.dJ[q][i][c] / P.det - m.J[i][c] * ddet[q] / (P.det * P.det);
            for (int j = 0; j < d; ++j) {
                double v = 0.0;
                for (int q = 0; q < d; ++q) v += al[q] * P.Jinv[q][j];
                P.acoef[c][i][j] = v;
            }
        }
}

// The finest operator on the mapped domain by Gauss quadrature (k+3 points
// per direction per element, faces likewise): sigma (v, u) + nu (grad v :
// grad u) + the Nitsche terms -nu (v, grad u n) - nu (grad v n, u) + C_I nu /
// h (v, u) with C_I = 4k, ds = det J |J^-T n_hat| and h = 1 / (N |J^-T
// n_hat|), and b(v, q) = (div v, q) = int div_x v q_hat dxi (the pressure
// pushed forward by q o F = q_hat / det J); coarser levels R K P.
//
// Per element the volume terms of the velocity block are a Gram matrix:
// with y_a the vector over points and components of sqrt(w det J) (sqrt(sigma)
// v_a, sqrt(nu) grad v_a), E_ab = y_a . y_b.  Elements are taken colour by
// colour, colour (e mod (k+2)) per direction: two elements of one colour are
// k+2 apart in some direction and share no basis function, so the threads of
// a colour scatter into disjoint rows (for_each_element_coloured).
static void assemble_mapped(const Problem &pb, Hierarchy &H) {
    const int d = pb.d, k = pb.k, N = pb.N, nq = k + 3, L = pb.L;
    BlockGeom G{d, k, true};
    HostLevel &F = H.lv[L - 1];
    std::vector<double> t, wt;
    gauss_legendre(nq, t, wt);
    const double h = 1.0 / N, CI = 4.0 * k;
    const double sqs = std::sqrt(pb.sigma), sqn = std::sqrt(pb.nu);
    const auto kn0 = open_knots(N, k), kn1 = open_knots(N, k + 1);
    const int npt = d == 3 ? nq * nq * nq : nq * nq;
    const int ncomp = d + d * d;      // value and gradient entries per point
    const int K = npt * ncomp;
    struct Fn {
        int blk;
        int64_t row;  // stored index in its block
        int m[3];
    };
    struct Work {
        std::vector<Fn> fns;
        std::vector<double> Vv, Tv, Qv, Y, Yd, Qp, E;
        double val[3][2][8], der[3][2][8];
    };
    const int nth = setup_threads();
    std::vector<Work> work(nth);
    // basis of the element's functions at parametric point xi: physical
    // values Vv (d per function), gradients Tv (d*d), pressure values Qv
    auto eval_point = [&](Work &w, const int *e, const double *xi, const Piola &P) {
        for (int j = 0; j < d; ++j) {
            span_basis(kn0, k, e[j] + k, xi[j], w.val[j][0], w.der[j][0]);
            span_basis(kn1, k + 1, e[j] + k + 1, xi[j], w.val[j][1], w.der[j][1]);
        }
        const size_t nf = w.fns.size();
        w.Vv.assign(nf * 3, 0.0);
        w.Tv.assign(nf * 9, 0.0);
        w.Qv.assign(nf, 0.0);
        for (size_t f = 0; f < nf; ++f) {
            const Fn &fn = w.fns[f];
            const int c = fn.blk;
            double nval = 1.0, dn[3];
            for (int j = 0; j < d; ++j) nval *= w.val[j][G.q(c, j) - k][fn.m[j]];
            if (c == d) {
                w.Qv[f] = nval;
                continue;
            }
            for (int q = 0; q < d; ++q) {
                double pp = 1.0;
                for (int j = 0; j < d; ++j) pp *= (j == q ? w.der : w.val)[j][G.q(c, j) - k][fn.m[j]];
                dn[q] = pp;
            }
            double gx[3];
            for (int j = 0; j < d; ++j) {
                gx[j] = 0.0;
                for (int q = 0; q < d; ++q) gx[j] += dn[q] * P.Jinv[q][j];
            }
            for (int i = 0; i < d; ++i) {
                w.Vv[f * 3 + i] = P.beta[c][i] * nval;
                for (int j = 0; j < d; ++j) w.Tv[f * 9 + i * 3 + j] = P.acoef[c][i][j] * nval + P.beta[c][i] * gx[j];
            }
        }
    };
    auto element = [&](int e0, int e1, int e2, Work &w) {
        const int e[3] = {e0, e1, e2};
        w.fns.clear();
        for (int c = 0; c <= d; ++c) {  // velocity functions first, then pressure
            int q[3] = {0, 0, 0};
            for (int j = 0; j < d; ++j) q[j] = G.q(c, j);
            for (int m2 = 0; m2 <= (d == 3 ? q[2] : 0); ++m2)
                for (int m1 = 0; m1 <= q[1]; ++m1)
                    for (int m0 = 0; m0 <= q[0]; ++m0) {
                        Fn f{c, 0, {m0, m1, m2}};
                        int64_t idx = 0, stride = 1;
                        bool ok = true;
                        for (int j = 0; j < d; ++j) {
                            const int st = e[j] + f.m[j] - G.s(c, j);
                            if (st < 0 || st >= F.nb[c][j]) ok = false;
                            idx += (int64_t)st * stride;
                            stride *= F.nb[c][j];
                        }
                        if (!ok) continue;
                        f.row = idx;
                        w.fns.push_back(f);
                    }
        }
        const size_t nf = w.fns.size();
        size_t nv = 0;
        while (nv < nf && w.fns[nv].blk < d) ++nv;
        const size_t np = nf - nv;
        w.Y.assign(nv * K, 0.0);
        w.Yd.assign(nv * npt, 0.0);
        w.Qp.assign(np * npt, 0.0);
        MapPoint mp;
        Piola P;
        double xi[3] = {0, 0, 0};
        int pt = 0;
        for (int g2 = 0; g2 < (d == 3 ? nq : 1); ++g2)
            for (int g1 = 0; g1 < nq; ++g1)
                for (int g0 = 0; g0 < nq; ++g0, ++pt) {
                    const int g[3] = {g0, g1, g2};
                    double wq = 1.0;
                    for (int j = 0; j < d; ++j) {
                        xi[j] = (e[j] + 0.5 * (t[g[j]] + 1.0)) * h;
                        wq *= 0.5 * h * wt[g[j]];
                    }
                    annulus_point(pb, xi, mp);
                    piola_point(d, mp, P);
                    eval_point(w, e, xi, P);
                    const double sw = std::sqrt(wq * P.det);
                    for (size_t a = 0; a < nv; ++a) {
                        double *y = &w.Y[a * K + (size_t)pt * ncomp];
                        double div = 0.0;
                        for (int i = 0; i < d; ++i) {
                            y[i] = sw * sqs * w.Vv[a * 3 + i];
                            for (int j = 0; j < d; ++j) y[d + i * d + j] = sw * sqn * w.Tv[a * 9 + i * 3 + j];
                            div += w.Tv[a * 9 + i * 3 + i];
                        }
                        w.Yd[a * npt + pt] = wq * div;
                    }
                    for (size_t p = 0; p < np; ++p) w.Qp[p * npt + pt] = w.Qv[nv + p];
                }
        w.E.assign(nf * nf, 0.0);
        for (size_t a = 0; a < nv; ++a) {
            const double *ya = &w.Y[a * K];
            for (size_t b = a; b < nv; ++b) {
                const double *yb = &w.Y[b * K];
                double acc = 0.0;
                for (int x = 0; x < K; ++x) acc += ya[x] * yb[x];
                w.E[a * nf + b] = acc;
                w.E[b * nf + a] = acc;
            }
            for (size_t p = 0; p < np; ++p) {
                // -(div v_a, q_p) in the velocity row, +(div v_a, q_p) in the pressure row
                const double *yd = &w.Yd[a * npt], *qp = &w.Qp[p * npt];
                double acc = 0.0;
                for (int x = 0; x < npt; ++x) acc += yd[x] * qp[x];
                w.E[a * nf + nv + p] = -acc;
                w.E[(nv + p) * nf + a] = acc;
            }
        }
        // boundary faces of this element (Nitsche terms)
        for (int fe = 0; fe < d; ++fe)
            for (int side = 0; side < 2; ++side) {
                if (e[fe] != (side ? N - 1 : 0)) continue;
                const int o1 = (fe + 1) % d, o2 = (fe + 2) % d;
                for (int g2 = 0; g2 < (d == 3 ? nq : 1); ++g2)
                    for (int g1 = 0; g1 < nq; ++g1) {
                        double wf = 0.5 * h * wt[g1];
                        xi[fe] = side ? 1.0 : 0.0;
                        xi[o1] = (e[o1] + 0.5 * (t[g1] + 1.0)) * h;
                        if (d == 3) {
                            xi[o2] = (e[o2] + 0.5 * (t[g2] + 1.0)) * h;
                            wf *= 0.5 * h * wt[g2];
                        }
                        annulus_point(pb, xi, mp);
                        piola_point(d, mp, P);
                        eval_point(w, e, xi, P);
                        // m = J^-T n_hat, n_hat = +-e_fe
                        const double sg = side ? 1.0 : -1.0;
                        double mv[3], ml = 0.0;
                        for (int i = 0; i < d; ++i) {
                            mv[i] = sg * P.Jinv[fe][i];
                            ml += mv[i] * mv[i];
                        }
                        ml = std::sqrt(ml);
                        double nrm[3];
                        for (int i = 0; i < d; ++i) nrm[i] = mv[i] / ml;
                        const double ds = wf * P.det * ml, hn = 1.0 / (N * ml);
                        for (size_t a = 0; a < nv; ++a) {
                            const double *va = &w.Vv[a * 3], *ta = &w.Tv[a * 9];
                            double tan_a[3];
                            for (int i = 0; i < d; ++i) {
                                tan_a[i] = 0.0;
                                for (int j = 0; j < d; ++j) tan_a[i] += ta[i * 3 + j] * nrm[j];
                            }
                            for (size_t b = 0; b < nv; ++b) {
                                const double *vb = &w.Vv[b * 3], *tb = &w.Tv[b * 9];
                                double s1 = 0.0, s2 = 0.0, s3 = 0.0;
                                for (int i = 0; i < d; ++i) {
                                    double tn_b = 0.0;
                                    for (int j = 0; j < d; ++j) tn_b += tb[i * 3 + j] * nrm[j];
                                    s1 += va[i] * tn_b;
                                    s2 += tan_a[i] * vb[i];
                                    s3 += va[i] * vb[i];
                                }
                                w.E[a * nf + b] += ds * (-pb.nu * s1 - pb.nu * s2 + CI * pb.nu / hn * s3);
                            }
                        }
                    }
            }
        for (size_t a = 0; a < nf; ++a)
            for (size_t b = 0; b < nf; ++b) {
                const double v = w.E[a * nf + b];
                if (v == 0.0) continue;
                const int slot = stencil_slot(F, G, w.fns[a].blk, w.fns[b].blk, w.fns[a].row, w.fns[b].row);
                if (slot < 0) throw std::runtime_error("mapped entry outside the stored pattern");
                F.val[F.ell_index(w.fns[a].blk, w.fns[a].row, slot)] += v;
            }
    };
    for_each_element_coloured(d, N, k, [&](int e0, int e1, int e2, int th) { element(e0, e1, e2, work[th]); });
    Csr cur = level_csr(F, G);
    for (int l = L - 1; l >= 1; --l) {
        Csr next = galerkin_rows(H.lv[l], cur, H.lv[l - 1].n, H.lv[l - 1].n);
        csr_to_level(H.lv[l - 1], G, next, H.lv[l - 1].n);
        cur = std::move(next);
    }
}

// 1D pressure mass bands of the divergence norm on the mapped domain: the
// weight 1 / det J = 1 / ((r_out - r_in) r(xi_1)) * 1 / theta'(xi_2) [* 1 /
// depth] separates, so the norm's mass is the tensor product of weighted 1D
// masses (same Gauss rule as the assembly).
static void mapped_pressure_mass(const Problem &pb, std::vector<double> &pm) {
    const int k = pb.k, N = pb.N, nq = k + 3, n1 = N + k, w = 2 * k + 1;
    std::vector<double> t, wt;
    gauss_legendre(nq, t, wt);
    const auto kn = open_knots(N, k);
    const double dr = pb.r_out - pb.r_in, a = std::tan(M_PI / 8.0);
    pm.assign((size_t)3 * n1 * w, 0.0);
    double val[8], der[8];
    for (int dir = 0; dir < 3; ++dir)
        for (int e = 0; e < N; ++e)
            for (int g = 0; g < nq; ++g) {
                const double x = (e + 0.5 * (t[g] + 1.0)) / N;
                double wgt = 0.5 * wt[g] / N;
                if (dir == 0) wgt /= dr * (pb.r_in + dr * x);
                else if (dir == 1) {
                    const double u = (2.0 * x - 1.0) * a;
                    wgt /= 4.0 * a / (1.0 + u * u);
                } else {
                    wgt /= pb.depth;
                }
                span_basis(kn, k, e + k, x, val, der);
                for (int i = 0; i <= k; ++i)
                    for (int j = 0; j <= k; ++j) {
                        const int gi = e + i, gj = e + j;  // pressure keeps every function
                        pm[((size_t)dir * n1 + gi) * w + (gj - gi) + k] += wgt * val[i] * val[j];
                    }
            }
}

void build_hierarchy(const Problem &pb, Hierarchy &H) {
    if (pb.d != 2 && pb.d != 3) throw std::runtime_error("dim must be 2 or 3");
    if (pb.k != 1 && pb.k != 2) throw std::runtime_error("k must be 1 or 2");
    if (pb.L < 1 || pb.N < 1) throw std::runtime_error("n_elem and n_levels must be positive");
    if (pb.N % (1 << (pb.L - 1)) != 0) throw std::runtime_error("n_elem must be divisible by 2^(n_levels-1)");
    if (!(pb.nu > 0.0) || !(pb.sigma >= 0.0)) throw std::runtime_error("need nu > 0 and sigma >= 0");
    if (pb.adv_kind < 0 || pb.adv_kind > 3) throw std::runtime_error("advection kind must be 0, 1, 2 or 3");
    if (pb.geometry != 0 && pb.geometry != 1) throw std::runtime_error("geometry must be 0 or 1");
    if (pb.geometry == 1) {
        if (pb.adv_kind != 0) throw std::runtime_error("mapped domains take generalized Stokes problems (advection 0)");
        if (!(pb.r_in > 0.0) || !(pb.r_out > pb.r_in) || (pb.d == 3 && !(pb.depth > 0.0)))
            throw std::runtime_error("need 0 < r_inner < r_outer and depth > 0");
    }
    H.pb = pb;
    const int L = pb.L;
    H.fac.assign(L, Factors());
    H.lv.assign(L, HostLevel());
    fine_factors(pb, H.fac[L - 1]);
    for (int l = L - 2; l >= 0; --l) coarse_factors(H.fac[l + 1], pb.k, H.fac[l]);
    for (int l = 0; l < L; ++l) {
        level_geometry(pb, H.fac[l].N, H.lv[l]);
        fill_matrix(pb, H.fac[l], H.lv[l]);
        pressure_integrals(pb, H.lv[l]);
    }
    for (int l = 1; l < L; ++l) build_prolongation(pb, H.lv[l - 1], H.lv[l]);
    if (pb.adv_kind == 3) add_field_advection(pb, H);
    if (pb.geometry == 1) assemble_mapped(pb, H);
    const bool share = pb.share_inverses && pb.adv_kind != 3 && pb.geometry == 0;
    for (int l = 1; l < L; ++l) build_patches(pb, H.lv[l], share);
    {
        HostLevel &C = H.lv[0];
        const int n = (int)C.n;
        std::vector<int32_t> all(n);
        for (int i = 0; i < n; ++i) all[i] = i;
        C.Kinv.assign((size_t)n * n, 0.0);
        bordered_inverse(pb, C, all.data(), n, C.Kinv.data());
    }
    if (pb.potentials) {
        if (pb.d == 2) {
            build_coarse_potentials(pb, H.lv[0]);
            for (int l = 1; l < L; ++l) {
                build_potential_maps(pb, H.lv[l]);
                build_potential_prolongation(pb, H.lv[l - 1], H.lv[l]);
            }
        } else {
            build_coarse_potentials_3d(pb, H.lv[0]);
            for (int l = 1; l < L; ++l) {
                build_potential_maps_3d(pb, H.lv[l]);
                build_potential_prolongation_3d(pb, H.lv[l - 1], H.lv[l]);
            }
        }
    }
    for (int l = 1; l < L; ++l) finalize_small(H.lv[l]);
    if (pb.multiplicative)
        for (int l = 1; l < L; ++l) build_sweep_lanes(H.lv[l]);
    // divergence norm data (finest grid)
    {
        const int k = pb.k, q = k + 1;
        const auto kn = open_knots(pb.N, q);
        const int n = pb.N + q;
        H.dcoef.assign(n, 0.0);
        for (int j = 0; j < n; ++j) {
            const double den = kn[j + q] - kn[j];
            H.dcoef[j] = den > 0 ? q / den : 0.0;
        }
        const Mat1 &Mq = H.fac[L - 1].mass[0];
        const int nq1 = pb.N + k, w = 2 * k + 1;
        if (pb.geometry == 1) {
            mapped_pressure_mass(pb, H.pmass);
        } else {
            H.pmass.assign((size_t)3 * nq1 * w, 0.0);
            for (int dir = 0; dir < 3; ++dir)
                for (int i = 0; i < nq1; ++i)
                    for (int o = -k; o <= k; ++o)
                        if (i + o >= 0 && i + o < nq1) H.pmass[((size_t)dir * nq1 + i) * w + o + k] = Mq(i, i + o);
        }
    }
    const double table[2][2] = {{0.35, 0.2}, {0.07, 0.02}};
    H.default_eta = table[pb.d - 2][pb.k - 1];
    {
        const int k = pb.k, N = pb.N, nq = k + 3, w = k + 2;
        std::vector<double> t, wt;
        gauss_legendre(nq, t, wt);
        H.qw.assign(nq, 0.0);
        for (int g = 0; g < nq; ++g) H.qw[g] = 0.5 * wt[g] / N;
        H.qbval.assign((size_t)2 * N * nq * w, 0.0);
        H.qbder.assign((size_t)2 * N * nq * w, 0.0);
        double v[8], dv[8];
        for (int a = 0; a < 2; ++a) {
            const int q = k + a;
            const auto kn = open_knots(N, q);
            for (int e = 0; e < N; ++e)
                for (int g = 0; g < nq; ++g) {
                    span_basis(kn, q, e + q, (e + 0.5 * (t[g] + 1.0)) / N, v, dv);
                    for (int m = 0; m <= q; ++m) {
                        const size_t at = (((size_t)a * N + e) * nq + g) * w + m;
                        H.qbval[at] = v[m];
                        H.qbder[at] = dv[m];
                    }
                }
        }
    }
}

// ------------------------------------------------------- manufactured forcing

static double sder(int n, double t) {
    const double pi = M_PI;
    switch (n) {
        case 0: return std::sin(pi * t) * std::sin(pi * t);
        case 1: return pi * std::sin(2 * pi * t);
        case 2: return 2 * pi * pi * std::cos(2 * pi * t);
        case 3: return -4 * pi * pi * pi * std::sin(2 * pi * t);
    }
    return 0.0;
}

// f = sigma u - nu Lap u + grad p + (a . grad) u at x for u = curl psi above.
static void forcing(const Problem &pb, const double *x, double *f) {
    const int d = pb.d;
    const double pi = M_PI;
    // velocity components as sums of c * prod_j s^{(n_j)}(x_j)
    const auto &U = velocity_terms(d);
    auto ev = [&](const std::vector<VelTerm> &terms, int dj, int dn) {
        double s = 0.0;
        for (auto &t : terms) {
            double p = t.c;
            for (int j = 0; j < d; ++j) p *= sder(t.n[j] + (j == dj ? dn : 0), x[j]);
            s += p;
        }
        return s;
    };
    double a[3] = {0, 0, 0};
    if (pb.adv_kind == 1) {
        a[0] = -pb.adv_c * (x[1] - 0.5);
        a[1] = pb.adv_c * (x[0] - 0.5);
    } else if (pb.adv_kind == 2) {
        for (int j = 0; j < d; ++j) a[j] = pb.adv_c * ev(U[j], -1, 0);
    }
    for (int c = 0; c < d; ++c) {
        double lap = 0.0, adv = 0.0;
        for (int j = 0; j < d; ++j) {
            lap += ev(U[c], j, 2);
            adv += a[j] * ev(U[c], j, 1);
        }
        double gp = 2 * pi;
        for (int j = 0; j < d; ++j) gp *= (j == c) ? std::cos(2 * pi * x[j]) : std::sin(2 * pi * x[j]);
        f[c] = pb.sigma * ev(U[c], -1, 0) - pb.nu * lap + gp + adv;
    }
}

double advection_speed(const Problem &pb) {
    if (pb.adv_kind == 1) return std::fabs(pb.adv_c) / std::sqrt(2.0);  // at the corners
    if (pb.adv_kind != 2) return 0.0;
    // max |u| of the manufactured velocity on a uniform sample grid, times |c|
    const int d = pb.d, m = d == 2 ? 400 : 80;
    const auto &U = velocity_terms(d);
    double best = 0.0;
    const int m2 = d == 3 ? m : 0;
    for (int i2 = 0; i2 <= m2; ++i2)
        for (int i1 = 0; i1 <= m; ++i1)
            for (int i0 = 0; i0 <= m; ++i0) {
                const double x[3] = {(double)i0 / m, (double)i1 / m, (double)i2 / m};
                double s2 = 0.0;
                for (int j = 0; j < d; ++j) {
                    double uj = 0.0;
                    for (const VelTerm &t : U[j]) {
                        double p = t.c;
                        for (int e = 0; e < d; ++e) p *= sder(t.n[e], x[e]);
                        uj += p;
                    }
                    s2 += uj * uj;
                }
                best = std::max(best, s2);
            }
    return std::fabs(pb.adv_c) * std::sqrt(best);
}

void manufactured_rhs(const Hierarchy &H, double *F) {
    const Problem &pb = H.pb;
    if (pb.geometry != 0) throw std::runtime_error("the manufactured load is defined on the unit square / cube");
    const HostLevel &L = H.lv[pb.L - 1];
    const int d = pb.d, k = pb.k, N = pb.N, nq = k + 3;
    BlockGeom G{d, k};
    std::vector<double> t, wt;
    gauss_legendre(nq, t, wt);
    std::fill(F, F + L.n, 0.0);
    const auto kn0 = open_knots(N, k), kn1 = open_knots(N, k + 1);
    const double h = 1.0 / N;
    const int E2 = d == 3 ? N : 1, G2 = d == 3 ? nq : 1;
    double val[3][2][8];  // [dir][degree index][m]
    for (int e2 = 0; e2 < E2; ++e2)
        for (int e1 = 0; e1 < N; ++e1)
            for (int e0 = 0; e0 < N; ++e0)
                for (int g2 = 0; g2 < G2; ++g2)
                    for (int g1 = 0; g1 < nq; ++g1)
                        for (int g0 = 0; g0 < nq; ++g0) {
                            const int e[3] = {e0, e1, e2}, g[3] = {g0, g1, g2};
                            double x[3] = {0, 0, 0}, wq = 1.0;
                            for (int j = 0; j < d; ++j) {
                                x[j] = (e[j] + 0.5 * (t[g[j]] + 1.0)) * h;
                                wq *= 0.5 * h * wt[g[j]];
                                span_basis(kn0, k, e[j] + k, x[j], val[j][0], nullptr);
                                span_basis(kn1, k + 1, e[j] + k + 1, x[j], val[j][1], nullptr);
                            }
                            double f[3];
                            forcing(pb, x, f);
                            for (int c = 0; c < d; ++c) {
                                int qd[3] = {0, 0, 0};
                                for (int j = 0; j < d; ++j) qd[j] = G.q(c, j) - k;
                                const int m2max = d == 3 ? k + qd[2] : 0;
                                for (int m2 = 0; m2 <= m2max; ++m2)
                                    for (int m1 = 0; m1 <= k + qd[1]; ++m1)
                                        for (int m0 = 0; m0 <= k + qd[0]; ++m0) {
                                            const int m[3] = {m0, m1, m2};
                                            int64_t idx = 0, stride = 1;
                                            bool ok = true;
                                            double phi = 1.0;
                                            for (int j = 0; j < d; ++j) {
                                                const int is = e[j] + m[j] - G.s(c, j);
                                                if (is < 0 || is >= L.nb[c][j]) ok = false;
                                                idx += is * stride;
                                                stride *= L.nb[c][j];
                                                phi *= val[j][qd[j]][m[j]];
                                            }
                                            if (ok) F[L.off[c] + idx] += wq * f[c] * phi;
                                        }
                            }
                        }
}

}  // namespace dfmg
