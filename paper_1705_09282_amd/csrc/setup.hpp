// Host-side construction of the multigrid hierarchy for the divergence-
// conforming B-spline discretization of generalized Stokes / Oseen problems
// on the unit square or cube.
//
// The fine-grid operator is a sum of tensor products of 1D factor matrices
// (mass, stiffness, first-derivative, (x - 1/2)-weighted mass, Nitsche
// boundary terms, and the derivative coupling of degree k+1 and k splines), so
// the Galerkin coarse operators K_l = R K_{l+1} P of the paper's nested
// hierarchy are obtained exactly by applying the 1D refinement matrices to
// every factor.  Matrices are stored in a sliced "stencil ELL" layout: for
// each row block (velocity component or pressure) and each coupled column
// block, every row holds the full box of tensor offsets in which two
// B-splines can overlap, values only (column indices follow from the offset).
// Rows are grouped in slices of 64 (one wavefront); inside a slice the values
// are slot-major, so a wavefront reads 64 consecutive values per slot and one
// contiguous block per slice.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "layout.hpp"

namespace dfmg {

struct Mat1 {
    int nr = 0, nc = 0;
    std::vector<double> a;
    void init(int r, int c) { nr = r; nc = c; a.assign((size_t)r * c, 0.0); }
    double &operator()(int i, int j) { return a[(size_t)i * nc + j]; }
    double operator()(int i, int j) const { return a[(size_t)i * nc + j]; }
};

// Open uniform knot vector of degree q on n elements of [0, 1].
std::vector<double> open_knots(int n_elem, int q);

// Values (and first derivatives) of the q+1 B-splines of degree q that are
// non-zero on knot span s, at x; val[j] belongs to function s-q+j.
void span_basis(const std::vector<double> &kn, int q, int s, double x, double *val, double *der);

// Gauss-Legendre nodes and weights on [-1, 1].
void gauss_legendre(int n, std::vector<double> &t, std::vector<double> &w);

// Refinement matrix T (n_coarse x n_fine) by Boehm knot insertion of every
// element midpoint: coarse N_i = sum_j T_ij fine N_j.
Mat1 refinement_matrix(int n_coarse_elem, int q);

// 1D factor matrices on one grid; index 0 = degree k, 1 = degree k+1.
struct Factors {
    int N = 0;
    Mat1 mass[2], stiff[2], dcol[2], xmass[2], nit[2];
    Mat1 grad;  // integral of (N^{k+1}_i)' N^k_j
    // advection by the manufactured velocity (kind 2): weighted mass
    // integral N_i w N_j and weighted derivative integral N_i w N_j' with
    // w = s (index 0) or s' (index 1), s(x) = sin^2(pi x), s' = pi sin(2 pi x)
    // (empty for the other kinds)
    Mat1 wmass[2][2], wdcol[2][2];
};

struct Problem {
    int d = 2, N = 0, L = 1, k = 1;
    double nu = 1.0, sigma = 1.0;
    // advection: 0 none; 1 rotation a = c (-(y - 1/2), x - 1/2[, 0]); 2 the
    // manufactured velocity, a = c u (the paper's Oseen problems); 3 c times
    // a field of the finest velocity space, coefficients adv_field (n_v, the
    // canonical velocity order)
    int adv_kind = 0;
    double adv_c = 0.0;
    std::vector<double> adv_field;
    // domain: 0 the unit square / cube; 1 the quarter annulus of radii r_in,
    // r_out (xi_1 radial, xi_2 the angle from the x axis), extruded along z by
    // depth in 3D (the hollow cylinder section).  On a mapped domain the
    // velocity rows couple every velocity component.
    int geometry = 0;
    double r_in = 0.075, r_out = 0.225, depth = 0.1;
    bool share_inverses = true;
    bool potentials = false;   // build the potential-form maps of the FP32 cycle
    bool multiplicative = false;  // build the lane tables of the multiplicative sweep
};

struct HostLevel {
    int N = 0;
    int nblk = 0;              // d + 1 blocks
    int nb[4][3] = {};         // stored count per block per direction
    int64_t off[5] = {};       // block offsets, off[nblk] = n
    int64_t n = 0, n_v = 0, n_q = 0;
    // stencil ELL: value (row, slot) of row block R at ell_index(R, row, slot):
    // slices of 64 rows, inside a slice chunks of kEllVec consecutive slots,
    // chunk-major, then row, then slot (one vector load per lane per chunk).
    // nslots[R] is the slot count rounded up to kEllVec (padding holds 0).
    // win: in every direction the stored box of a row is the window of W
    // consecutive column indices starting at clamp(i + lo, 0, n - W) (always
    // inside the grid, so the columns of a row need no clamping); otherwise
    // (a grid narrower than a box) slot o is column i + lo + o, 0 outside.
    std::vector<double> val;
    int64_t val_off[5] = {};
    int nslots[4] = {};
    bool win = false;
    int64_t ell_index(int R, int64_t row, int slot) const {
        return val_off[R] + (((row >> 6) * (nslots[R] / kEllVec) + slot / kEllVec) * 64 + (row & 63)) * kEllVec +
               slot % kEllVec;
    }
    std::vector<double> w;     // pressure basis integrals
    // subdomains (levels >= 1)
    int64_t n_patch = 0;
    std::vector<int32_t> pptr, pdofs, color, moff, inv_ptr, inv_pos;
    std::vector<double> M;     // local inverses, row-major n_i x n_i at moff
    int64_t n_class = 0;       // distinct stored inverses
    std::vector<int32_t> col_ptr, col_list;
    // multiplicative sweep: coupling-free colour per subdomain ((o, a mod
    // (k+2), ...) lexicographic), and per colour c the workgroups
    // mwave_ptr[c] .. mwave_ptr[c+1] of the lane table mlane (mwidth entry
    // indices per workgroup, -1 unused); in workgroup w, entry m of a
    // subdomain sits mstride[w] threads after entry m - 1 (1: a subdomain's
    // entries are consecutive; S: S subdomains of one size interleaved, local
    // row m of all of them on threads m S .. m S + S - 1); built with
    // Problem::multiplicative
    std::vector<int32_t> mcolor, mwave_ptr, mlane, mstride;
    // the potential of each subdomain: (orientation, true index x, y, z)
    std::vector<int32_t> ppot;
    int mwidth = 0;            // entries per workgroup of mlane
    // subdomains with <= kSmallPatch DOFs, and the entries of the others
    std::vector<int32_t> small_list, big_ent;
    // smoother form 4 keeps the corrections of small subdomain q, row m at
    // m * n_small + q (coalesced stores) and those of the other entries e at
    // kSmallPatch * n_small + e; small_dofs[c * n_small + q] is DOF c of small
    // subdomain q (kSmallPatch per subdomain, padded by repetition), and
    // inv_pos4 relabels inv_pos in that layout (same order).
    std::vector<int32_t> small_dofs, inv_pos4;
    // the subdomains outside small_list (one wavefront each in form 4):
    // big_sub[s] and big_mesh[4 s .. 4 s + 3] = (first entry pptr[p], size,
    // first beta entry qptr[p], number of local potentials; both 0 when the
    // potentials are not built); max_big = largest size
    std::vector<int32_t> big_sub, big_mesh;
    int max_big = 0;
    // fixed-width forms of inv_pos, inv_pos4 and qinv_pos (see kEllMax);
    // width 0: not stored
    int inv_w = 0, qinv_w = 0;
    std::vector<int32_t> inv_ell, inv4_ell, qinv_ell;
    // potential form of the FP32 cycle (2D): the streamfunction coefficient
    // (a, b), a, b in [1, N+k-1], is stored at (a-1) + (N+k-1)(b-1), the same
    // index as the subdomain that is its support.  Per subdomain i: its local
    // potentials qpsi[qptr[i] .. qptr[i+1]) (supports inside the subdomain)
    // and Q_i (row-major n_psi_i x n_i at qoff[i]), the left inverse of the
    // local curl applied to the velocity rows of M_i, so that Q_i E_i r are
    // the potential coefficients of the local velocity correction.
    int64_t n_psi = 0;
    std::vector<int32_t> qptr, qpsi, qoff, qinv_ptr, qinv_pos;
    std::vector<double> Q;
    std::vector<int32_t> big_beta;          // beta entries of subdomains outside small_list
    std::vector<int32_t> beta_row, beta_patch;  // per beta entry: Q row offset, subdomain
    // potential prolongation from level - 1 (rows: this level)
    std::vector<int32_t> Ps_rp, Ps_ci;
    std::vector<double> Ps_v;
    // coarse level: potential coefficients of the coarse velocity solution,
    // n_psi x n row-major
    std::vector<double> Q0;
    int max_patch = 0;
    // prolongation from level-1 (CSR, rows = this level) and restriction,
    // with their fixed-width forms (width 0: not stored); also of Ps
    std::vector<int32_t> P_rp, P_ci, R_rp, R_ci;
    std::vector<double> P_v, R_v;
    int P_w = 0, R_w = 0, Ps_w = 0;
    std::vector<int32_t> P_eci, R_eci, Ps_eci;
    std::vector<double> P_ev, R_ev, Ps_ev;
    // coarse level: leading n x n block of the bordered inverse
    std::vector<double> Kinv;
};

struct Hierarchy {
    Problem pb;
    std::vector<Factors> fac;
    std::vector<HostLevel> lv;
    // divergence-norm data on the finest grid
    std::vector<double> dcoef;     // derivative coefficients of degree k+1 splines
    std::vector<double> pmass;     // 1D pressure mass bands, one per direction (3 x n_q1 x (2k+1))
    double default_eta = 0.2;
    // quadrature tables of the finest grid (Crank-Nicolson / Adams-Bashforth
    // load): values and derivatives of the q+1 B-splines of degree q = k, k+1
    // non-zero on element e at its Gauss point g, [deg][e][g][m] with m < k+2;
    // per-direction weights (times h / 2)
    std::vector<double> qbval, qbder, qw;
};

// Build everything.  Throws std::runtime_error on invalid input.
void build_hierarchy(const Problem &pb, Hierarchy &H);

// Stencil-ELL helpers shared by setup and export.
struct BlockGeom {
    int d, k;
    bool xc = false;  // velocity rows couple every velocity component (mapped domain)
    int q(int R, int dir) const { return (R < d && dir == R) ? k + 1 : k; }
    int s(int R, int dir) const { return (R < d && dir == R) ? 1 : 0; }
    int lo(int R, int C, int dir) const { return s(R, dir) - s(C, dir) - q(R, dir); }
    int width(int R, int C, int dir) const { return q(R, dir) + q(C, dir) + 1; }
    bool coupled(int R, int C) const { return (R < d) ? (C == R || C == d || (xc && C < d)) : (C < d); }
    int box(int R, int C) const {
        int w = 1;
        for (int j = 0; j < d; ++j) w *= width(R, C, j);
        return w;
    }
    // column blocks of row block R in storage order: a velocity row stores
    // its own component, the pressure, then (xc) the other components in
    // increasing order; a pressure row the velocity components in order
    int order(int R, int *cs) const {
        int n = 0;
        if (R < d) {
            cs[n++] = R;
            cs[n++] = d;
            if (xc)
                for (int C = 0; C < d; ++C)
                    if (C != R) cs[n++] = C;
        } else {
            for (int C = 0; C < d; ++C) cs[n++] = C;
        }
        return n;
    }
    // first slot of block (R, C) in a row of block R
    int slot_base(int R, int C) const {
        int cs[4];
        const int n = order(R, cs);
        int s0 = 0;
        for (int i = 0; i < n && cs[i] != C; ++i) s0 += box(R, cs[i]);
        return s0;
    }
};

// Entry K(g_row, g_col) of a level (0 if outside the stored pattern).
double level_entry(const Hierarchy &H, int level, int64_t grow, int64_t gcol);

// max |a| over the domain (rotation: at the corners; manufactured velocity:
// on a uniform sample grid).
double advection_speed(const Problem &pb);

// Manufactured load vector on the finest grid.
void manufactured_rhs(const Hierarchy &H, double *F);

}  // namespace dfmg
