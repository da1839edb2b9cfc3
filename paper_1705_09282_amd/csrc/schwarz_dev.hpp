// Device pieces of the additive Schwarz smoother and the grid transfers
// (included by the per-level kernels and the single-workgroup coarse cycle).
// Every sum runs in a fixed order, so all kernels built from these pieces
// produce the same bits.
#pragma once

#include "device_util.hpp"

namespace dfmg {

// One row of M_p E_p r: m points at the row of the local inverse, dofs at the
// subdomain's nn DOFs.  Gathers are issued 8 at a time; the tail is padded
// with zero coefficients on a valid index, which leaves the sum unchanged.
template <class T>
__device__ __forceinline__ T patch_row(const T *m, const int32_t *dofs, int nn, const T *r) {
    T acc = 0;
    for (int c = 0; c < nn; c += 8) {
        int d[8];
        T mv[8], rv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const bool ok = c + u < nn;
            d[u] = dofs[ok ? c + u : c];
            mv[u] = ok ? m[c + u] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) rv[u] = r[d[u]];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fma(mv[u], rv[u], acc);
    }
    return acc;
}

// The residual entries of a subdomain of nn <= kSmallPatch DOFs (DOF c at
// dofs[c * dstride]), zero past nn.
template <class T>
__device__ __forceinline__ void gather_small(const int32_t *dofs, int64_t dstride, int nn, const T *r, T *rv) {
#pragma unroll
    for (int c = 0; c < kSmallPatch; ++c) rv[c] = c < nn ? r[dofs[c * dstride]] : T(0);
}

// Row m of M times the gathered entries: the same sum as patch_row.
template <class T>
__device__ __forceinline__ T small_row(const T *mrow, int nn, const T *rv) {
    T acc = 0;
#pragma unroll
    for (int c = 0; c < kSmallPatch; ++c)
        if (c < nn) acc = fma(mrow[c], rv[c], acc);
    return acc;
}

// Every row of M_p E_p r for a subdomain of nn <= kSmallPatch DOFs (m: its
// row-major inverse), row m written to delta[m * stride].  Same sums as
// patch_row.
template <class T>
__device__ __forceinline__ void apply_small(const T *m, int nn, const T *rv, T *delta, int64_t stride) {
    if (nn == kSmallPatch) {
#pragma unroll
        for (int row = 0; row < kSmallPatch; ++row) {
            T acc = 0;
#pragma unroll
            for (int c = 0; c < kSmallPatch; ++c) acc = fma(m[row * kSmallPatch + c], rv[c], acc);
            delta[row * stride] = acc;
        }
    } else {
        for (int row = 0; row < nn; ++row) delta[row * stride] = small_row(m + row * nn, nn, rv);
    }
}

// Every row of a small subdomain's M_p E_p r into delta[0 .. nn).
template <class T>
__device__ __forceinline__ void patch_small(const T *m, const int32_t *dofs, int nn, const T *r, T *delta) {
    T rv[kSmallPatch];
    gather_small(dofs, 1, nn, r, rv);
    apply_small(m, nn, rv, delta, 1);
}

// Sum of the corrections of every subdomain holding DOF j, in entry order.
template <class T>
__device__ __forceinline__ T dof_sum(const int32_t *inv_ptr, const int32_t *inv_pos, const T *delta, int j) {
    T acc = 0;
    const int e0 = inv_ptr[j], e1 = inv_ptr[j + 1];
    for (int e = e0; e < e1; e += 4) {
        int pos[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) pos[v] = inv_pos[e + v < e1 ? e + v : e];
        T dv[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) dv[v] = delta[pos[v]];
#pragma unroll
        for (int v = 0; v < 4; ++v) acc += (e + v < e1) ? dv[v] : T(0);
    }
    return acc;
}

// The same sum from the fixed-width map (W <= WB columns of `rows` rows, -1
// unused): every index load, then every correction load, is issued at once,
// so a DOF costs two dependent loads however many subdomains hold it.  All WB
// slots load unconditionally (slots past W re-read column W - 1, unused
// entries read delta[0]) and unused ones add zero: a branch around a load
// would make the compiler wait for that load before the next one.
template <int WB, class T>
__device__ __forceinline__ T ell_sum(const int32_t *ell, int64_t rows, int W, int64_t j, const T *delta) {
    int pos[WB];
#pragma unroll
    for (int w = 0; w < WB; ++w) {
        const int p = ell[(int64_t)(w < W ? w : W - 1) * rows + j];
        pos[w] = w < W ? p : -1;
    }
    T dv[WB];
#pragma unroll
    for (int w = 0; w < WB; ++w) dv[w] = delta[pos[w] >= 0 ? pos[w] : 0];
    T acc = 0;
#pragma unroll
    for (int w = 0; w < WB; ++w) acc += pos[w] >= 0 ? dv[w] : T(0);
    return acc;
}

// (A x)_i of a CSR matrix, gathers issued 4 at a time.
template <class T>
__device__ __forceinline__ T csr_row(const int32_t *rp, const int32_t *ci, const T *v, const T *x, int i) {
    T acc = 0;
    const int e0 = rp[i], e1 = rp[i + 1];
    for (int e = e0; e < e1; e += 4) {
        int col[4];
        T w[4], xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool ok = e + u < e1;
            col[u] = ci[ok ? e + u : e];
            w[u] = ok ? v[e + u] : T(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = x[col[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = fma(w[u], xv[u], acc);
    }
    return acc;
}

// The same row from the fixed-width form of A (W <= WB columns, index -1
// unused), loaded as in ell_sum: all indices and coefficients, then all
// gathers; unused slots read x[0] and add nothing.
template <int WB, class T>
__device__ __forceinline__ T ell_row(const int32_t *ci, const T *v, int64_t rows, int W, int64_t i, const T *x) {
    int col[WB];
    T w[WB];
#pragma unroll
    for (int u = 0; u < WB; ++u) {
        const int64_t at = (int64_t)(u < W ? u : W - 1) * rows + i;
        const int c = ci[at];
        const T wv = v[at];
        col[u] = u < W ? c : -1;
        w[u] = wv;
    }
    T xv[WB];
#pragma unroll
    for (int u = 0; u < WB; ++u) xv[u] = x[col[u] >= 0 ? col[u] : 0];
    T acc = 0;
#pragma unroll
    for (int u = 0; u < WB; ++u) acc = col[u] >= 0 ? fma(w[u], xv[u], acc) : acc;
    return acc;
}

// Row `row` of a dense FP64 matrix times x by one wavefront (lane-strided
// partial sums, then a shuffle tree); the result is valid in lane 0.
template <class T>
__device__ __forceinline__ double gemv_row_wave(const double *A, int cols, const T *x, int row, int lane) {
    double acc = 0.0;
    for (int j = lane; j < cols; j += 64) acc = fma(A[(int64_t)row * cols + j], (double)x[j], acc);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    return acc;
}

}  // namespace dfmg
