// Device pieces of the residual r = F - K U in the stencil-ELL layout
// (included by the residual kernel and the single-workgroup coarse cycle).
#pragma once

#include "device_util.hpp"
#include "layout.hpp"

namespace dfmg {

template <int D, int K>
struct Geo {
    __host__ __device__ static constexpr int q(int R, int dir) { return (R < D && dir == R) ? K + 1 : K; }
    __host__ __device__ static constexpr int s(int R, int dir) { return (R < D && dir == R) ? 1 : 0; }
    __host__ __device__ static constexpr int lo(int R, int C, int dir) {
        return dir < D ? s(R, dir) - s(C, dir) - q(R, dir) : 0;
    }
    __host__ __device__ static constexpr int w(int R, int C, int dir) {
        return dir < D ? q(R, dir) + q(C, dir) + 1 : 1;
    }
};

// Offset of slot s from a row's slot 0 in the sliced, chunked layout (chunks
// of kEll consecutive slots; a chunk of one row is kEll consecutive values).
constexpr int kEll = kEllVec;
__host__ __device__ constexpr int slot_off(int s) { return (s / kEll) * (64 * kEll) + s % kEll; }

// Contribution of column block C to row (i0, i1, i2) of row block R.  The
// box of column offsets is walked as W2*W1 "stencil rows" of W0 consecutive
// x-offsets; with LPR lanes per matrix row, lane l takes stencil rows
// l, l + LPR, ...  WIN: the stored box starts at the clamped window origin
// and lies inside the grid (no per-slot clamping, x-offsets become constant
// address offsets); otherwise slots outside the grid hold 0 and read a
// clamped (valid) vector entry.  vp points at slot 0 of the row, s0 is the
// first slot of this block.  NT: the values are loaded non-temporally (read
// once per launch; used where a level's values far exceed the Infinity Cache,
// so that they stream past the caches that hold the vector).
template <int D, int K, int R, int C, int LPR, bool WIN, class T, bool NT = false>
__device__ __forceinline__ T block_dot(const SpmvArgsT<T> &a, int i0, int i1, int i2, int lane, const T *vp,
                                       int s0) {
    using G = Geo<D, K>;
    constexpr int W0 = G::w(R, C, 0), W1 = G::w(R, C, 1), W2 = G::w(R, C, 2);
    constexpr int L0 = G::lo(R, C, 0), L1 = G::lo(R, C, 1), L2 = G::lo(R, C, 2);
    constexpr int NS = W1 * W2;
    const T *Uc = a.U + a.off[C];
    const int n0 = a.nb[C][0], n1 = a.nb[C][1], n2 = a.nb[C][2];
    const int b0 = WIN ? clampi(i0 + L0, 0, n0 - W0) : i0 + L0;
    const int b1 = WIN ? clampi(i1 + L1, 0, n1 - W1) : i1 + L1;
    const int b2 = (D == 3) ? (WIN ? clampi(i2 + L2, 0, n2 - W2) : i2 + L2) : 0;
    T acc = 0;
#pragma unroll
    for (int it = 0; it < (NS + LPR - 1) / LPR; ++it) {
        const int sr = it * LPR + lane;
        if (LPR > 1 && sr >= NS) break;
        const int o1 = sr % W1, o2 = sr / W1;
        const int j2 = (D == 3) ? (WIN ? b2 + o2 : clampi(b2 + o2, 0, n2 - 1)) : 0;
        const int j1 = WIN ? b1 + o1 : clampi(b1 + o1, 0, n1 - 1);
        const T *urow = Uc + ((int64_t)j2 * n1 + j1) * n0 + (WIN ? b0 : 0);
#pragma unroll
        for (int o0 = 0; o0 < W0; ++o0) {
            const int j0 = WIN ? o0 : clampi(b0 + o0, 0, n0 - 1);
            const T *vq = vp + slot_off(s0 + sr * W0 + o0);
            acc = fma(NT ? __builtin_nontemporal_load(vq) : *vq, urow[j0], acc);
        }
    }
    return acc;
}

template <int D, int K, int R, int C>
__host__ __device__ constexpr int block_slots() {
    return Geo<D, K>::w(R, C, 0) * Geo<D, K>::w(R, C, 1) * Geo<D, K>::w(R, C, 2);
}

// Velocity rows of a mapped domain (XC) also couple the other velocity
// components: their blocks follow (R, R) and (R, D), in increasing order of
// the component.
template <int D, int K, int R>
__host__ __device__ constexpr int cross_slots() {
    int s = 0;
    if constexpr (R != 0) s += block_slots<D, K, R, 0>();
    if constexpr (R != 1) s += block_slots<D, K, R, 1>();
    if constexpr (D == 3 && R != 2) s += block_slots<D, K, R, (D == 3 ? 2 : 0)>();
    return s;
}

template <int D, int K, int R, bool XC>
__host__ __device__ constexpr int row_slots() {
    if constexpr (R < D) {
        return block_slots<D, K, R, R>() + block_slots<D, K, R, D>() + (XC ? cross_slots<D, K, R>() : 0);
    } else {
        return block_slots<D, K, R, 0>() + block_slots<D, K, R, 1>() + (D == 3 ? block_slots<D, K, R, 2 % D>() : 0);
    }
}

template <int D, int K, int R, bool XC>
__host__ __device__ constexpr int row_slots_padded() {
    return (row_slots<D, K, R, XC>() + kEll - 1) / kEll * kEll;
}

// (K U) of row li of block R with its values at vp (slot 0 of the row; its
// chunks 64 * kEll values apart)
template <int D, int K, int R, int LPR, bool WIN, bool XC, class T, bool NT = false>
__device__ __forceinline__ T row_dot_vp(const SpmvArgsT<T> &a, int li, int lane, const T *vp) {
    const int nb0 = a.nb[R][0], nb1 = a.nb[R][1];
    const int i0 = li % nb0;
    const int t = li / nb0;
    const int i1 = t % nb1;
    const int i2 = t / nb1;
    T acc;
    if constexpr (R < D) {
        acc = block_dot<D, K, R, R, LPR, WIN, T, NT>(a, i0, i1, i2, lane, vp, 0);
        acc += block_dot<D, K, R, D, LPR, WIN, T, NT>(a, i0, i1, i2, lane, vp, block_slots<D, K, R, R>());
        if constexpr (XC) {
            int s0 = block_slots<D, K, R, R>() + block_slots<D, K, R, D>();
            if constexpr (R != 0) {
                acc += block_dot<D, K, R, 0, LPR, WIN, T, NT>(a, i0, i1, i2, lane, vp, s0);
                s0 += block_slots<D, K, R, 0>();
            }
            if constexpr (R != 1) {
                acc += block_dot<D, K, R, 1, LPR, WIN, T, NT>(a, i0, i1, i2, lane, vp, s0);
                s0 += block_slots<D, K, R, 1>();
            }
            if constexpr (D == 3 && R != 2)
                acc += block_dot<D, K, R, (D == 3 ? 2 : 0), LPR, WIN, T, NT>(a, i0, i1, i2, lane, vp, s0);
        }
    } else {
        constexpr int s1 = block_slots<D, K, R, 0>(), s2 = s1 + block_slots<D, K, R, 1>();
        acc = block_dot<D, K, R, 0, LPR, WIN, T, NT>(a, i0, i1, i2, lane, vp, 0);
        acc += block_dot<D, K, R, 1, LPR, WIN, T, NT>(a, i0, i1, i2, lane, vp, s1);
        if constexpr (D == 3) acc += block_dot<D, K, R, 2, LPR, WIN, T, NT>(a, i0, i1, i2, lane, vp, s2);
    }
    return acc;
}

template <int D, int K, int R, int LPR, bool WIN, bool XC, class T, bool NT = false>
__device__ __forceinline__ T row_dot(const SpmvArgsT<T> &a, int li, int lane) {
    const T *vp = a.val + a.val_off[R] + (int64_t)(li >> 6) * (row_slots_padded<D, K, R, XC>() * 64) + (li & 63) * kEll;
    return row_dot_vp<D, K, R, LPR, WIN, XC, T, NT>(a, li, lane, vp);
}

// (K U)_g of row g of a level (LPR = 1; args already offset to one problem)
template <int D, int K, bool WIN, bool XC, class T>
__device__ __forceinline__ T spmv_row(const SpmvArgsT<T> &a, int g) {
    if (g < a.off[1]) return row_dot<D, K, 0, 1, WIN, XC, T>(a, g, 0);
    if (g < a.off[2]) return row_dot<D, K, 1, 1, WIN, XC, T>(a, g - (int)a.off[1], 0);
    if (D == 3 && g < a.off[3]) return row_dot<D, K, (D == 3 ? 2 : 1), 1, WIN, XC, T>(a, g - (int)a.off[2], 0);
    return row_dot<D, K, D, 1, WIN, XC, T>(a, g - (int)a.off[D], 0);
}

// (K U)_g of row g with its values at vp (a copy of the row in another order)
template <int D, int K, bool WIN, bool XC, class T>
__device__ __forceinline__ T spmv_row_vp(const SpmvArgsT<T> &a, int g, const T *vp) {
    if (g < a.off[1]) return row_dot_vp<D, K, 0, 1, WIN, XC, T>(a, g, 0, vp);
    if (g < a.off[2]) return row_dot_vp<D, K, 1, 1, WIN, XC, T>(a, g - (int)a.off[1], 0, vp);
    if (D == 3 && g < a.off[3]) return row_dot_vp<D, K, (D == 3 ? 2 : 1), 1, WIN, XC, T>(a, g - (int)a.off[2], 0, vp);
    return row_dot_vp<D, K, D, 1, WIN, XC, T>(a, g - (int)a.off[D], 0, vp);
}

}  // namespace dfmg
