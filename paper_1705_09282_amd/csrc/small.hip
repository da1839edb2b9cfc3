// Additive Schwarz, step 1, form 4, in a tunable tile shape (TileShape).
//
// Blocks below nb_small: one thread per small subdomain (at most kSmallPatch
// DOFs, the interior ones), BS per workgroup; its DOFs are stored
// subdomain-minor, so the gather coalesces, and its rows of M_p E_p r are
// written row-major over the small subdomains (coalesced stores).  When every
// small subdomain of a wavefront (MS 0) or of the workgroup (MS 1) shares one
// inverse (the interior class), that inverse is read with scalar loads (one
// per wavefront, from the scalar cache) or staged once in LDS; MS 2 reads it
// per thread like any other.  The other blocks: TB threads per remaining
// (boundary) subdomain, BS / TB subdomains per workgroup; the threads gather
// the residual entries into LDS while each preloads its row of the local
// inverse (or of the potential map) into registers, then thread t sums row t
// (and rows t + TB, ...).  Every row is summed in the order of patch_row, so
// all tile shapes and the other smoother forms agree bit for bit;
// k_dof_update reads the corrections through the relabelled inverse map.  No
// load waits on more than one earlier load.  Every thread of a workgroup
// reaches its barriers (threads past the last subdomain work on a valid one
// and store nothing).
#include "schwarz_dev.hpp"

#include <algorithm>

namespace dfmg {

template <bool EXIT, int BS, int MS, int TB, class T>
__global__ __launch_bounds__(BS) void k_patch_solve_small(PatchArgsT<T> a, int nb_small) {
    const int prob = blockIdx.y;
    const int halt = stop_flag(a.stop, prob);  // block-uniform; gates the stores
    if (EXIT && halt) return;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const T *r = a.r + prob * a.svec;
    T *delta = a.delta + prob * a.sdelta;
    if (b < nb_small) {
        const int q0 = b * BS + (int)threadIdx.x;
        const bool live = q0 < a.nsmall;
        const int q = live ? q0 : a.nsmall - 1;
        const int4 si = a.sinfo[(int64_t)prob * a.nsmall + q];
        const int nn = si.x;
        T rv[kSmallPatch];
#pragma unroll
        for (int c = 0; c < kSmallPatch; ++c) {  // padded by repetition: always a valid index
            const T x = r[a.small_dofs[(int64_t)c * a.nsmall + q]];
            rv[c] = c < nn ? x : T(0);
        }
        const bool store = live && !halt;
        const T *m = a.M + prob * a.sM + si.y;
        T out[kSmallPatch];
        bool done = false;
        if constexpr (MS == 1) {
            // one inverse for the whole workgroup: staged in LDS
            __shared__ T sm[kSmallPatch * kSmallPatch];
            __shared__ int s_m0;
            if (threadIdx.x == 0) s_m0 = si.y;
            __syncthreads();
            const int m0 = s_m0;
            if (__syncthreads_and(si.y == m0 && nn == kSmallPatch)) {
                const T *mu = a.M + prob * a.sM + m0;
                for (int i = threadIdx.x; i < kSmallPatch * kSmallPatch; i += BS) sm[i] = mu[i];
                __syncthreads();
#pragma unroll
                for (int row = 0; row < kSmallPatch; ++row) {
                    T acc = 0;
#pragma unroll
                    for (int c = 0; c < kSmallPatch; ++c) acc = fma(sm[row * kSmallPatch + c], rv[c], acc);
                    out[row] = acc;
                }
                done = true;
            }
        } else if constexpr (MS == 0) {
            const int m0 = __builtin_amdgcn_readfirstlane(si.y);
            if (__all(si.y == m0) && __builtin_amdgcn_readfirstlane(nn) == kSmallPatch) {
                // the wave shares one inverse (the interior class): read it with
                // scalar loads instead of one vector load per lane
                const T *mu = a.M + prob * a.sM + m0;
#pragma unroll
                for (int row = 0; row < kSmallPatch; ++row) {
                    T acc = 0;
#pragma unroll
                    for (int c = 0; c < kSmallPatch; ++c) acc = fma(scalar_ld(mu + row * kSmallPatch + c), rv[c], acc);
                    out[row] = acc;
                }
                done = true;
            }
        }
        if (done) {
            if (store)
#pragma unroll
                for (int row = 0; row < kSmallPatch; ++row) delta[(int64_t)row * a.nsmall + q] = out[row];
        } else if (nn == kSmallPatch) {
            if (a.msoa) {
                // per-subdomain inverses, interleaved in 16-byte chunks (W
                // consecutive coefficients of a row): each load coalesces
                constexpr int W = 16 / (int)sizeof(T), NCH = kSmallPatch / W;
                const T *ms = a.msoa + (int64_t)prob * kSmallPatch * kSmallPatch * a.nsmall + (int64_t)q * W;
#pragma unroll
                for (int row = 0; row < kSmallPatch; ++row) {
                    T acc = 0;
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) {
                        const T *p4 = ms + (int64_t)(row * NCH + ch) * a.nsmall * W;
                        T v[W];
                        if constexpr (W == 4) {
                            const float4 x = *reinterpret_cast<const float4 *>(p4);
                            v[0] = x.x, v[1] = x.y, v[2] = x.z, v[3] = x.w;
                        } else {
                            const double2 x = *reinterpret_cast<const double2 *>(p4);
                            v[0] = x.x, v[1] = x.y;
                        }
#pragma unroll
                        for (int j = 0; j < W; ++j) acc = fma(v[j], rv[ch * W + j], acc);
                    }
                    out[row] = acc;
                }
            } else {
#pragma unroll
                for (int row = 0; row < kSmallPatch; ++row) {
                    T acc = 0;
#pragma unroll
                    for (int c = 0; c < kSmallPatch; ++c) acc = fma(m[row * kSmallPatch + c], rv[c], acc);
                    out[row] = acc;
                }
            }
            if (store)
#pragma unroll
                for (int row = 0; row < kSmallPatch; ++row) delta[(int64_t)row * a.nsmall + q] = out[row];
        } else {
            for (int row = 0; row < nn; ++row) {
                const T v = small_row(m + row * nn, nn, rv);
                if (store) delta[(int64_t)row * a.nsmall + q] = v;
            }
        }
        if (a.psi) {  // the subdomain's single potential
            T v;
            bool qdone = false;
            if constexpr (MS == 0) {
                const int z0 = __builtin_amdgcn_readfirstlane(si.z);
                if (__all(si.z == z0) && __builtin_amdgcn_readfirstlane(nn) == kSmallPatch) {
                    const T *qu = a.Q + prob * a.sQ + z0;
                    v = 0;
#pragma unroll
                    for (int c = 0; c < kSmallPatch; ++c) v = fma(scalar_ld(qu + c), rv[c], v);
                    qdone = true;
                }
            }
            if (!qdone && a.qsoa && nn == kSmallPatch) {
                // per-subdomain maps, interleaved (the order of small_row)
                const T *qs = a.qsoa + (int64_t)prob * kSmallPatch * a.nsmall + q;
                v = 0;
#pragma unroll
                for (int c = 0; c < kSmallPatch; ++c) v = fma(qs[(int64_t)c * a.nsmall], rv[c], v);
                qdone = true;
            }
            if (!qdone) v = small_row(a.Q + prob * a.sQ + si.z, nn, rv);
            if (store) a.beta[prob * a.nbeta + si.w] = v;
        }
        return;
    }
    extern __shared__ unsigned char smem[];
    const int width = a.max_big > kBigRegs ? a.max_big : kBigRegs;
    const int sub = (int)threadIdx.x / TB;
    T *sr = reinterpret_cast<T *>(smem) + sub * width;
    const int t = (int)threadIdx.x % TB;
    int sb = (b - nb_small) * (BS / TB) + sub;
    if constexpr (TB == 64) sb = __builtin_amdgcn_readfirstlane(sb);
    const bool live = sb < a.nbsub;
    const int4 bm = live ? a.bmesh[sb] : make_int4(0, 0, 0, 0);
    const int2 bp = live ? a.binfo[(int64_t)prob * a.nbsub + sb] : make_int2(0, 0);
    const int base = bm.x, nn = bm.y, rows = nn + (a.psi ? bm.w : 0);
    const T *Mp = a.M + prob * a.sM + bp.x;
    const T *Qp = a.Q ? a.Q + prob * a.sQ + bp.y : nullptr;
    // thread t's first row: its coefficients into registers (independent of r;
    // unconditional loads, clamped to the row, so none waits for another)
    const T *mr = t >= rows ? Mp : (t < nn ? Mp + (int64_t)t * nn : Qp + (int64_t)(t - nn) * nn);
    const int last = nn > 0 ? nn - 1 : 0;
    T mv[kBigRegs];
#pragma unroll
    for (int c = 0; c < kBigRegs; ++c) mv[c] = T(0);
    if (t < rows) {
#pragma unroll
        for (int c0 = 0; c0 < kBigRegs; c0 += 8) {
            if (c0 < nn)  // only the chunks the row has
#pragma unroll
                for (int c = c0; c < c0 + 8; ++c) mv[c] = mr[c < nn ? c : last];  // past nn: times sr = 0
        }
    }
    // the residual entries, zero up to kBigRegs (the padded terms, finite
    // coefficients times zero, add zero)
    const int span = nn > kBigRegs ? nn : kBigRegs;
    for (int c = t; c < span; c += TB) sr[c] = c < nn ? r[a.pdofs[base + c]] : T(0);
    __syncthreads();
    if (t < rows) {
        T acc = 0;
#pragma unroll
        for (int c = 0; c < kBigRegs; ++c) acc = fma(mv[c], sr[c], acc);
        for (int c = kBigRegs; c < nn; ++c) acc = fma(mr[c], sr[c], acc);
        if (!halt) {
            if (t < nn) delta[(int64_t)kSmallPatch * a.nsmall + base + t] = acc;
            else a.beta[prob * a.nbeta + bm.z + (t - nn)] = acc;
        }
    }
    for (int u = t + TB; u < rows; u += TB) {  // subdomains of more than TB rows
        const T *ur = u < nn ? Mp + (int64_t)u * nn : Qp + (int64_t)(u - nn) * nn;
        T acc = 0;
        for (int c = 0; c < nn; ++c) acc = fma(ur[c], sr[c], acc);
        if (!halt) {
            if (u < nn) delta[(int64_t)kSmallPatch * a.nsmall + base + u] = acc;
            else a.beta[prob * a.nbeta + bm.z + (u - nn)] = acc;
        }
    }
}

template <int BS, int MS, int TB, class T>
static void launch_shape(const PatchArgsT<T> &a, hipStream_t s) {
    constexpr int per = BS / TB;  // boundary subdomains per workgroup
    const int nbs = (a.nsmall + BS - 1) / BS, nbb = (a.nbsub + per - 1) / per;
    const size_t lds = (size_t)per * std::max(a.max_big, kBigRegs) * sizeof(T);
    const dim3 grid(padded_grid(nbs + nbb), a.nprob);
    if (a.exit_early)
        hipLaunchKernelGGL((k_patch_solve_small<true, BS, MS, TB, T>), grid, dim3(BS), lds, s, a, nbs);
    else
        hipLaunchKernelGGL((k_patch_solve_small<false, BS, MS, TB, T>), grid, dim3(BS), lds, s, a, nbs);
}

template <int BS, int MS, class T>
static void launch_tb(const PatchArgsT<T> &a, hipStream_t s) {
    if (a.tile.tb == 32) launch_shape<BS, MS, 32, T>(a, s);
    else launch_shape<BS, MS, 64, T>(a, s);
}

template <int BS, class T>
static void launch_ms(const PatchArgsT<T> &a, hipStream_t s) {
    if (a.tile.ms == 1) launch_tb<BS, 1, T>(a, s);
    else if (a.tile.ms == 2) launch_tb<BS, 2, T>(a, s);
    else launch_tb<BS, 0, T>(a, s);
}

// dynamic LDS above which a shape falls back to the default one
constexpr size_t kTileLdsMax = 48 * 1024;

template <class T>
void launch_schwarz_small(const PatchArgsT<T> &a, hipStream_t s) {
    PatchArgsT<T> b = a;
    const size_t lds = (size_t)(b.tile.bs / b.tile.tb) * std::max(b.max_big, kBigRegs) * sizeof(T);
    if (lds > kTileLdsMax) b.tile = TileShape{};
    if (b.tile.bs == 64) launch_ms<64, T>(b, s);
    else if (b.tile.bs == 128) launch_ms<128, T>(b, s);
    else if (b.tile.bs == 512) launch_ms<512, T>(b, s);
    else launch_ms<256, T>(b, s);
    launch_dof_update<T>(b, s);
}

template void launch_schwarz_small<double>(const PatchArgsT<double> &, hipStream_t);
template void launch_schwarz_small<float>(const PatchArgsT<float> &, hipStream_t);

}  // namespace dfmg
