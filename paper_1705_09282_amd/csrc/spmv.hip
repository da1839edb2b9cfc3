// Residual r = F - K U of one level in the stencil-ELL layout, FP64 or FP32
// (values, vectors and accumulation all in T).
#include "spmv_dev.hpp"

namespace dfmg {

// r = F - K U, optionally with per-block partial sums of r^2.  Each block
// covers kBlock / LPR rows.  A stopped problem's blocks return at once
// (GATE false: large grids, where the loads cost bandwidth), or load as usual
// and skip the stores (GATE true: small grids, where the flag's load would
// otherwise add its latency in front of every other load).  XC: the
// velocity rows couple every velocity component (mapped domains).  NT:
// non-temporal value loads (see block_dot).
template <int D, int K, int LPR, bool WIN, bool GATE, bool XC, class T, bool NT = false>
__global__ __launch_bounds__(kBlock) void k_spmv(SpmvArgsT<T> a) {
    const int prob = blockIdx.y;
    a.val += prob * a.sval;
    a.F += prob * a.svec;
    a.U += prob * a.svec;
    a.r += prob * a.svec;
    if (a.partial) a.partial += prob * a.spart;
    const int halt = stop_flag(a.stop, prob);  // block-uniform
    if (!GATE && halt) return;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int lane = (LPR > 1) ? (threadIdx.x % LPR) : 0;
    const int g = b * (kBlock / LPR) + threadIdx.x / LPR;
    double rr = 0.0;
    const bool active = b < a.nblocks && g < a.n;
    T acc = 0;
    if (active) {
        if (g < a.off[1]) {
            acc = row_dot<D, K, 0, LPR, WIN, XC, T, NT>(a, g, lane);
        } else if (g < a.off[2]) {
            acc = row_dot<D, K, 1, LPR, WIN, XC, T, NT>(a, g - (int)a.off[1], lane);
        } else if (D == 3 && g < a.off[3]) {
            acc = row_dot<D, K, (D == 3 ? 2 : 1), LPR, WIN, XC, T, NT>(a, g - (int)a.off[2], lane);
        } else {
            acc = row_dot<D, K, D, LPR, WIN, XC, T, NT>(a, g - (int)a.off[D], lane);
        }
    }
    // combine the LPR partial dot products of a row (lanes of a row are
    // consecutive within one wave)
#pragma unroll
    for (int o = 1; o < LPR; o <<= 1) acc += __shfl_xor(acc, o, 64);
    if (active && lane == 0) {
        const T v = a.F[g] - acc;
        if (!halt) a.r[g] = v;
        rr = (double)v * (double)v;
    }
    if (a.partial) {
        __shared__ double sh[kBlock / 64];
        const double s = block_sum(rr, sh);
        if (threadIdx.x == 0 && b < a.nblocks && !halt) a.partial[b] = s;
    }
}

template <int D, int K, bool WIN, bool GATE, class T>
static void launch_dkwg(const SpmvArgsT<T> &a, int lpr, hipStream_t s) {
    const dim3 grid(padded_grid(a.nblocks), a.nprob);
    if (a.xc) hipLaunchKernelGGL((k_spmv<D, K, 1, WIN, GATE, true, T>), grid, dim3(kBlock), 0, s, a);  // lpr is 1
    else if (a.nt && lpr == 1) hipLaunchKernelGGL((k_spmv<D, K, 1, WIN, GATE, false, T, true>), grid, dim3(kBlock), 0, s, a);
    else if (lpr == 4) hipLaunchKernelGGL((k_spmv<D, K, 4, WIN, GATE, false, T>), grid, dim3(kBlock), 0, s, a);
    else if (lpr == 2) hipLaunchKernelGGL((k_spmv<D, K, 2, WIN, GATE, false, T>), grid, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_spmv<D, K, 1, WIN, GATE, false, T>), grid, dim3(kBlock), 0, s, a);
}

// rows per problem below which a stopped problem's blocks gate their stores
// instead of returning at once (latency-bound launches)
constexpr int kGateRows = 1 << 16;

template <int D, int K, class T>
static void launch_dk(const SpmvArgsT<T> &a, int lpr, hipStream_t s) {
    const bool gate = !a.exit_early && a.n < kGateRows;
    if (a.win) {
        if (gate) launch_dkwg<D, K, true, true, T>(a, lpr, s);
        else launch_dkwg<D, K, true, false, T>(a, lpr, s);
    } else {
        if (gate) launch_dkwg<D, K, false, true, T>(a, lpr, s);
        else launch_dkwg<D, K, false, false, T>(a, lpr, s);
    }
}

// a.nblocks must equal spmv_blocks(a.n, lpr); with a.xc, lpr must be 1
template <class T>
void launch_spmv(int d, int k, int lpr, const SpmvArgsT<T> &a, hipStream_t s) {
    if (d == 2 && k == 1) launch_dk<2, 1, T>(a, lpr, s);
    else if (d == 2 && k == 2) launch_dk<2, 2, T>(a, lpr, s);
    else if (d == 3 && k == 1) launch_dk<3, 1, T>(a, lpr, s);
    else launch_dk<3, 2, T>(a, lpr, s);
}

template void launch_spmv<double>(int, int, int, const SpmvArgsT<double> &, hipStream_t);
template void launch_spmv<float>(int, int, int, const SpmvArgsT<float> &, hipStream_t);

}  // namespace dfmg
