// Multiplicative Schwarz sweep (equation MSM): the subdomains are solved one
// after the other, each on the residual that the previous ones left, with no
// damping.  The sweep visits them colour by colour in a coupling-free
// colouring: two subdomains of one colour share no DOF and no entry of K
// couples a DOF of one with a DOF of the other, so solving a colour's
// subdomains at the same time is the same as solving them in turn -- no
// update inside a colour changes the residual another one reads.  One launch
// per colour; a workgroup takes up to B (subdomain, row) entries of the
// colour (B = 256, or 1024 on levels with larger subdomains; from the host's
// lane table, where a subdomain's entries lie in one workgroup, `stride`
// threads apart: consecutive, or interleaved with those of other subdomains
// of the same size, so that a wavefront holds one local row of many
// subdomains -- rows of one block, one row form): thread t computes the
// residual of its DOF, (F - K U)_g, straight from the operator row, the
// workgroup's residual entries meet in LDS, and thread t then applies its row
// of the subdomain's bordered local inverse and adds the result to U_g in
// place (plain read-modify-write: the colour's subdomains hold disjoint
// DOFs).  The layout decides only which thread does what: every sum runs in
// the same order.
// The rows of one colour are k+2 apart in the grid, so in the stencil-ELL
// layout (64 consecutive rows per slice) a wavefront uses a fraction of
// every line it loads; the sweep reads a copy of the operator values in lane
// order instead, where a wavefront's rows are consecutive slots of a slice
// (same values and order, so the same sums).
#include "spmv_dev.hpp"

namespace dfmg {

template <int D, int K, bool WIN, bool XC, int B, class T>
__global__ __launch_bounds__(B) void k_schwarz_mult(MultArgsT<T> a) {
    const int prob = blockIdx.y;
    const int halt = stop_flag(a.sp.stop, prob);  // block-uniform
    if (a.sp.exit_early && halt) return;
    SpmvArgsT<T> sp = a.sp;
    sp.val += prob * sp.sval;
    sp.F += prob * sp.svec;
    sp.U += prob * sp.svec;
    T *U = a.U + prob * sp.svec;
    __shared__ T sr[B];
    const int w = blockIdx.x;
    const int e = w < a.nwaves ? a.lanes[(int64_t)w * B + threadIdx.x] : -1;
    const int stride = w < a.nwaves ? a.strides[w] : 1;
    int g = 0;
    int4 info = make_int4(0, 0, 0, 0);
    T r = 0;
    if (e >= 0) {
        g = a.pdofs[e];
        info = a.ent_info[(int64_t)prob * a.nent + e];
        if (a.mval) {  // the rows in lane order: a wavefront's value loads are contiguous
            const int64_t lane = a.lane0 + (int64_t)w * B + threadIdx.x;
            const T *vp = a.mval + prob * a.smval + (lane >> 6) * ((int64_t)a.mslots * 64) + (lane & 63) * kEll;
            r = sp.F[g] - spmv_row_vp<D, K, WIN, XC, T>(sp, g, vp);
        } else {
            r = sp.F[g] - spmv_row<D, K, WIN, XC, T>(sp, g);
        }
    }
    // U_g before the barrier: no other thread of the colour writes it
    const T u0 = e >= 0 ? U[g] : T(0);
    sr[threadIdx.x] = r;
    __syncthreads();
    if (e >= 0) {
        // this thread holds local row m = e - (first entry of the subdomain);
        // entry c of the subdomain sits on thread t + (c - m) * stride
        const T *loc = sr + (int)threadIdx.x - (e - info.y) * stride;
        const T *mrow = a.M + prob * a.sM + info.x;
        T acc = 0;
        for (int c = 0; c < info.z; ++c) acc = fma(mrow[c], loc[c * stride], acc);
        if (!halt) U[g] = u0 + acc;
    }
}

template <int D, int K, bool XC, int B, class T>
static void launch_dkxb(const MultArgsT<T> &a, hipStream_t s) {
    const dim3 grid(a.nwaves, a.sp.nprob);
    if (a.sp.win) hipLaunchKernelGGL((k_schwarz_mult<D, K, true, XC, B, T>), grid, dim3(B), 0, s, a);
    else hipLaunchKernelGGL((k_schwarz_mult<D, K, false, XC, B, T>), grid, dim3(B), 0, s, a);
}

template <int D, int K, int B, class T>
static void launch_dkb(const MultArgsT<T> &a, hipStream_t s) {
    if (a.sp.xc) launch_dkxb<D, K, true, B, T>(a, s);
    else launch_dkxb<D, K, false, B, T>(a, s);
}

template <int D, int K, class T>
static void launch_dk(const MultArgsT<T> &a, hipStream_t s) {
    if (a.width == kMultLanes) launch_dkb<D, K, kMultLanes, T>(a, s);
    else launch_dkb<D, K, kMultLanesBig, T>(a, s);
}

template <class T>
void launch_schwarz_mult(int d, int k, const MultArgsT<T> &a, hipStream_t s) {
    if (a.nwaves <= 0) return;
    if (d == 2 && k == 1) launch_dk<2, 1, T>(a, s);
    else if (d == 2 && k == 2) launch_dk<2, 2, T>(a, s);
    else if (d == 3 && k == 1) launch_dk<3, 1, T>(a, s);
    else launch_dk<3, 2, T>(a, s);
}

template void launch_schwarz_mult<double>(int, int, const MultArgsT<double> &, hipStream_t);
template void launch_schwarz_mult<float>(int, int, const MultArgsT<float> &, hipStream_t);

}  // namespace dfmg
