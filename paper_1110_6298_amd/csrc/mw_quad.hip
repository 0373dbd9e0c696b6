// Explicit quadrature of the MW sampling theorem (Sec. IV-F, Eq.(quadrature)):
//   I = int dOmega f = sum_{t<L} sum_{p<nphi} f(theta_t, 2 pi p/nphi) q(theta_t) L/nphi,
//   q(theta_t) = (2 pi/L) [wt(theta_t) + (1 - delta_{t,L-1}) (-1)^s wt(theta_{2L-2-t})],
//   wt(theta_t) = 1/(2L-1) sum_{m'=-(L-1)}^{L-1} w(-m') e^{i m' theta_t},
// exact for maps band-limited at L.  nphi = L is the rule's own grid (phi'_p =
// 2 pi p/L); nphi = 2L-1 is the transform grid, on which the phi sum is the
// same exact phi integral of a band-limited ring.
//
// The reduction is HBM-bound (one read of the map): one workgroup per ring sums
// its samples and evaluates its weight (two O(L) sums of the reflected weights),
// and a second small kernel adds the rings of each map.  Both reductions run in
// a fixed order, so results do not depend on scheduling.
#include "mw_internal.h"

namespace mw {
namespace {

constexpr int QT = 256;   // threads per workgroup (4 waves)

// w(k) of the theta convolution (Sec. IV-D): +-i pi/2 at k = +-1, 0 at other
// odd k, 2/(1 - k^2) at even k.
__device__ __forceinline__ double2 weight_k(int k)
{
    if (k == 1) return make_double2(0.0, 1.5707963267948966192);
    if (k == -1) return make_double2(0.0, -1.5707963267948966192);
    if (k & 1) return make_double2(0.0, 0.0);
    return make_double2(2.0 / (1.0 - (double)k * (double)k), 0.0);
}

// Sum of v over the workgroup, in a fixed order: a shuffle tree within each
// wave, then the wave sums in wave order.  Every thread gets the result.
__device__ __forceinline__ double2 block_sum(double2 v, double2* red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v.x += __shfl_down(v.x, o, 64);
        v.y += __shfl_down(v.y, o, 64);
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();   // red may still be read by a previous call
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double2 s = red[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
        s.x += red[k].x;
        s.y += red[k].y;
    }
    return s;
}

// wt(theta_t), t < 2L-1: e^{i m' theta_t} = e^{i pi r/N1} with r = m'(2t+1)
// reduced exactly modulo 2 N1.  The terms of m' and -m' are conjugate, so the
// sum is real; its real part is returned.
__device__ double wtilde(int L, int t, double2* red)
{
    const int N1 = 2 * L - 1;
    double2 acc = make_double2(0.0, 0.0);
    for (int mp = -(L - 1) + (int)threadIdx.x; mp <= L - 1; mp += blockDim.x) {
        long long r = ((long long)mp * (2 * t + 1)) % (2LL * N1);
        if (r < 0) r += 2LL * N1;
        double sn, cs;
        sincospi((double)r / (double)N1, &sn, &cs);
        const double2 w = weight_k(-mp);
        acc.x += w.x * cs - w.y * sn;
        acc.y += w.x * sn + w.y * cs;
    }
    return block_sum(acc, red).x / (double)N1;
}

__device__ double qweight(int L, int s, int t, double2* red)
{
    double v = wtilde(L, t, red);
    if (t != L - 1) v += ((s & 1) ? -1.0 : 1.0) * wtilde(L, 2 * L - 2 - t, red);
    return (6.283185307179586476925286766559 / (double)L) * v;
}

// q(theta_t) for t < L, one workgroup per t.
__global__ __launch_bounds__(QT) void k_quad_weights(int L, int s, double* __restrict__ q)
{
    __shared__ double2 red[QT / 64];
    const int t = blockIdx.x;
    const double v = qweight(L, s, t, red);
    if (threadIdx.x == 0) q[t] = v;
}

// Ring t of map blockIdx.y: partial[map*L + t] = (sum_p f(t, p)) q(theta_t) L/nphi.
template <int REAL>
__global__ __launch_bounds__(QT) void k_integrate_rings(Batch B, int L, int nphi, double2* __restrict__ partial)
{
    __shared__ double2 red[QT / 64];
    const int t = blockIdx.x, b = blockIdx.y;
    const void* __restrict__ f = B.in[b];
    double2 acc = make_double2(0.0, 0.0);
    for (int p = threadIdx.x; p < nphi; p += blockDim.x) {
        if (REAL) {
            acc.x += ((const double*)f)[(size_t)t * nphi + p];
        } else {
            const double2 v = ((const double2*)f)[(size_t)t * nphi + p];
            acc.x += v.x;
            acc.y += v.y;
        }
    }
    const double2 ring = block_sum(acc, red);
    const double q = qweight(L, B.s[b], t, red) * ((double)L / (double)nphi);
    if (threadIdx.x == 0) partial[(size_t)b * L + t] = make_double2(ring.x * q, ring.y * q);
}

// I of map blockIdx.x: the sum of its L ring partials.
__global__ __launch_bounds__(QT) void k_integrate_sum(Batch B, int L, const double2* __restrict__ partial)
{
    __shared__ double2 red[QT / 64];
    const int b = blockIdx.x;
    double2 acc = make_double2(0.0, 0.0);
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        const double2 v = partial[(size_t)b * L + t];
        acc.x += v.x;
        acc.y += v.y;
    }
    const double2 I = block_sum(acc, red);
    if (threadIdx.x == 0) *(double2*)B.out[b] = I;
}

}  // namespace

hipError_t launch_quad_weights(int L, int s, double* q, hipStream_t st)
{
    hipLaunchKernelGGL(k_quad_weights, dim3(L), dim3(QT), 0, st, L, s, q);
    return hipGetLastError();
}

hipError_t launch_integrate(int L, int nphi, int real, const Batch& B, double2* partial, hipStream_t st)
{
    if (real) hipLaunchKernelGGL(k_integrate_rings<1>, dim3(L, B.n), dim3(QT), 0, st, B, L, nphi, partial);
    else hipLaunchKernelGGL(k_integrate_rings<0>, dim3(L, B.n), dim3(QT), 0, st, B, L, nphi, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_integrate_sum, dim3(B.n), dim3(QT), 0, st, B, L, (const double2*)partial);
    return hipGetLastError();
}

}  // namespace mw
