// Fourier stages of the MW transforms (the O(L^2 log L) part):
//   phi stage   : one workgroup per ring t, DFT of length N1 = 2L-1 along phi
//   theta stage : one workgroup per order m, periodic extension in theta,
//                 DFT of length N1 with the half-sample twiddle, and (forward)
//                 the weight convolution done as a product on an N2-point grid.
// Every DFT of the odd length N1 is evaluated with Bluestein's chirp identity
// on a power-of-two FFT of length N2 >= 4L-3 (the same N2 that the weight
// convolution needs), held entirely in LDS.
#include <type_traits>

#include "mw_internal.h"

namespace mw {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// multiply by DIR * i
template <int DIR>
__device__ __forceinline__ double2 mul_dir_i(double2 a)
{
    return DIR < 0 ? make_double2(a.y, -a.x) : make_double2(-a.y, a.x);
}

// LDS index of FFT entry i.  A 128-byte LDS row holds 8 complex entries.  For
// RB = 8 the column (i mod 8) is XOR-ed with the row's low three bits, so the
// stride-8 stores of a main pass and the unit-stride loads both fall on distinct
// banks with no padding (the buffer is exactly N entries); for RB = 16 one pad
// entry per 16 does the same for the stride-16 stores.
template <int RB>
__device__ __forceinline__ int Pr(int i)
{
    if constexpr (RB == 8) return i ^ ((i >> 3) & 7);
    else return i + i / RB;
}

// Entries b + t*S (t = 0, 1, ...) of a pass sit at x + Pr(b) + t*S whenever
// pr_linear(S): for RB = 8, when S is a multiple of 64 (the step leaves the row's
// low three bits, and so the XOR, unchanged, and does not touch the column
// bits).  One swizzled base per thread then serves all RB accesses with
// constant offsets.  (The padded RB = 16 layout is linear too for S a multiple
// of 16, but there the extra live base registers cost the 512-thread kernels
// more spills than the address arithmetic they save.)
template <int RB>
__device__ __forceinline__ bool pr_linear(int S)
{
    return RB == 8 && (S & 63) == 0;
}

// Block-wide loop over j = threadIdx.x + q*blockDim.x < n (n <= 16*blockDim.x):
// the global loads ld(j) of eight consecutive q are all issued before any result
// is used by use(j, value), so a thread waits for memory twice, not 16 times.
struct Pair2 { double2 a, b; };

template <class Ld, class Use>
__device__ __forceinline__ void staged_loop(int n, Ld ld, Use use)
{
    using V = decltype(ld(0));
#pragma unroll
    for (int h = 0; h < 16; h += 8) {
        V v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = threadIdx.x + (h + q) * blockDim.x;
            if (j < n) v[q] = ld(j);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = threadIdx.x + (h + q) * blockDim.x;
            if (j < n) use(j, v[q]);
        }
    }
}

// The same loop with its global values read ahead: read_ahead<Q>(n, ld) issues
// the loads ld(j) of every j = threadIdx.x + q*blockDim.x < n (q < Q, which must
// cover n) at once, early in a kernel (before the transforms), and
// use_ahead<Q>(n, a, use) later calls use(j, value), so that their latency
// overlaps the transforms instead of following the last barrier.
template <int Q, class V>
struct Ahead { V v[Q]; };

template <int Q, class Ld>
__device__ __forceinline__ auto read_ahead(int n, Ld ld)
{
    Ahead<Q, decltype(ld(0))> a;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = threadIdx.x + q * blockDim.x;
        if (j < n) a.v[q] = ld(j);
    }
    return a;
}

template <int Q, class V, class Use>
__device__ __forceinline__ void use_ahead(int n, const Ahead<Q, V>& a, Use use)
{
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = threadIdx.x + q * blockDim.x;
        if (j < n) use(j, a.v[q]);
    }
}

// In-place DFT of 4 values: a_k <- sum_j a_j w^{jk}, w = exp(DIR 2 pi i/4).
template <int DIR>
__device__ __forceinline__ void bf4(double2& a0, double2& a1, double2& a2, double2& a3)
{
    const double2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3);
    const double2 t3 = mul_dir_i<DIR>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a1 = cadd(t1, t3);
    a2 = csub(t0, t2);
    a3 = csub(t1, t3);
}

// exp(DIR 2 pi i e/16) for a compile-time e
template <int DIR, int E>
__device__ __forceinline__ double2 w16()
{
    constexpr double C[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                              0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                              -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                              0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
    constexpr double S[16] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                              1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                              0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                              -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};
    return make_double2(C[E & 15], DIR * S[E & 15]);
}

// DFT of 16 values in registers as 4 x 4: inner DFT4 over j of x[a + 4j], twiddle
// w16^{ab}, outer DFT4 over a; X[b + 4c] ends in v[4b + c] and is moved to v[b + 4c].
template <int DIR>
__device__ __forceinline__ void dft16(double2 (&v)[16])
{
#pragma unroll
    for (int a = 0; a < 4; ++a) bf4<DIR>(v[a], v[a + 4], v[a + 8], v[a + 12]);
    // now v[a + 4b] = inner result b of column a
    v[1 + 4] = cmul(v[1 + 4], w16<DIR, 1>());
    v[1 + 8] = cmul(v[1 + 8], w16<DIR, 2>());
    v[1 + 12] = cmul(v[1 + 12], w16<DIR, 3>());
    v[2 + 4] = cmul(v[2 + 4], w16<DIR, 2>());
    v[2 + 8] = mul_dir_i<DIR>(v[2 + 8]);   // w16^4 = DIR i
    v[2 + 12] = cmul(v[2 + 12], w16<DIR, 6>());
    v[3 + 4] = cmul(v[3 + 4], w16<DIR, 3>());
    v[3 + 8] = cmul(v[3 + 8], w16<DIR, 6>());
    v[3 + 12] = cmul(v[3 + 12], w16<DIR, 9>());
#pragma unroll
    for (int b = 0; b < 4; ++b) bf4<DIR>(v[4 * b], v[4 * b + 1], v[4 * b + 2], v[4 * b + 3]);
    // v[4b + c] = X[b + 4c]: transpose the 4 x 4 block
    double2 t;
    t = v[1]; v[1] = v[4]; v[4] = t;
    t = v[2]; v[2] = v[8]; v[8] = t;
    t = v[3]; v[3] = v[12]; v[12] = t;
    t = v[6]; v[6] = v[9]; v[9] = t;
    t = v[7]; v[7] = v[13]; v[13] = t;
    t = v[11]; v[11] = v[14]; v[14] = t;
}

// DFT of 8 values in registers as 2 x 4 (natural order in and out).
template <int DIR>
__device__ __forceinline__ void dft8(double2* v)
{
    double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    bf4<DIR>(e0, e1, e2, e3);
    bf4<DIR>(o0, o1, o2, o3);
    o1 = cmul(o1, w16<DIR, 2>());
    o2 = mul_dir_i<DIR>(o2);   // w16^4 = DIR i
    o3 = cmul(o3, w16<DIR, 6>());
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// u_t *= w^t for t = 1..15, each power formed from w, w^2, w^4, w^8 (bits of t),
// i.e. a product of at most four factors.
template <int R>
__device__ __forceinline__ void twiddle_powers(double2* u, double2 w)
{
    const double2 w2 = cmul(w, w);
    const double2 w4 = cmul(w2, w2);
    const double2 w8 = cmul(w4, w4);
#pragma unroll
    for (int t = 1; t < R; ++t) {
        double2 f;
        bool have = false;
        if (t & 1) { f = w; have = true; }
        if (t & 2) { f = have ? cmul(f, w2) : w2; have = true; }
        if (t & 4) { f = have ? cmul(f, w4) : w4; have = true; }
        if (t & 8) { f = have ? cmul(f, w8) : w8; }
        u[t] = cmul(u[t], f);
    }
}

// Final Stockham pass of radix R = 2, 4 or 8 (the factor left after the main
// radix-RB passes): each thread holds RB/R butterflies in one RB-value register
// set.  With post != nullptr every output X_j is stored as X_j * post[j].
// Final store of a transform: PlainStore keeps output X_o at slot o; any other
// Store is called as st(o, X_o) once per output in the last pass's write phase
// (after every read of that pass), so it may write X_o, changed, to a slot of
// its choosing as long as the slots of all outputs are distinct.
struct PlainStore {
    __device__ void operator()(int, double2) const {}   // never called
};

// First load of a transform: PlainLoad reads the input from LDS; any other Load
// is called as ld(j) for every input j < N by the first pass (which needs no
// twiddles), so the input can come straight from global memory.
struct PlainLoad {
    __device__ double2 operator()(int) const { return make_double2(0.0, 0.0); }   // never called
};

// First load from registers: with N == RB * blockDim.x the first pass of thread
// i reads the inputs j = i + t*blockDim.x (t < RB) into its register t, so an
// input that thread i already holds as its t-th value can be passed as
// RegLoad{f}, f(t, j) returning input j from the thread's register t (t is a
// compile-time index after unrolling).
template <class F>
struct RegLoad {
    F f;
};
template <class F>
__device__ __forceinline__ RegLoad<F> reg_load(F f) { return RegLoad<F>{f}; }
template <class T> struct is_reg_load : std::false_type {};
template <class F> struct is_reg_load<RegLoad<F>> : std::true_type {};

template <int DIR, int R, int RB, class Store = PlainStore>
__device__ __forceinline__ void last_pass(double2* x, int N, int p, const double2 (&wl)[RB / 2],
                                          const double2* __restrict__ post, const Store& st = Store())
{
    constexpr int r = (R == 2) ? 1 : (R == 4) ? 2 : 3;
    constexpr int QM = RB / R;
    const int NB = N >> r;
    double2 u[RB];
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int i = threadIdx.x + q * blockDim.x;
        if (i < NB) {
            const int k = i & (p - 1);
            if (RB == 8 && pr_linear<RB>(NB)) {
                const double2* xb = x + Pr<RB>(i);
#pragma unroll
                for (int t = 0; t < R; ++t) u[q * R + t] = xb[t * NB];
            } else {
#pragma unroll
                for (int t = 0; t < R; ++t) u[q * R + t] = x[Pr<RB>(i + t * NB)];
            }
            double2 w = wl[q];
            if (DIR > 0) w = cconj(w);
            (void)k;
            twiddle_powers<R>(u + q * R, w);
            double2* v = u + q * R;
            if (R == 2) {
                const double2 a = v[0], b = v[1];
                v[0] = cadd(a, b); v[1] = csub(a, b);
            } else if (R == 4) {
                bf4<DIR>(v[0], v[1], v[2], v[3]);
            } else {
                dft8<DIR>(v);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int i = threadIdx.x + q * blockDim.x;
        if (i < NB) {
            const int k = i & (p - 1);
            const int j = ((i - k) << r) + k;
            if constexpr (!std::is_same_v<Store, PlainStore>) {
#pragma unroll
                for (int t = 0; t < R; ++t) st(j + t * p, u[q * R + t]);
            } else if (RB == 8 && pr_linear<RB>(p)) {
                double2* xb = x + Pr<RB>(j);
#pragma unroll
                for (int t = 0; t < R; ++t) xb[t * p] = post ? cmul(u[q * R + t], post[j + t * p]) : u[q * R + t];
            } else if (post) {
#pragma unroll
                for (int t = 0; t < R; ++t) x[Pr<RB>(j + t * p)] = cmul(u[q * R + t], post[j + t * p]);
            } else {
#pragma unroll
                for (int t = 0; t < R; ++t) x[Pr<RB>(j + t * p)] = u[q * R + t];
            }
        }
    }
    __syncthreads();
}

// Twiddle bases of one thread for every FFT of length N = 2^logN in a kernel
// (all FFTs of a kernel share N and the thread layout, so they are read from
// the table once, at the kernel's start, instead of once per pass):
//   w[s-1]  = exp(-2 pi i k / (p RB)) of main pass s >= 1 (p = RB^s, k = i mod p)
//   wl[q]   = the bases of the final radix-2^r pass for butterfly i + q*blockDim.
template <int RB>
struct FftTw {
    double2 w[3];
    double2 wl[RB / 2];   // the final pass has radix >= 2: at most RB/2 butterflies per thread
};

// shift: the table holds exp(-2 pi i e/(N 2^shift)) (a plan's N2 table serves
// the half-length transforms of split plans with shift = 1).
template <int RB>
__device__ __forceinline__ FftTw<RB> fft_twiddles(int N, int logN, const double2* __restrict__ tw, int shift = 0)
{
    constexpr int lr = (RB == 16) ? 4 : 3;
    const int i = threadIdx.x;
    const int np = logN / lr;
    const int r = logN - lr * np;
    FftTw<RB> T;
#pragma unroll
    for (int s = 1; s < 4; ++s) {
        T.w[s - 1] = make_double2(1.0, 0.0);
        if (s < np) {
            const int logp = lr * s;
            T.w[s - 1] = tw[(i & ((1 << logp) - 1)) << (logN - logp - lr + shift)];
        }
    }
    const int logp = lr * np;
    const int NB = r ? (N >> r) : 0;
#pragma unroll
    for (int q = 0; q < RB / 2; ++q) {
        const int iq = i + q * blockDim.x;
        T.wl[q] = make_double2(1.0, 0.0);
        if (r && q < (RB >> r) && iq < NB) T.wl[q] = tw[(iq & ((1 << logp) - 1)) << (logN - logp - r + shift)];
    }
    return T;
}

// The RB entries b + t*S of a thread's butterfly, read from or written to LDS
// (constant offsets from one swizzled base where pr_linear(S)).
template <int RB>
__device__ __forceinline__ void lds_read(double2 (&u)[RB], const double2* x, int b, int S)
{
    if (pr_linear<RB>(S)) {
        const double2* xb = x + Pr<RB>(b);
#pragma unroll
        for (int t = 0; t < RB; ++t) u[t] = xb[t * S];
    } else {
#pragma unroll
        for (int t = 0; t < RB; ++t) u[t] = x[Pr<RB>(b + t * S)];
    }
}
template <int RB>
__device__ __forceinline__ void lds_write(double2* x, const double2 (&u)[RB], int b, int S)
{
    if (pr_linear<RB>(S)) {
        double2* xb = x + Pr<RB>(b);
#pragma unroll
        for (int t = 0; t < RB; ++t) xb[t * S] = u[t];
    } else {
#pragma unroll
        for (int t = 0; t < RB; ++t) x[Pr<RB>(b + t * S)] = u[t];
    }
}

// Block-wide in-place FFT of length N = 2^logN (16 <= N <= 8192) held in LDS
// at padded positions Pr<RB>(j): Stockham passes of radix RB (16 or 8), one
// butterfly per thread in registers, then one radix-2/4/8 pass for the
// remaining factor.  Needs blockDim.x >= N/RB.
//   DIR = -1:  X_j = sum_k x_k exp(-2 pi i j k / N)
//   DIR = +1:  X_j = sum_k x_k exp(+2 pi i j k / N)   (no 1/N)
// T: the thread's twiddle bases for this N.  With post != nullptr the result is
// X_j * post[j].  st: the final store (see PlainStore); with a Store other than
// PlainStore, post is not applied.  ld: the first load (see PlainLoad).
template <int DIR, int RB, class Store = PlainStore, class Load = PlainLoad>
__device__ __forceinline__ void block_fft(double2* x, int N, int logN, const FftTw<RB>& T,
                                          const double2* __restrict__ post = nullptr, const Store& st = Store(),
                                          const Load& ld = Load())
{
    constexpr bool plain = std::is_same_v<Store, PlainStore>;
    constexpr bool plain_ld = std::is_same_v<Load, PlainLoad>;
    constexpr bool reg_ld = is_reg_load<Load>::value;
    constexpr int lr = (RB == 16) ? 4 : 3;
    const int i = threadIdx.x;
    const int np = logN / lr;        // main passes (at most 4 for N <= 8192)
    const int r = logN - lr * np;    // final radix 2^r, none when r = 0
    int p = 1;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (s >= np) break;
        const int NB = N >> lr;
        double2 u[RB];
        const int k = i & (p - 1);
        // with no final radix-2/4/8 pass, the last main pass applies post, its
        // factors read ahead of the pass (as in last_pass)
        const bool fold_post = plain && post && r == 0 && s == np - 1;
        double2 pv[RB];
        if (RB == 8 && fold_post && i < NB) {
            const int j = ((i - k) << lr) + k;
#pragma unroll
            for (int t = 0; t < RB; ++t) pv[t] = post[j + t * p];
        }
        if (i < NB) {
            if constexpr (reg_ld) {
                if (s == 0) {
#pragma unroll
                    for (int t = 0; t < RB; ++t) u[t] = ld.f(t, i + t * NB);
                } else if constexpr (RB == 8) {
                    lds_read<RB>(u, x, i, NB);
                } else {
#pragma unroll
                    for (int t = 0; t < RB; ++t) u[t] = x[Pr<RB>(i + t * NB)];
                }
            } else if (!plain_ld && s == 0) {
#pragma unroll
                for (int t = 0; t < RB; ++t) u[t] = ld(i + t * NB);
            } else if constexpr (RB == 8) {
                lds_read<RB>(u, x, i, NB);
            } else {
#pragma unroll
                for (int t = 0; t < RB; ++t) u[t] = x[Pr<RB>(i + t * NB)];
            }
            if (s > 0) {   // the first pass has k = 0: no twiddles
                double2 w = T.w[s > 0 ? s - 1 : 0];
                if (DIR > 0) w = cconj(w);
                twiddle_powers<RB>(u, w);
            }
            if constexpr (RB == 16) dft16<DIR>(u);
            else dft8<DIR>(u);
        }
        __syncthreads();
        if (i < NB) {
            const int j = ((i - k) << lr) + k;
            if (!plain && r == 0 && s == np - 1) {   // the last pass: outputs through st
#pragma unroll
                for (int t = 0; t < RB; ++t) st(j + t * p, u[t]);
            } else if constexpr (RB == 8) {
                if (fold_post) {
#pragma unroll
                    for (int t = 0; t < RB; ++t) u[t] = cmul(u[t], pv[t]);
                }
                lds_write<RB>(x, u, j, p);
            } else if (fold_post) {
#pragma unroll
                for (int t = 0; t < RB; ++t) x[Pr<RB>(j + t * p)] = cmul(u[t], post[j + t * p]);
            } else {
#pragma unroll
                for (int t = 0; t < RB; ++t) x[Pr<RB>(j + t * p)] = u[t];
            }
        }
        p <<= lr;
        __syncthreads();
    }
    if (r == 1) last_pass<DIR, 2, RB>(x, N, p, T.wl, post, st);
    else if (r == 2) last_pass<DIR, 4, RB>(x, N, p, T.wl, post, st);
    else if constexpr (RB == 16) {
        if (r == 3) last_pass<DIR, 8, RB>(x, N, p, T.wl, post, st);
    }
}

// Bluestein DFT of length N1 of the chirped, zero-padded sequence a_j already in
// x[P(j)], j < N2: on return x[P(k)] * chirp[k] = sum_j a_j exp(-2 pi i j k / N1), k < N1.
template <int RB>
__device__ __forceinline__ void bluestein_core(double2* x, const Plan& p, const FftTw<RB>& T)
{
    block_fft<-1, RB>(x, p.N2, p.logN2, T, p.bhat);
    block_fft<+1, RB>(x, p.N2, p.logN2, T);
}

// The same with the first load ld (see PlainLoad: ld(j) returns the chirped,
// zero-padded input a_j, j < N2) and the final store st (see PlainStore:
// st(k, X_k) receives the output before the chirp, k < N2).
template <int RB, class Load, class Store = PlainStore>
__device__ __forceinline__ void bluestein_core(double2* x, const Plan& p, const FftTw<RB>& T, const Load& ld,
                                               const Store& st = Store())
{
    block_fft<-1, RB>(x, p.N2, p.logN2, T, p.bhat, PlainStore(), ld);
    block_fft<+1, RB>(x, p.N2, p.logN2, T, nullptr, st);
}

// Split plans (N2 = 2 NH larger than the LDS holds, L > 2048): the N2-point
// transforms of a convolution run as two NH-point convolutions, one per parity
// of the frequency index (decimation in frequency).  With w = exp(-2 pi i/N2)
// and an input a_j that vanishes for j >= NH,
//   even:  E = IFFT_NH( FFT_NH(a_j)      * K[2k'] )
//   odd:   O = IFFT_NH( FFT_NH(a_j w^j)  * K[2k'+1] )
//   y_n = E_n + w^{-n} O_n   (n < NH),
// where K is the kernel spectrum, stored de-interleaved by the plan (even
// frequencies first, then odd).  NH = RB * blockDim.x: each thread holds RB
// values of a vector, those at j = threadIdx.x + q*blockDim.x.
//
// Bluestein DFT of length N1 <= NH on a split plan: lde(j) / ldo(j) (or
// RegLoad forms) give the first-pass inputs a_j and a_j w^j; on return
// x[Pr(n)] = y_n for n < NH, the same values bluestein_core leaves for n < N1.
template <int RB, class LdE, class LdO>
__device__ __forceinline__ void bluestein_split(double2* x, const Plan& p, const FftTw<RB>& T, const LdE& lde,
                                                const LdO& ldo)
{
    const int NH = p.N2 >> 1, logNH = p.logN2 - 1;
    block_fft<-1, RB>(x, NH, logNH, T, p.bhat, PlainStore(), lde);
    block_fft<+1, RB>(x, NH, logNH, T);
    double2 e[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) e[q] = x[Pr<RB>(threadIdx.x + q * blockDim.x)];
    block_fft<-1, RB>(x, NH, logNH, T, p.bhat + NH, PlainStore(), ldo);   // begins with a barrier
    block_fft<+1, RB>(x, NH, logNH, T);
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        const int j = threadIdx.x + q * blockDim.x;
        x[Pr<RB>(j)] = cadd(e[q], cmul(cconj(p.tw[j]), x[Pr<RB>(j)]));
    }
    __syncthreads();
}

// Kernels compiled for one transform length: LOGN = log2 of the length held in
// LDS (N2, or N2/2 on a split plan), -1 for any length.  With a fixed length the
// pass count, strides and guards of every transform are compile-time constants.
template <int LOGN, bool SP>
__device__ __forceinline__ void fix_length(Plan& p)
{
    if constexpr (LOGN > 0) {
        p.logN2 = LOGN + (SP ? 1 : 0);
        p.N2 = 1 << p.logN2;
    }
}

// Twiddle bases of a kernel's FFTs: length N2, or NH = N2/2 on a split plan.
template <int RB, bool SP>
__device__ __forceinline__ FftTw<RB> plan_twiddles(const Plan& p)
{
    if constexpr (SP) return fft_twiddles<RB>(p.N2 >> 1, p.logN2 - 1, p.tw, 1);
    else return fft_twiddles<RB>(p.N2, p.logN2, p.tw);
}

// Bluestein DFT of length N1 of the input ld(j) (zero for j >= N1) on either
// kind of plan; on return x[Pr(k)] * chirp[k] = sum_j a_j exp(-2 pi i j k/N1), k < N1.
template <int RB, bool SP, class Load>
__device__ __forceinline__ void bluestein_any(double2* x, const Plan& p, const FftTw<RB>& T, const Load& ld)
{
    if constexpr (SP) bluestein_split<RB>(x, p, T, ld, [&](int j) { return cmul(ld(j), p.tw[j]); });
    else bluestein_core<RB>(x, p, T, ld);
}

// XCD-aware column index: consecutive workgroups are dealt round-robin over the
// 8 XCDs; give each XCD a contiguous range of columns so neighbouring columns
// (which share cache lines of the row-major intermediates) meet in one L2.
__device__ __forceinline__ int xcd_column(int ncol)
{
    const int per = (ncol + 7) >> 3;
    const int b = blockIdx.x;
    return (b & 7) * per + (b >> 3);
}

// e^{i s phi_p} = e^{2 pi i s p/N1}, the angle reduced exactly modulo N1.
__device__ __forceinline__ double2 spin_phase(int s, int pp, int N1)
{
    int r = (int)(((long long)s * pp) % N1);
    if (r < 0) r += N1;
    double sn, cs;
    sincospi(2.0 * (double)r / (double)N1, &sn, &cs);
    return make_double2(cs, sn);
}

// ---------------------------------------------------------------------------
// Forward phi stage (Sec. IV-D): G_m(theta_t) = sc sum_p f(t, p) e^{-i m phi_p}, with
// sc = 2pi/N1 for the forward transform and sc = 1 for the adjoint of the inverse.
// Output order-major, G[m + L-1][t], so that the theta stage reads each order's
// column as one contiguous row; rings are dealt to XCDs in contiguous ranges,
// so the L2 of one XCD merges the partial lines that neighbouring rings write.
// pole: how the south-pole ring t = L-1 is read (Sec. IV-C counts it as one
// sample): 0 = a full ring of the map; 1 = compact storage, the ring being the
// one stored sample C = f(pi, 0) times e^{i s phi_p} (the form of every
// band-limited spin-s map at theta = pi, where only m = s survives);
// 2 = C at p = 0 and zeros elsewhere (the adjoint of keeping only p = 0).
template <int REAL, int RB, bool SP, int LOGN>
__global__ __launch_bounds__(512) void k_phi_forward(Plan p, Batch B, double sc, int pole)
{
    fix_length<LOGN, SP>(p);
    extern __shared__ double2 A[];
    const void* __restrict__ map = B.in[blockIdx.y];
    double2* __restrict__ G = (double2*)B.out[blockIdx.y];
    const int L = p.L, N1 = p.N1;
    const int t = xcd_column(L);
    if (t >= L) return;
    const bool pring = pole != 0 && t == L - 1;
    const int s = B.s[blockIdx.y];
    // twiddle bases of all FFTs below, read before the first pass (it needs none)
    const FftTw<RB> T = plan_twiddles<RB, SP>(p);
    // up to N2 = 1024: the output chirp factors read ahead (N1 < N2/2 =
    // (RB/2) blockDim.x); measured neutral at N2 = 2048, and at 4096 their
    // registers cost the workgroup its second slot on a compute unit
    constexpr bool AH = RB == 8 && LOGN > 0 && LOGN <= 10;
    constexpr int QA = AH ? RB / 2 : 1;
    Ahead<QA, double2> ca;
    if constexpr (AH) ca = read_ahead<QA>(N1, [&](int k) { return p.chirp[k]; });
    // the ring's samples, chirped and zero-padded, read by the first pass; the
    // outputs are stored from LDS in batches (written straight from the last pass,
    // the stride-L stores of G were measured slower)
    bluestein_any<RB, SP>(A, p, T, [&](int j) {
        if (j >= N1) return make_double2(0.0, 0.0);
        const size_t at = (size_t)t * N1 + (pring ? 0 : j);
        double2 a = REAL ? make_double2(((const double*)map)[at], 0.0) : ((const double2*)map)[at];
        if (pring) a = (pole == 1) ? cmul(a, spin_phase(s, j, N1)) : (j == 0 ? a : make_double2(0.0, 0.0));
        return cmul(a, p.chirp[j]);
    });
    auto out = [&](int k, double2 c) {
        const int m = (k <= L - 1) ? k : k - N1;
        G[(size_t)(m + L - 1) * L + t] = cscale(cmul(A[Pr<RB>(k)], c), sc);
    };
    if constexpr (AH) use_ahead<QA>(N1, ca, out);
    else staged_loop(N1, [&](int k) { return p.chirp[k]; }, out);
}

// Forward phi stage of a real map for the rings t1 = 2c and t2 = 2c+1 together:
// the spectrum of a real ring is Hermitian (Sec. IV-G), so one DFT X of
// x_p = f(t1, p) + i f(t2, p) gives both, G1_m = (X_m + conj(X_{-m}))/2 and
// G2_m = (X_m - conj(X_{-m}))/(2i).  Half the transforms of k_phi_forward for
// real maps; full rings only (pole = 0).  Output as k_phi_forward.
template <int RB, int LOGN>
__global__ __launch_bounds__(512) void k_phi_forward_real2(Plan p, Batch B, double sc)
{
    fix_length<LOGN, false>(p);
    extern __shared__ double2 A[];
    const double* __restrict__ map = (const double*)B.in[blockIdx.y];
    double2* __restrict__ G = (double2*)B.out[blockIdx.y];
    const int L = p.L, N1 = p.N1;
    const int npair = (L + 1) >> 1;
    const int c = xcd_column(npair);
    if (c >= npair) return;
    const int t1 = 2 * c, t2 = 2 * c + 1;
    const bool has2 = t2 < L;
    const FftTw<RB> T = plan_twiddles<RB, false>(p);
    bluestein_any<RB, false>(A, p, T, [&](int j) {
        if (j >= N1) return make_double2(0.0, 0.0);
        const double a = map[(size_t)t1 * N1 + j];
        const double b = has2 ? map[(size_t)t2 * N1 + j] : 0.0;
        return cmul(make_double2(a, b), p.chirp[j]);
    });
    const double h = 0.5 * sc;
    for (int k = threadIdx.x; k < N1; k += blockDim.x) {
        const int kn = (k == 0) ? 0 : N1 - k;
        const double2 x = cmul(A[Pr<RB>(k)], p.chirp[k]);        // X_k
        const double2 y = cconj(cmul(A[Pr<RB>(kn)], p.chirp[kn]));   // conj(X_{-k})
        const int m = (k <= L - 1) ? k : k - N1;
        double2* __restrict__ row = G + (size_t)(m + L - 1) * L;
        row[t1] = make_double2(h * (x.x + y.x), h * (x.y + y.y));
        if (has2) row[t2] = make_double2(h * (x.y - y.y), -h * (x.x - y.x));   // (x - y)/(2i)
    }
}

// Forward theta stage for order m (Sec. IV-B..IV-D):
//   extension  Gext(theta_t) = (-1)^{m+s} G_m(theta_{2L-2-t}) for t >= L,
//   F_{m m'} = 1/(2 pi N1) sum_t Gext(theta_t) e^{-i m' theta_t},
//   G_{m m'} = 2 pi sum_{m''} F_{m m''} w(m'' - m')  (product on the N2 grid),
//   fold     H_{m,0} = G_{m,0},  H_{m,n} = G_{m,n} + (-1)^{m+s} G_{m,-n}  (Eq.(Fmm_sym1)).
// Output: Hp records (see mw_internal.h); order m writes its slot of row |m|,
// including the zero pad entry n = L when L is odd.
// ADJ_INV = 1 gives the theta step of the adjoint of the inverse transform
// instead: Z_{m m'} = sum_{t<L} G_m(theta_t) e^{-i m' theta_t} (the conjugate
// transpose of Eq.(Fmt): no extension, no 1/(2 pi N1), no weights), folded the
// same way, because the adjoint's contraction is the forward's.
// OUT32 = 1 writes H in FP32 at [(|m|*4 + comp)*Lp + n] instead, comp = (Re, Im)
// of sigma_+(n) H_{m,n} (m >= 0) and of sigma_-(n) H_{-m,n} (m <= 0), with the
// parity split of the contraction folded in: sigma_+ = (-1)^n for s >= 0 and
// sigma_- = (-1)^n for s < 0 (1 otherwise).
// HALF = 1 (real scalar maps, Sec. IV-G): only the orders m >= 0 run; the map
// being real, G_{-m}(theta) = conj(G_m(theta)) and hence H_{-m,n} =
// (-1)^{m+s} conj(H_{m,n}), which order m writes into the -m half of its row.
//
// Split plans (L > 2048): the Bluestein step and the weight step run as pairs of
// half-length convolutions (bluestein_split); the weight step's N2-grid input
// lies in [0, L) (m' >= 0) and [N2 - L + 1, N2) (m' < 0), so its two halves do
// not overlap and fold onto one half grid, and the fold of the output is split
// in the same way: H_n = P_n + w^n O_n - (-1)^{m+s} w^{NH-n} O_{NH-n} with
// P_n = E_n + (-1)^{m+s} E_{NH-n} from the even pass (P_0 = E_0, H_0 = P_0 + O_0).
template <int ADJ_INV, int OUT32, int HALF, int RB, bool SP, int LOGN>
__global__ __launch_bounds__(512) void k_theta_forward(Plan p, Batch B)
{
    fix_length<LOGN, SP>(p);
    extern __shared__ double2 A[];
    const int s = B.s[blockIdx.y];
    const double2* __restrict__ G = (const double2*)B.in[blockIdx.y];
    void* __restrict__ Hout = B.out[blockIdx.y];
    const int L = p.L, N1 = p.N1, N2 = p.N2;
    // columns interleave +m and -m (c = 0, 1, 2, ... -> m = 0, 1, -1, 2, -2, ...), so
    // the two workgroups that write the halves of one row of H records share an XCD
    const int c = HALF ? xcd_column(L) : xcd_column(N1);
    if (c >= (HALF ? L : N1)) return;
    const int mi = HALF ? c + (L - 1) : ((c & 1) ? (L - 1) + ((c + 1) >> 1) : (L - 1) - (c >> 1));
    const int m = mi - (L - 1);
    const double sig = ((m + s) & 1) ? -1.0 : 1.0;
    // twiddle bases of all FFTs below, read before the first pass (it needs none)
    const FftTw<RB> T = plan_twiddles<RB, SP>(p);
    // the extended column (t < L as given, then (-1)^{m+s} times the mirror image;
    // the adjoint of the inverse has no extension), chirped and zero-padded
    auto ld = [&](int j) {
        if (j >= N1) return make_double2(0.0, 0.0);
        double2 a = make_double2(0.0, 0.0);
        if (j < L) a = G[(size_t)mi * L + j];
        else if (!ADJ_INV) a = cscale(G[(size_t)mi * L + (2 * L - 2 - j)], sig);
        return cmul(a, p.chirp[j]);
    };
    const int am = m < 0 ? -m : m;
    // output of order m for n < Lp (pad entry n = L of odd L: v = 0)
    auto store = [&](int n, double2 v) {
        // the -m half: H_{-m,n} itself, or (-1)^{m+s} conj(H_{m,n}) for a real map
        const double2 vm = HALF ? cscale(cconj(v), sig) : v;
        const bool pos = m >= 0, neg = HALF || m <= 0;
        if (OUT32) {
            float* h = (float*)Hout + (size_t)am * 4 * p.Lp + n;
            const double par = (n & 1) ? -1.0 : 1.0;
            if (pos) {
                const double sg = (s >= 0) ? par : 1.0;
                h[0] = (float)(sg * v.x);
                h[(size_t)p.Lp] = (float)(sg * v.y);
            }
            if (neg) {
                const double sg = (s < 0) ? par : 1.0;
                h[2 * (size_t)p.Lp] = (float)(sg * vm.x);
                h[3 * (size_t)p.Lp] = (float)(sg * vm.y);
            }
        } else {
            double* rec = (double*)Hout + ((size_t)am * p.Lp + n) * 4;
            if (pos) { rec[0] = v.x; rec[1] = v.y; }
            if (neg) { rec[2] = vm.x; rec[3] = vm.y; }
        }
    };
    if constexpr (SP && !ADJ_INV) {
        const int NH = N2 >> 1, logNH = p.logN2 - 1;
        const double scale = p.thsc;
        bluestein_split<RB>(A, p, T, ld, [&](int j) { return cmul(ld(j), p.tw[j]); });
        // the weight step's input on the half grid: F_{m'} for m' = j (j < L) and
        // m' = j - NH (j > NH - L), Bluestein output k = j or j - NH + N1
        double2 v[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int j = threadIdx.x + q * blockDim.x;
            const int k = (j < L) ? j : (j > NH - L) ? j - NH + N1 : -1;
            v[q] = (k >= 0) ? cscale(cmul(A[Pr<RB>(k)], p.thwc[k]), scale) : make_double2(0.0, 0.0);
        }
        // even frequencies (block_fft begins with a barrier: the reads above are done)
        block_fft<+1, RB>(A, NH, logNH, T, p.what, PlainStore(), reg_load([&](int t, int) { return v[t]; }));
        block_fft<-1, RB>(A, NH, logNH, T);
        double2 P[RB / 2];   // n = threadIdx.x + q*blockDim.x < L <= NH/2
#pragma unroll
        for (int q = 0; q < RB / 2; ++q) {
            const int n = threadIdx.x + q * blockDim.x;
            P[q] = make_double2(0.0, 0.0);
            if (n < L) {
                P[q] = A[Pr<RB>(n)];
                if (n > 0) P[q] = cadd(P[q], cscale(A[Pr<RB>(NH - n)], sig));
            }
        }
        // odd frequencies: input (c_lo - c_hi)_j w^{-j}
        block_fft<+1, RB>(A, NH, logNH, T, p.what + NH, PlainStore(), reg_load([&](int t, int j) {
                              const double2 c = cmul(v[t], cconj(p.tw[j]));
                              return (j < L) ? c : cscale(c, -1.0);
                          }));
        block_fft<-1, RB>(A, NH, logNH, T);
#pragma unroll
        for (int q = 0; q < RB / 2; ++q) {
            const int n = threadIdx.x + q * blockDim.x;
            if (n < p.Lp) {
                double2 h = make_double2(0.0, 0.0);
                if (n == 0) {
                    h = cadd(P[q], A[Pr<RB>(0)]);
                } else if (n < L) {
                    h = cadd(P[q], cmul(p.tw[n], A[Pr<RB>(n)]));
                    h = csub(h, cscale(cmul(p.tw[NH - n], A[Pr<RB>(NH - n)]), sig));
                }
                store(n, h);
            }
        }
        return;
    }
    int wrap = N2;   // index of -n is wrap - n
    if constexpr (ADJ_INV) {
        bluestein_any<RB, SP>(A, p, T, ld);
        // F_{m'} = chirp_k e^{-i m' pi/N1} times the Bluestein output, k < N1
        constexpr int Q = SP ? RB : 8;   // N1 <= Q * blockDim.x
        double2 r[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int k = threadIdx.x + q * blockDim.x;
            if (k < N1) r[q] = cmul(A[Pr<RB>(k)], p.thwc[k]);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int k = threadIdx.x + q * blockDim.x;
            if (k < N1) A[Pr<RB>(k)] = r[q];
        }
        __syncthreads();
        wrap = N1;
    } else if constexpr (!SP) {
        // Bluestein with its last store fused with the move onto the N2 grid:
        // output k < N1 is F_{m'} / (chirp_k e^{-i m' pi/N1} / (2 pi N1)) and goes to
        // slot m' mod N2 (m' = k, or k - N1 for k >= L); outputs k >= N1 are not
        // needed and their slots k - N1 + L fill the zeros in between (a bijection).
        const double scale = p.thsc;
        block_fft<-1, RB>(A, N2, p.logN2, T, p.bhat, PlainStore(), ld);
        block_fft<+1, RB>(A, N2, p.logN2, T, nullptr, [&](int k, double2 v) {
            if (k < N1) A[Pr<RB>(k < L ? k : k + (N2 - N1))] = cscale(cmul(v, p.thwc[k]), scale);
            else A[Pr<RB>(k - N1 + L)] = make_double2(0.0, 0.0);
        });
        block_fft<+1, RB>(A, N2, p.logN2, T, p.what);
        block_fft<-1, RB>(A, N2, p.logN2, T);
    }
    for (int n = threadIdx.x; n < p.Lp; n += blockDim.x) {
        double2 v = make_double2(0.0, 0.0);
        if (n < L) {
            v = A[Pr<RB>(n)];
            if (n > 0) v = cadd(v, cscale(A[Pr<RB>(wrap - n)], sig));
        }
        store(n, v);
    }
}

// Forward theta stage for a pair of orders with extensions of opposite parity
// (Sec. IV-B..IV-D): the order a with (-1)^{m_a+s} = +1 extends its column
// symmetrically about theta = pi, the order b antisymmetrically, so the DFT of
// their sum splits into a symmetric part (a's F_{m'}) and an antisymmetric part
// (b's F_{m'}, without b's pole sample, whose DFT is symmetric and is added
// separately).  The fold H_n = G_n + (-1)^{m+s} G_{-n} of a symmetric or
// antisymmetric F keeps only the even part w_e of the weights, so one
// correlation with w_e serves both orders:  Y = 2 pi sum_k F_k w_e(k - n),
//   H^a_0 = Y_0,  H^a_n = Y_n + Y_{-n},  H^b_n = Y_n - Y_{-n}  (n >= 1),
// and b's pole sample P = G^b(theta_{L-1}) and the odd weights w(+-1) enter
// only H^b_0 = 2 pi^2 i (F_1 - F_{-1})/2 + P sum_{|k|<L} w_e(k)/N1 and
// H^b_{L-1} += -i pi (-1)^L P/N1.  One Bluestein DFT and one correlation per
// two orders instead of two of each.  Pairs: (m, -m-1), m = 0..L-2, and L-1
// alone; real maps (HALF): (2c, 2c+1), only the orders m >= 0.
template <int OUT32, int HALF, int RB, int LOGN>
__global__ __launch_bounds__(512) void k_theta_forward_pair(Plan p, Batch B)
{
    fix_length<LOGN, false>(p);
    extern __shared__ double2 A[];
    __shared__ double2 f1[2];   // F_{+1} and F_{-1} of the packed column
    const int s = B.s[blockIdx.y];
    const double2* __restrict__ G = (const double2*)B.in[blockIdx.y];
    void* __restrict__ Hout = B.out[blockIdx.y];
    const int L = p.L, N1 = p.N1, N2 = p.N2;
    const int npair = HALF ? (L + 1) >> 1 : L;
    const int c = xcd_column(npair);
    if (c >= npair) return;
    const int m1 = HALF ? 2 * c : c, m2 = HALF ? 2 * c + 1 : -(c + 1);
    const bool has2 = HALF ? (m2 < L) : (c < L - 1);
    const bool m1sym = ((m1 + s) & 1) == 0;
    const int ma = m1sym ? m1 : m2, mb = m1sym ? m2 : m1;
    const bool hasa = m1sym || has2, hasb = !m1sym || has2;
    const double2* __restrict__ Ga = G + (size_t)(ma + L - 1) * L;
    const double2* __restrict__ Gb = G + (size_t)(mb + L - 1) * L;
    const FftTw<RB> T = plan_twiddles<RB, false>(p);
    // b's pole sample (used by the fold below), read before the transforms
    const double2 P = hasb ? Gb[L - 1] : make_double2(0.0, 0.0);
    // the packed extended column, chirped and zero-padded
    auto ld = [&](int j) {
        if (j >= N1) return make_double2(0.0, 0.0);
        double2 v = make_double2(0.0, 0.0);
        if (j < L) {
            if (hasa) v = Ga[j];
            if (hasb && j != L - 1) v = cadd(v, Gb[j]);
        } else {
            const int t = 2 * L - 2 - j;
            if (hasa) v = Ga[t];
            if (hasb) v = csub(v, Gb[t]);
        }
        return cmul(v, p.chirp[j]);
    };
    const double scale = p.thsc;
    block_fft<-1, RB>(A, N2, p.logN2, T, p.bhat, PlainStore(), ld);
    block_fft<+1, RB>(A, N2, p.logN2, T, nullptr, [&](int k, double2 v) {
        if (k < N1) {
            const double2 f = cscale(cmul(v, p.thwc[k]), scale);
            A[Pr<RB>(k < L ? k : k + (N2 - N1))] = f;
            if (k == 1) f1[0] = f;
            if (k == N1 - 1) f1[1] = f;
        } else {
            A[Pr<RB>(k - N1 + L)] = make_double2(0.0, 0.0);
        }
    });
    block_fft<+1, RB>(A, N2, p.logN2, T, p.whate);
    block_fft<-1, RB>(A, N2, p.logN2, T);
    // the odd-weight term of H^b_0 (L >= 2: with L = 1 the only order is 0 and
    // the pair has no b unless s is odd; then F_{+-1} = 0)
    const double2 b1 = (L >= 2) ? cscale(csub(f1[0], f1[1]), 0.5) : make_double2(0.0, 0.0);
    const double PI2 = 9.8696044010893586188;   // pi^2
    const double sgnL = (L & 1) ? -1.0 : 1.0;
    auto put = [&](int m, int n, double2 v) {
        const double sig = ((m + s) & 1) ? -1.0 : 1.0;
        const int am = m < 0 ? -m : m;
        // the -m half: H_{-m,n} itself, or (-1)^{m+s} conj(H_{m,n}) for a real map
        const double2 vm = HALF ? cscale(cconj(v), sig) : v;
        const bool pos = m >= 0, neg = HALF || m <= 0;
        if (OUT32) {
            float* h = (float*)Hout + (size_t)am * 4 * p.Lp + n;
            const double par = (n & 1) ? -1.0 : 1.0;
            if (pos) {
                const double sg = (s >= 0) ? par : 1.0;
                h[0] = (float)(sg * v.x);
                h[(size_t)p.Lp] = (float)(sg * v.y);
            }
            if (neg) {
                const double sg = (s < 0) ? par : 1.0;
                h[2 * (size_t)p.Lp] = (float)(sg * vm.x);
                h[3 * (size_t)p.Lp] = (float)(sg * vm.y);
            }
        } else {
            double* rec = (double*)Hout + ((size_t)am * p.Lp + n) * 4;
            if (pos) { rec[0] = v.x; rec[1] = v.y; }
            if (neg) { rec[2] = vm.x; rec[3] = vm.y; }
        }
    };
    for (int n = threadIdx.x; n < p.Lp; n += blockDim.x) {
        double2 ha = make_double2(0.0, 0.0), hb = make_double2(0.0, 0.0);
        if (n == 0) {
            ha = A[Pr<RB>(0)];
            // 2 pi (i pi/2)(F_1 - F_{-1}) + P sum w_e / N1
            hb = cadd(make_double2(-2.0 * PI2 * b1.y, 2.0 * PI2 * b1.x), cscale(P, p.wsum_e / (double)N1));
        } else if (n < L) {
            const double2 yp = A[Pr<RB>(n)], ym = A[Pr<RB>(N2 - n)];
            ha = cadd(yp, ym);
            hb = csub(yp, ym);
            if (n == L - 1) {   // -i pi (-1)^L P / N1
                const double f = 3.14159265358979323846 * sgnL / (double)N1;
                hb = cadd(hb, make_double2(f * P.y, -f * P.x));
            }
        }
        if (hasa) put(ma, n, ha);
        if (hasb) put(mb, n, hb);
    }
}

// Inverse theta stage for a pair of orders of opposite parity (Eq.(Fmt)): the
// unfolded F_{m,m'} of order a is symmetric in m' and that of order b
// antisymmetric (Eq.(Fmm_sym1); its m' = 0 entry vanishes), so
// F_a(theta) + F_b(theta) over the whole period gives both orders:
// F_a(theta_t) = (x_t + x_{2L-2-t})/2 and F_b(theta_t) = (x_t - x_{2L-2-t})/2
// for t < L-1 (theta_{2L-2-t} = 2 pi - theta_t), F_a = x_{L-1} and F_b = 0 at the
// pole.  One Bluestein DFT per two orders.  Pairs as in k_theta_forward_pair.
template <int HALF, int RB, int LOGN>
__global__ __launch_bounds__(512) void k_theta_inverse_pair(Plan p, Batch B)
{
    fix_length<LOGN, false>(p);
    extern __shared__ double2 A[];
    const int s = B.s[blockIdx.y];
    const double2* __restrict__ F = (const double2*)B.in[blockIdx.y];
    double2* __restrict__ Ft = (double2*)B.out[blockIdx.y];
    const int L = p.L, N1 = p.N1;
    const int npair = HALF ? (L + 1) >> 1 : L;
    const int c = xcd_column(npair);
    if (c >= npair) return;
    const int m1 = HALF ? 2 * c : c, m2 = HALF ? 2 * c + 1 : -(c + 1);
    const bool has2 = HALF ? (m2 < L) : (c < L - 1);
    const bool m1sym = ((m1 + s) & 1) == 0;
    const int ma = m1sym ? m1 : m2, mb = m1sym ? m2 : m1;
    const bool hasa = m1sym || has2, hasb = !m1sym || has2;
    const int ia = ma + L - 1, ib = mb + L - 1;
    const double2* __restrict__ Fa = F + (size_t)ia * L;
    const double2* __restrict__ Fb = F + (size_t)ib * L;
    const FftTw<RB> T = plan_twiddles<RB, false>(p);
    // up to N2 = 2048 (radix 8, at most 256 threads): the output chirp factors
    // read ahead (L <= N2/4 = (RB/4) blockDim.x)
    constexpr bool AH = RB == 8 && LOGN > 0 && LOGN <= 11;
    constexpr int QA = AH ? RB / 4 : 1;
    auto chirps = [&](int t) { return Pair2{p.chirp[t], p.chirp[2 * L - 2 - t]}; };
    Ahead<QA, Pair2> ca;
    if constexpr (AH) ca = read_ahead<QA>(L, chirps);
    bluestein_core<RB>(A, p, T, [&](int j) {   // conj of the packed unfolded F times e^{-i m' pi/N1} chirp_j
        if (j >= N1) return make_double2(0.0, 0.0);
        const int mp = (j <= L - 1) ? j : j - N1;
        const int n = mp < 0 ? -mp : mp;
        double2 f = make_double2(0.0, 0.0);
        if (hasa) f = Fa[n];
        if (hasb && n > 0) f = (mp < 0) ? csub(f, Fb[n]) : cadd(f, Fb[n]);
        return cmul(cconj(f), p.thwc[j]);
    });
    auto out = [&](int t, const Pair2& cp) {
        const double2 x = cconj(cmul(A[Pr<RB>(t)], cp.a));
        if (t == L - 1) {
            if (hasa) Ft[(size_t)t * N1 + ia] = x;
            if (hasb) Ft[(size_t)t * N1 + ib] = make_double2(0.0, 0.0);
        } else {
            const double2 y = cconj(cmul(A[Pr<RB>(2 * L - 2 - t)], cp.b));
            if (hasa) Ft[(size_t)t * N1 + ia] = cscale(cadd(x, y), 0.5);
            if (hasb) Ft[(size_t)t * N1 + ib] = cscale(csub(x, y), 0.5);
        }
    };
    if constexpr (AH) use_ahead<QA>(L, ca, out);
    else staged_loop(L, chirps, out);
}

// Theta step of the adjoint of the forward transform, for order m: the
// conjugate transposes of the forward's theta stages in reverse order.
//   unfold   Y_{m,-n} = (-1)^{m+s} Y_{m,n}     (input: folded Y[m + L-1][n], n >= 0)
//   weights  Z_{m m''} = 2 pi sum_{m'} conj(w(m'' - m')) Y_{m m'}
//            (the forward's N2-grid product with conj of its weight spectrum)
//   DFT^H    Gext(theta_t) = 1/(2 pi N1) sum_{m''} Z_{m m''} e^{+i m'' theta_t}, t < N1
//   fold     G_m(theta_t) = Gext(theta_t) + (-1)^{m+s} Gext(theta_{2L-2-t}), t < L-1;
//            G_m(theta_{L-1}) = Gext(theta_{L-1})
// Output G[t][m + L-1] (the layout the inverse phi stage reads).
// Split plans (L > 2048): the correlation runs as its even- and odd-frequency
// halves on the half grid (see k_theta_forward), its output at slot j of the half
// grid being E_j + w^j O_j (m' = j >= 0) or E_j - w^j O_j (m' = j - NH < 0), and
// the Bluestein step as bluestein_split on inputs held in registers.
template <int RB, bool SP, int LOGN>
__global__ __launch_bounds__(512) void k_theta_forward_adjoint(Plan p, Batch B)
{
    fix_length<LOGN, SP>(p);
    extern __shared__ double2 A[];
    const int s = B.s[blockIdx.y];
    const double2* __restrict__ Y = (const double2*)B.in[blockIdx.y];
    double2* __restrict__ Gt = (double2*)B.out[blockIdx.y];
    const int L = p.L, N1 = p.N1, N2 = p.N2;
    const int mi = xcd_column(N1);
    if (mi >= N1) return;
    const int m = mi - (L - 1);
    const double sig = ((m + s) & 1) ? -1.0 : 1.0;
    auto finish = [&]() {   // the Bluestein output in A: fold back onto t < L
        staged_loop(
            L, [&](int t) { return Pair2{p.chirp[t], p.chirp[2 * L - 2 - t]}; },
            [&](int t, const Pair2& c) {
                double2 v = cconj(cmul(A[Pr<RB>(t)], c.a));
                if (t <= L - 2) v = cadd(v, cscale(cconj(cmul(A[Pr<RB>(2 * L - 2 - t)], c.b)), sig));
                Gt[(size_t)t * N1 + mi] = v;
            });
    };
    if constexpr (SP) {
        const int NH = N2 >> 1, logNH = p.logN2 - 1;
        const FftTw<RB> T = plan_twiddles<RB, SP>(p);
        // the unfolded Y on the half grid: m' = j (j < L) or j - NH (j > NH - L)
        auto ldY = [&](int j) {
            const int mp = (j < L) ? j : (j > NH - L) ? j - NH : NH;
            if (mp == NH) return make_double2(0.0, 0.0);
            const double2 y = Y[(size_t)mi * L + (mp < 0 ? -mp : mp)];
            return (mp < 0) ? cscale(y, sig) : y;
        };
        block_fft<+1, RB>(A, NH, logNH, T, p.whatc, PlainStore(), ldY);
        block_fft<-1, RB>(A, NH, logNH, T);
        double2 e[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) e[q] = A[Pr<RB>(threadIdx.x + q * blockDim.x)];
        block_fft<+1, RB>(A, NH, logNH, T, p.whatc + NH, PlainStore(), [&](int j) {
            const double2 c = cmul(ldY(j), cconj(p.tw[j]));
            return (j < L) ? c : cscale(c, -1.0);
        });
        block_fft<-1, RB>(A, NH, logNH, T);
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int j = threadIdx.x + q * blockDim.x;
            const double2 o = cmul(p.tw[j], A[Pr<RB>(j)]);
            A[Pr<RB>(j)] = (j < L) ? cadd(e[q], o) : csub(e[q], o);
        }
        __syncthreads();
        // Z_{m''} conj(thtw), conjugated and chirped (the Bluestein input, k < N1)
        double2 r[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int k = threadIdx.x + q * blockDim.x;
            r[q] = make_double2(0.0, 0.0);
            if (k < N1) {
                const int mp = (k <= L - 1) ? k : k - N1;
                const double2 y = cmul(A[Pr<RB>((mp + NH) & (NH - 1))], cconj(p.thtw[k]));
                r[q] = cmul(cconj(y), p.chirp[k]);
            }
        }
        bluestein_split<RB>(A, p, T, reg_load([&](int t, int) { return r[t]; }),
                            reg_load([&](int t, int j) { return cmul(r[t], p.tw[j]); }));
        finish();
        return;
    }
    for (int j = threadIdx.x; j < N2; j += blockDim.x) A[Pr<RB>(j)] = make_double2(0.0, 0.0);
    __syncthreads();
    staged_loop(
        N1,
        [&](int k) {
            const int mp = (k <= L - 1) ? k : k - N1;
            return Y[(size_t)mi * L + (mp < 0 ? -mp : mp)];
        },
        [&](int k, double2 y) {
            const int mp = (k <= L - 1) ? k : k - N1;
            A[Pr<RB>((mp + N2) & (N2 - 1))] = (mp < 0) ? cscale(y, sig) : y;
        });
    // twiddle bases of all FFTs below, read while the first pass runs (it needs none)
    const FftTw<RB> T = fft_twiddles<RB>(p.N2, p.logN2, p.tw);
    block_fft<+1, RB>(A, N2, p.logN2, T, p.whatc);
    block_fft<-1, RB>(A, N2, p.logN2, T);
    // Z_{m''} e^{+i m'' pi/N1}/(2 pi N1) = Z conj(thtw), conjugated and chirped for the
    // Bluestein evaluation of the positive-exponent DFT
    double2 r[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = threadIdx.x + q * blockDim.x;
        if (k < N1) {
            const int mp = (k <= L - 1) ? k : k - N1;
            const double2 y = cmul(A[Pr<RB>((mp + N2) & (N2 - 1))], cconj(p.thtw[k]));
            r[q] = cmul(cconj(y), p.chirp[k]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int k = threadIdx.x + q * blockDim.x;
        if (k < N2) A[Pr<RB>(k)] = (k < N1) ? r[q] : make_double2(0.0, 0.0);
    }
    for (int j = threadIdx.x + 8 * blockDim.x; j < N2; j += blockDim.x) A[Pr<RB>(j)] = make_double2(0.0, 0.0);
    bluestein_core<RB>(A, p, T);
    finish();
}

// Inverse theta stage for order m (Sec. IV-E, Eq.(Fmt)):
//   F_m(theta_t) = sum_{m'} F_{m m'} e^{i m' theta_t}, t < L only,
// from the folded F[m + L-1][n] (n >= 0) with F_{m,-n} = (-1)^{m+s} F_{m,n}.
// Output Ft[t][m + L-1].
// HALF = 1 (real scalar maps): only the orders m >= 0 run; the inverse phi stage
// takes F_{-m}(theta) = conj(F_m(theta)).
template <int HALF, int RB, bool SP, int LOGN>
__global__ __launch_bounds__(512) void k_theta_inverse(Plan p, Batch B)
{
    fix_length<LOGN, SP>(p);
    extern __shared__ double2 A[];
    const int s = B.s[blockIdx.y];
    const double2* __restrict__ F = (const double2*)B.in[blockIdx.y];
    double2* __restrict__ Ft = (double2*)B.out[blockIdx.y];
    const int L = p.L, N1 = p.N1, N2 = p.N2;
    const int mi = HALF ? xcd_column(L) + (L - 1) : xcd_column(N1);
    if (mi >= N1) return;
    const int m = mi - (L - 1);
    const double sig = ((m + s) & 1) ? -1.0 : 1.0;
    // twiddle bases of all FFTs below, read before the first pass (it needs none)
    const FftTw<RB> T = plan_twiddles<RB, SP>(p);
    auto ld = [&](int j) {   // the unfolded F_{mm'}, m' = j or j - N1, as conj(f e^{+i m' pi/N1}) chirp_j
        if (j >= N1) return make_double2(0.0, 0.0);
        const int mp = (j <= L - 1) ? j : j - N1;
        double2 f = F[(size_t)mi * L + (mp < 0 ? -mp : mp)];
        if (mp < 0) f = cscale(f, sig);
        return cmul(cconj(f), p.thwc[j]);   // thwc_j = e^{-i m' pi/N1} chirp_j
    };
    if constexpr (SP) {
        bluestein_split<RB>(A, p, T, ld, [&](int j) { return cmul(ld(j), p.tw[j]); });
        staged_loop(
            L, [&](int t) { return p.chirp[t]; },
            [&](int t, double2 c) { Ft[(size_t)t * N1 + mi] = cconj(cmul(A[Pr<RB>(t)], c)); });
    } else {
        bluestein_core<RB>(A, p, T, ld, [&](int t, double2 v) {   // outputs t < L, straight to Ft
            if (t < L) Ft[(size_t)t * N1 + mi] = cconj(cmul(v, p.chirp[t]));
        });
    }
}

// Inverse phi stage (Eq.(f_pfft)): f(t, p) = sc sum_m F_m(theta_t) e^{i m phi_p}, with
// sc = 1 for the inverse transform and sc = 2pi/N1 for the adjoint of the forward
// (whose phi step is the conjugate transpose of the forward's).  REAL = 1 stores
// Re f; REAL = 2 (real scalar maps) reads the orders m >= 0 only, takes
// F_{-m} = conj(F_m) and stores f, which is then real.
// pole: how the south-pole ring t = L-1 is stored: 0 = in full; 1 = compact
// storage, its sample p = 0 only; 2 = the single value sum_p e^{-i s phi_p} f(L-1, p)
// at p = 0 (the adjoint of the compact expansion C -> C e^{i s phi_p}).
template <int REAL, int RB, bool SP, int LOGN>
__global__ __launch_bounds__(512) void k_phi_inverse(Plan p, Batch B, double sc, int pole)
{
    fix_length<LOGN, SP>(p);
    extern __shared__ double2 A[];
    const double2* __restrict__ Ft = (const double2*)B.in[blockIdx.y];
    void* __restrict__ map = B.out[blockIdx.y];
    const int L = p.L, N1 = p.N1;
    const int t = xcd_column(L);
    if (t >= L) return;
    // twiddle bases of all FFTs below, read before the first pass (it needs none)
    const FftTw<RB> T = plan_twiddles<RB, SP>(p);
    auto ld = [&](int j) {   // conj(F_m) chirp_j, m = j or j - N1 (F_m = conj(F_{-m}) for REAL = 2)
        if (j >= N1) return make_double2(0.0, 0.0);
        const int m = (j <= L - 1) ? j : j - N1;
        const double2 a = Ft[(size_t)t * N1 + ((REAL == 2 && m < 0 ? -m : m) + L - 1)];
        const bool neg = REAL == 2 && m < 0;
        return cmul(neg ? a : cconj(a), p.chirp[j]);
    };
    auto value = [&](int k, double2 v) {   // output k < N1 (v before the chirp)
        const double2 out = cscale(cconj(cmul(v, p.chirp[k])), sc);
        return REAL ? make_double2(out.x, 0.0) : out;
    };
    auto put = [&](int k, double2 v) {
        const double2 out = value(k, v);
        if (REAL) ((double*)map)[(size_t)t * N1 + k] = out.x;
        else ((double2*)map)[(size_t)t * N1 + k] = out;
    };
    if (pole != 0 && t == L - 1) {   // the pole ring of compact storage
        bluestein_any<RB, SP>(A, p, T, ld);
        if (pole == 1) {
            if (threadIdx.x == 0) put(0, A[Pr<RB>(0)]);
            return;
        }
        // sum_p e^{-i s phi_p} f_p: per-thread partial sums, then thread 0 adds
        // them in thread order (fixed order)
        const int s = B.s[blockIdx.y];
        double2 acc = make_double2(0.0, 0.0);
        for (int k = threadIdx.x; k < N1; k += blockDim.x)
            acc = cadd(acc, cmul(value(k, A[Pr<RB>(k)]), cconj(spin_phase(s, k, N1))));
        __syncthreads();
        A[threadIdx.x] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double2 tot = A[0];
            for (int i = 1; i < (int)blockDim.x; ++i) tot = cadd(tot, A[i]);
            if (REAL) ((double*)map)[(size_t)t * N1] = tot.x;
            else ((double2*)map)[(size_t)t * N1] = tot;
        }
        return;
    }
    if constexpr (SP) {
        bluestein_split<RB>(A, p, T, ld, [&](int j) { return cmul(ld(j), p.tw[j]); });
        for (int k = threadIdx.x; k < N1; k += blockDim.x) put(k, A[Pr<RB>(k)]);
    } else {
        bluestein_core<RB>(A, p, T, ld, [&](int k, double2 v) {   // outputs k < N1, straight to the map
            if (k < N1) put(k, v);
        });
    }
}

// Inverse phi stage of a real map (orders m >= 0 stored, F_{-m} = conj(F_m),
// Sec. IV-G) for the rings t1 = 2c and t2 = 2c+1 together: one inverse DFT of
// Y_m = F1_m + i F2_m (each F extended to m < 0 by conjugation) gives
// f(t1, p) + i f(t2, p), both real.  Half the transforms of k_phi_inverse<2>;
// full rings only (pole = 0).
template <int RB, int LOGN>
__global__ __launch_bounds__(512) void k_phi_inverse_real2(Plan p, Batch B, double sc)
{
    fix_length<LOGN, false>(p);
    extern __shared__ double2 A[];
    const double2* __restrict__ Ft = (const double2*)B.in[blockIdx.y];
    double* __restrict__ map = (double*)B.out[blockIdx.y];
    const int L = p.L, N1 = p.N1;
    const int npair = (L + 1) >> 1;
    const int c = xcd_column(npair);
    if (c >= npair) return;
    const int t1 = 2 * c, t2 = 2 * c + 1;
    const bool has2 = t2 < L;
    const FftTw<RB> T = plan_twiddles<RB, false>(p);
    // conj(Y_m) chirp_j: with F1 = (a1, b1), F2 = (a2, b2) at |m|,
    // conj(F1) - i conj(F2) = (a1 - b2, -b1 - a2) for m >= 0 and
    // F1 - i F2 = (a1 + b2, b1 - a2) for m < 0.  At m = 0 only the real parts
    // enter, as in k_phi_inverse<2>, which stores the real part of the
    // synthesis: f = Re F_0 + 2 sum_{m>0} Re(F_m e^{i m phi}) for any input.
    bluestein_core<RB>(A, p, T, [&](int j) {
        if (j >= N1) return make_double2(0.0, 0.0);
        const int m = (j <= L - 1) ? j : j - N1;
        const int am = m < 0 ? -m : m;
        double2 f1 = Ft[(size_t)t1 * N1 + am + L - 1];
        double2 f2 = has2 ? Ft[(size_t)t2 * N1 + am + L - 1] : make_double2(0.0, 0.0);
        if (am == 0) { f1.y = 0.0; f2.y = 0.0; }
        const double2 y = (m >= 0) ? make_double2(f1.x - f2.y, -f1.y - f2.x) : make_double2(f1.x + f2.y, f1.y - f2.x);
        return cmul(y, p.chirp[j]);
    }, [&](int k, double2 v) {   // outputs k < N1: conj(v chirp_k) sc = f(t1, k) + i f(t2, k)
        if (k < N1) {
            const double2 o = cconj(cmul(v, p.chirp[k]));
            map[(size_t)t1 * N1 + k] = sc * o.x;
            if (has2) map[(size_t)t2 * N1 + k] = sc * o.y;
        }
    });
}

// Main radix of the FFTs for a plan.  It depends on the band-limit only, so a
// map's result does not depend on the batch it runs in.  Radix 8 runs twice the
// threads per transform of radix 16 for the same work; both keep a workgroup
// within the kernels' 512-thread launch bound (radix 8 up to N2 = 4096).  Split
// plans (N2 above the 8192-point transforms the LDS holds) run their
// half-length transforms in radix 16 with one butterfly per thread, NH / 16
// threads (512 at L = 4096; every thread holds RB values of a half-length vector).
bool fft_split(const Plan& p) { return p.split; }

int fft_radix(const Plan& p)
{
    if (fft_split(p)) return 16;
    return (p.N2 / 8 <= 512) ? 8 : 16;
}

// Length of the transforms a kernel runs in LDS: N2, or N2/2 on a split plan.
int fft_len(const Plan& p) { return fft_split(p) ? p.N2 / 2 : p.N2; }

// Threads per FFT workgroup: one main-pass butterfly each (length/rb <= 512,
// the kernels' launch bound), at least one wavefront.
int fft_threads(const Plan& p, int rb)
{
    int t = fft_len(p) / rb;
    if (t < 64) t = 64;
    return t;
}

size_t fft_lds(const Plan& p, int rb)
{
    const int n = fft_len(p);
    return (size_t)(n + (rb == 8 ? 0 : n / rb)) * sizeof(double2);
}

template <class K>
hipError_t set_lds(K kernel, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

int xcd_grid(int ncol) { return 8 * ((ncol + 7) >> 3); }

template <class K, class... Args>
hipError_t fft_go(K k, const Plan& p, int rb, dim3 grid, hipStream_t st, Args... args)
{
    hipError_t e;
    if ((e = set_lds(k, fft_lds(p, rb))) != hipSuccess) return e;
    hipLaunchKernelGGL(k, grid, dim3(fft_threads(p, rb)), fft_lds(p, rb), st, args...);
    return hipGetLastError();
}

// Launches kernel K<RB, SP, LOGN> with the radix and split mode of the plan,
// compiled for its transform length when that is one of the common ones
// (512 .. 8192 points in LDS: band-limits 65 .. 4096), else for any length.
template <template <int, bool, int> class KS, class... Args>
hipError_t fft_launch(const Plan& p, dim3 grid, hipStream_t st, Args... args)
{
    const int logn = fft_split(p) ? p.logN2 - 1 : p.logN2;
    if (fft_split(p)) {
        if (logn == 13) return fft_go(KS<16, true, 13>::fn(), p, 16, grid, st, args...);
        return fft_go(KS<16, true, -1>::fn(), p, 16, grid, st, args...);
    }
    if (fft_radix(p) == 16) {
        if (logn == 13) return fft_go(KS<16, false, 13>::fn(), p, 16, grid, st, args...);
        return fft_go(KS<16, false, -1>::fn(), p, 16, grid, st, args...);
    }
    switch (logn) {
        case 7: return fft_go(KS<8, false, 7>::fn(), p, 8, grid, st, args...);
        case 8: return fft_go(KS<8, false, 8>::fn(), p, 8, grid, st, args...);
        case 9: return fft_go(KS<8, false, 9>::fn(), p, 8, grid, st, args...);
        case 10: return fft_go(KS<8, false, 10>::fn(), p, 8, grid, st, args...);
        case 11: return fft_go(KS<8, false, 11>::fn(), p, 8, grid, st, args...);
        case 12: return fft_go(KS<8, false, 12>::fn(), p, 8, grid, st, args...);
        default: return fft_go(KS<8, false, -1>::fn(), p, 8, grid, st, args...);
    }
}

// The same for kernels that exist only for split plans (KS<16, true, LOGN>) ...
template <template <int, bool, int> class KS, class... Args>
hipError_t fft_launch_split(const Plan& p, dim3 grid, hipStream_t st, Args... args)
{
    if (p.logN2 - 1 == 13) return fft_go(KS<16, true, 13>::fn(), p, 16, grid, st, args...);
    return fft_go(KS<16, true, -1>::fn(), p, 16, grid, st, args...);
}

// ... and for those that exist only for unsplit plans (KS<RB, LOGN>).
template <template <int, int> class KS, class... Args>
hipError_t fft_launch_unsplit(const Plan& p, dim3 grid, hipStream_t st, Args... args)
{
    const int logn = p.logN2;
    if (fft_radix(p) == 16) {
        if (logn == 13) return fft_go(KS<16, 13>::fn(), p, 16, grid, st, args...);
        return fft_go(KS<16, -1>::fn(), p, 16, grid, st, args...);
    }
    switch (logn) {
        case 7: return fft_go(KS<8, 7>::fn(), p, 8, grid, st, args...);
        case 8: return fft_go(KS<8, 8>::fn(), p, 8, grid, st, args...);
        case 9: return fft_go(KS<8, 9>::fn(), p, 8, grid, st, args...);
        case 10: return fft_go(KS<8, 10>::fn(), p, 8, grid, st, args...);
        case 11: return fft_go(KS<8, 11>::fn(), p, 8, grid, st, args...);
        case 12: return fft_go(KS<8, 12>::fn(), p, 8, grid, st, args...);
        default: return fft_go(KS<8, -1>::fn(), p, 8, grid, st, args...);
    }
}

template <int O, int H> struct ThFP {
    template <int RB, int LN> struct K { static auto fn() { return k_theta_forward_pair<O, H, RB, LN>; } };
};
template <int H> struct ThIP {
    template <int RB, int LN> struct K { static auto fn() { return k_theta_inverse_pair<H, RB, LN>; } };
};

template <int RB, int LN> struct PhiF2 { static auto fn() { return k_phi_forward_real2<RB, LN>; } };
template <int RB, int LN> struct PhiI2 { static auto fn() { return k_phi_inverse_real2<RB, LN>; } };
template <int REAL> struct PhiF {
    template <int RB, bool SP, int LN> struct K { static auto fn() { return k_phi_forward<REAL, RB, SP, LN>; } };
};
template <int REAL> struct PhiI {
    template <int RB, bool SP, int LN> struct K { static auto fn() { return k_phi_inverse<REAL, RB, SP, LN>; } };
};
template <int A, int O, int H> struct ThF {
    template <int RB, bool SP, int LN> struct K {
        static auto fn() { return k_theta_forward<A, O, H, RB, SP, LN>; }
    };
};
template <int H> struct ThI {
    template <int RB, bool SP, int LN> struct K { static auto fn() { return k_theta_inverse<H, RB, SP, LN>; } };
};
template <int RB, bool SP, int LN> struct ThFA { static auto fn() { return k_theta_forward_adjoint<RB, SP, LN>; } };

}  // namespace

hipError_t launch_phi_forward(const Plan& p, const Batch& B, int real, double sc, int pole, hipStream_t st)
{
    if (real && pole == 0 && !fft_split(p))   // two real rings per transform
        return fft_launch_unsplit<PhiF2>(p, dim3(xcd_grid((p.L + 1) / 2), B.n), st, p, B, sc);
    const dim3 grid(xcd_grid(p.L), B.n);
    if (real) return fft_launch<PhiF<1>::K>(p, grid, st, p, B, sc, pole);
    return fft_launch<PhiF<0>::K>(p, grid, st, p, B, sc, pole);
}

hipError_t launch_theta_forward(const Plan& p, const Batch& B, int out32, int half, hipStream_t st)
{
    if (!fft_split(p)) {   // pairs of orders of opposite extension parity
        const dim3 grid(xcd_grid(half ? (p.L + 1) / 2 : p.L), B.n);
        if (half) {
            if (out32) return fft_launch_unsplit<ThFP<1, 1>::K>(p, grid, st, p, B);
            return fft_launch_unsplit<ThFP<0, 1>::K>(p, grid, st, p, B);
        }
        if (out32) return fft_launch_unsplit<ThFP<1, 0>::K>(p, grid, st, p, B);
        return fft_launch_unsplit<ThFP<0, 0>::K>(p, grid, st, p, B);
    }
    const dim3 grid(xcd_grid(half ? p.L : p.N1), B.n);
    if (half) {
        if (out32) return fft_launch_split<ThF<0, 1, 1>::K>(p, grid, st, p, B);
        return fft_launch_split<ThF<0, 0, 1>::K>(p, grid, st, p, B);
    }
    if (out32) return fft_launch_split<ThF<0, 1, 0>::K>(p, grid, st, p, B);
    return fft_launch_split<ThF<0, 0, 0>::K>(p, grid, st, p, B);
}

hipError_t launch_theta_inverse_adjoint(const Plan& p, const Batch& B, int out32, hipStream_t st)
{
    const dim3 grid(xcd_grid(p.N1), B.n);
    if (out32) return fft_launch<ThF<1, 1, 0>::K>(p, grid, st, p, B);
    return fft_launch<ThF<1, 0, 0>::K>(p, grid, st, p, B);
}

hipError_t launch_theta_forward_adjoint(const Plan& p, const Batch& B, hipStream_t st)
{
    return fft_launch<ThFA>(p, dim3(xcd_grid(p.N1), B.n), st, p, B);
}

hipError_t launch_theta_inverse(const Plan& p, const Batch& B, int half, hipStream_t st)
{
    if (!fft_split(p)) {   // pairs of orders of opposite extension parity
        const dim3 grid(xcd_grid(half ? (p.L + 1) / 2 : p.L), B.n);
        if (half) return fft_launch_unsplit<ThIP<1>::K>(p, grid, st, p, B);
        return fft_launch_unsplit<ThIP<0>::K>(p, grid, st, p, B);
    }
    if (half) return fft_launch_split<ThI<1>::K>(p, dim3(xcd_grid(p.L), B.n), st, p, B);
    return fft_launch_split<ThI<0>::K>(p, dim3(xcd_grid(p.N1), B.n), st, p, B);
}

hipError_t launch_phi_inverse(const Plan& p, const Batch& B, int real, double sc, int pole, hipStream_t st)
{
    if (real == 2 && pole == 0 && !fft_split(p))   // two real rings per transform
        return fft_launch_unsplit<PhiI2>(p, dim3(xcd_grid((p.L + 1) / 2), B.n), st, p, B, sc);
    const dim3 grid(xcd_grid(p.L), B.n);   // rings dealt to XCDs in contiguous ranges
    if (real == 2) return fft_launch<PhiI<2>::K>(p, grid, st, p, B, sc, pole);
    if (real) return fft_launch<PhiI<1>::K>(p, grid, st, p, B, sc, pole);
    return fft_launch<PhiI<0>::K>(p, grid, st, p, B, sc, pole);
}

}  // namespace mw
