// Internal declarations shared by the libmw sources (host plan, kernels, C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace mw {

// Chains whose start value lies below 2^-EXT_LIMIT are carried with an extra
// binary exponent in steps of 2^EXT_STEP (see the contraction kernels).
constexpr int EXT_STEP = 600;
constexpr int EXT_LIMIT = 900;

// Waves per contraction workgroup = maximum number of segments of one chain:
// SEG_MAX for the forward row recursions, SEGI_MAX for the inverse degree
// recursions.  Eight inverse segments were measured slower than four: the
// extra restarts cost more than the added waves hide.
constexpr int SEG_MAX = 4;
constexpr int SEGI_MAX = 4;
// The FP64 inverse over the triangle n >= m (half the chains of the square
// kernels) splits its chains into up to SEGT_MAX segments, one wave each.
// Eight segments were measured slower than four at L = 512 (47 against 41 us):
// more restarts and more waves than fit at once.
constexpr int SEGT_MAX = 4;
// Complex maps use the triangle kernel from this band-limit up (real maps at
// every band-limit); below, the square kernels.
constexpr int INV_TRI_MIN_L = 1024;
// Real maps from this band-limit up read their spin values from the scaled spin
// rows in the triangle kernel (below, they run a third chain).
constexpr int INV_TRI_SPT_MIN_L = 1024;
// The forward contractions (FP64 and mixed) read their spin rows from the spin
// tables from this band-limit up (below, they run them as chains).
constexpr int FWD_SPT_MIN_L = 1024;
// Test hook (mw_profile_inverse_triangle): 1 runs every FP64 inverse on the
// triangle kernel.
extern int g_inv_tri_all;
// Checkpoint planes of the inverse: at most CKI_MAX - 1 of them.
constexpr int CKI_MAX = 16;

// Order-major index of the triangle l >= m of an L x L table (see Plan::edgem).
__host__ __device__ inline size_t tri_m(int m, int l, int L)
{
    return (size_t)m * L - (size_t)m * (m - 1) / 2 + (size_t)(l - m);
}

// Band-limit-dependent constants, built once per (device, L) on the host in
// long double and uploaded.  All device pointers are owned by the plan.
struct Plan {
    int L = 0, N1 = 0, N2 = 0, logN2 = 0;
    int Lp = 0;              // L rounded up to even (row length of the forward H layout)
    // The Fourier kernels run their N2-point transforms as pairs of N2/2-point
    // ones (N2 above what the LDS holds, or forced by mw_profile_split_fft).
    bool split = false;
    bool ext = false;        // some start value needs the exponent extension
    // Wigner tables
    double* rtab = nullptr;     // rtab[j] = 1/sqrt(j-1) for j >= 2, rtab[0] = rtab[1] = 0; 2L+8 entries
    // Chain start values, order-major and square: at [m*L + n] the value of
    // Delta^{l0}_{n,m} at l0 = max(n, m), i.e. (-1)^(n-m) Delta^n_{m,n} for n >= m
    // and Delta^m_{n,m} for n < m (edge values, Delta^l_{m,l} = 2^-l sqrt(C(2l, l+m))),
    // as mantissa * 2^(EXT_STEP*k).  64 consecutive n (or l) of one order are one
    // contiguous read.
    double* edge = nullptr;
    int* edgek = nullptr;       // k of each entry
    double2* lco = nullptr;     // scaled l-recursion factor and scale (Pu'_m(l), h_m(l)) at [m*Lp + l]
    double* cl = nullptr;       // sqrt((2l+1)/(4 pi))
    // Fourier tables
    double2* tw = nullptr;      // exp(-2 pi i e/N2), e < N2
    double2* chirp = nullptr;   // exp(-i pi j^2/N1), j < N1
    // The three spectra below are stored in frequency order, or for split plans
    // even frequencies first, then odd ones (the half-length convolutions).
    double2* bhat = nullptr;    // FFT_N2 of the Bluestein kernel, divided by N2
    double2* what = nullptr;    // (2 pi/N2) * DFT_N2 of the theta weights w(k)
    double2* whatc = nullptr;   // conj(what), for the adjoint of the weight step
    double2* whate = nullptr;   // (2 pi/N2) * DFT_N2 of the even part of the weights (frequency order)
    double wsum_e = 0.0;        // sum of the even part of the weights over |k| <= L-1
    double2* thtw = nullptr;    // exp(-i m' pi/N1)/(2 pi N1) at slot k = m' mod N1
    double2* thwc = nullptr;    // exp(-i m' pi/N1) chirp_k at slot k = m' mod N1
    double thsc = 0.0;          // 1/(2 pi N1)
    // Work list of the forward contractions (FP64 and mixed), dealt over the 8
    // XCDs: SEG_MAX wave slots per workgroup, slot i of workgroup g at
    // [g*SEG_MAX + i] = (l0, mb, seg | nseg << 8 | lead << 16 | barrier << 24,
    // lo | hi << 16) for segment seg, rows [lo, hi), of the chain group (degrees
    // l0 .., orders mb, mb+1) whose nseg segments sit in slots lead ..
    // lead+nseg-1 of the same workgroup; (-1, 0, barrier << 24, 0) marks an empty
    // slot
    int4* workf4 = nullptr; int nworkf4 = 0;   // workgroups
    // Chain segmentation: each chain group splits its chain into at most
    // SEG_MAX / SEGI_MAX segments, choosing the boundaries among checkpoint
    // planes on a grid finer than the segments (forward_work, inverse_work).
    // The forward's planes lie at rows n = j*ckfg (j = 1..nckf-1); ckf holds,
    // for plane j at [(j-1)*L(L+1)/2 + tri_m(m, l)], the pair
    // (Delta^l_{m,n-1}, Delta^l_{m,n}) as mantissas with exponent levels ckfk.
    // The inverse's planes lie at degrees c = k*ckg (k = 1..nck-1); cki holds,
    // for plane k, the pair (Delta^{c-1}_{n,m}, Delta^{c}_{n,m}) at
    // cki_off[k] + m*(c+1) + n (n, m <= c), with levels ckik.  segf, segi: the
    // segment lengths the grids derive from.
    int segf = 0, nsegf = 1, segi = 0, nsegi = 1;
    int ckg = 0, nck = 1, ckfg = 0, nckf = 1;
    double2* ckf = nullptr; int2* ckfk = nullptr;
    double2* cki = nullptr; int2* ckik = nullptr;
    size_t cki_off[CKI_MAX] = {0};
    size_t bytes = 0;
};

// Spin-row start table for the inverse l-recursion: Delta^l_{n,|s|} at [l*L + n]
// (mantissa * 2^(EXT_STEP*k)), with its exponent level.  It also holds the
// work list of the FP64 inverse contraction, whose segmentation depends on |s|:
// SEGI_MAX wave slots per workgroup, slot i of workgroup g at [g*SEGI_MAX + i] =
// (n0, m0, seg | nseg << 8 | lead << 16 | barrier << 24, cs | ce << 16) for
// segment seg, degrees [cs, ce), of the chain group (n0 .. n0+63, orders m0,
// m0+1) whose nseg segments sit in slots lead .. lead+nseg-1 of the same
// workgroup (cs of a later segment is a checkpoint plane); (-1, 0, barrier << 24,
// 0) marks an empty slot.
//
// The FP64 inverse runs each chain Delta^l_{n,m} with n >= m once for the pairs
// (m, n) and (n, m) (Delta^l_{m,n} = (-1)^{m-n} Delta^l_{n,m}); its work list
// wtri holds only the chain groups that meet n >= m (n0 + 63 >= m0), in the
// layout of winv.  lcos[m*Lp + l] = (Pu'_m(l), c_l Delta^l_{m,|s|} / h_m(l)),
// c_l = sqrt((2l+1)/(4 pi)): the chain factor of order m and the factor of row
// m in the transposed sums (zero where |Delta^l_{m,|s|}| is below 2^-900 or
// l < max(m, |s|)).
struct SpinTable {
    int L = 0, as = 0;
    double* val = nullptr;
    int* k = nullptr;
    int4* winv = nullptr;
    int nwinv = 0;   // workgroups
    double2* lcos = nullptr;
    double* sval = nullptr;   // h_|s|(l) Delta^l_{n,|s|} at [l*L + n], l < Lp (the FP64 inverses' spin values)
    double* svalf = nullptr;  // Delta^l_{|s|,n} at [n*L + l], n < Lp (the FP64 forward's spin values)
    int4* wtri = nullptr;
    int nwtri = 0;   // workgroups
    size_t bytes = 0;
};

// Chains per lane in the contraction kernels (work-list granularity in m).
constexpr int MT_FWD = 2;

// Mixed-precision contraction: a group of up to GMAX maps shares the FP64 order
// chains; its maps have at most NSMAX different |s|, the spin rows of the launch
// (MixBatch::as, the same for all its groups).  src/dst are per-map device
// pointers (FP32 staged H or stream; f_lm or F), L the per-map band-limits
// (<= the plan's); meta packs the map count (bits 0-3), for each map b the row of
// its |s| (bit 4+b) and the sign of its spin (bit 12+b).  Passed by value (the
// launch's kernel arguments stay under 1.5 KB).
constexpr int GMAX = 8;
constexpr int NSMAX = 2;
struct MixMaps {
    const float* src[GMAX];
    double2* dst[GMAX];
    int L[GMAX];
    int meta;
};
__host__ __device__ inline int mix_n(const MixMaps& m) { return m.meta & 15; }
__host__ __device__ inline int mix_row(const MixMaps& m, int b) { return (m.meta >> (4 + b)) & 1; }
__host__ __device__ inline bool mix_neg(const MixMaps& m, int b) { return (m.meta >> (12 + b)) & 1; }
// Groups of one mixed launch (blockIdx.y = group), with their spin rows |s_j|,
// j < ns, and (inverse only) the spin tables Delta^l_{n,|s_j|} of those rows.
constexpr int MIXG = 8;
struct MixBatch {
    MixMaps g[MIXG];
    int ng;
    int ns;
    int as[NSMAX];
    const double* stab[NSMAX];
    const int* stabk[NSMAX];
    const double* ssv[NSMAX];   // inverse: the scaled spin rows of those tables (SpinTable::sval)
    const double* ssvf[NSMAX];  // forward: their transposed rows (SpinTable::svalf), or null
};
__host__ __device__ inline int mix_spin(const MixBatch& B, const MixMaps& m, int b)
{
    const int a = B.as[mix_row(m, b)];
    return mix_neg(m, b) ? -a : a;
}

// Maps of one batched launch (blockIdx.y, or z for 3-D grids, = map): per-map
// input and output device pointers and spins; all maps of a launch share the
// plan (band-limit).  Passed by value as a kernel argument.
constexpr int MAXB = 32;
struct Batch {
    const void* in[MAXB];
    void* out[MAXB];
    int s[MAXB];
    int n;
};

// Smallest N2 whose plans are split (plan_split_min): 16384 by default; 2048
// under the test hook mw_profile_split_fft(1).
extern int g_split_min_n2;
int build_plan(int L, Plan& p, std::string& err);
void free_plan(Plan& p);
int build_spin_table(const Plan& p, int as, SpinTable& t, std::string& err);
void free_spin_table(SpinTable& t);

// Kernel launchers (enqueue only); each runs the maps of B (one plan) in one launch.
// sc: 2 pi/N1 for the forward transform, 1 for the adjoint of the inverse.
// pole (compact storage of the south-pole ring, Sec. IV-C): 0 = full ring;
// 1 = expand the stored sample C to C e^{i s phi_p}; 2 = C at p = 0, zeros elsewhere.
hipError_t launch_phi_forward(const Plan& p, const Batch& B, int real, double sc, int pole, hipStream_t st);
// Forward theta stage.  Output: Hp records (Re H_{m,n}, Im H_{m,n}, Re H_{-m,n}, Im H_{-m,n})
// at [(m * Lp + n) * 4], m < L, n < Lp (pad rows zero); with out32 = 1 FP32 H at
// [(m*4 + comp)*Lp + n] with the parity signs folded (the mixed contraction's layout).
// half = 1: real scalar maps, only the orders m >= 0 run (the -m halves by symmetry).
hipError_t launch_theta_forward(const Plan& p, const Batch& B, int out32, int half, hipStream_t st);
// Theta step of the adjoint of the inverse (same output layouts as launch_theta_forward).
hipError_t launch_theta_inverse_adjoint(const Plan& p, const Batch& B, int out32, hipStream_t st);
// Theta step of the adjoint of the forward: folded Y (N1 x L) -> Gt (L x N1).
hipError_t launch_theta_forward_adjoint(const Plan& p, const Batch& B, hipStream_t st);
// FP64 contractions: map k of the launch reads in0 + k*stride (doubles; the
// chunk's workspace slots are equally spaced) and writes B.out[k].  real = 1
// (real scalar maps): the forward writes f_{l,-m} = (-1)^m conj(f_{l,m}) and the
// inverse writes only the orders m >= 0 of F.
hipError_t launch_contract_forward(const Plan& p, const SpinTable& sp, int s, int real, const double* in0,
                                   size_t stride, const Batch& B, hipStream_t st);
// Inverse coefficient stream (L x Lp x 4 doubles, or FP32 at [(m*4+comp)*Lp + l]),
// each map with its own spin B.s[k].
hipError_t launch_inverse_stream(const Plan& p, int real, const Batch& B, int out32, hipStream_t st);
// FP64 inverse contraction: map k reads the stream at in0 + k*stride (doubles)
// and its coefficients f_lm at B.in[k] (the transposed sums), and writes F to
// B.out[k].
hipError_t launch_contract_inverse(const Plan& p, const SpinTable& sp, int s, int real, const double* in0,
                                   size_t stride, const Batch& B, hipStream_t st);
// half = 1: real scalar maps, only the orders m >= 0 (for launch_phi_inverse with real = 2).
hipError_t launch_theta_inverse(const Plan& p, const Batch& B, int half, hipStream_t st);
// sc: 1 for the inverse transform, 2 pi/N1 for the adjoint of the forward.
// real: 0 complex output; 1 the real part of the full synthesis; 2 a real map
// synthesised from the orders m >= 0 with F_{-m} = conj(F_m).
// pole: 0 = full pole ring; 1 = its sample p = 0 only (compact storage);
// 2 = sum_p e^{-i s phi_p} f(L-1, p) at p = 0 (adjoint of the compact expansion).
hipError_t launch_phi_inverse(const Plan& p, const Batch& B, int real, double sc, int pole, hipStream_t st);
// Adjoint of the real-map coefficient expansion: y_{l,m} += (-1)^m conj(y_{l,-m}),
// y_{l,-m} = 0 for m > 0 (in place on the L^2 layout of B.out).
hipError_t launch_real_fold(int L, const Batch& B, hipStream_t st);
// Coefficients of the conjugate maps (spin -s) of the maps of B (spin B.s[k]):
// out_{l,m} = (-1)^{s+m} conj(in_{l,-m}); out may equal in.
hipError_t launch_spin_flip(int L, const Batch& B, hipStream_t st);
// Largest group size (1, 2 or 4) whose staging fits the LDS (independent of L).
int mix_group_max();
// Mixed-precision contractions of up to MIXG groups (each maps.n <= G <= GMAX, G
// in {1,2,4,8}; each with at most NS <= NSMAX spin rows).  The inverse runs the work
// list of wsp, the spin table of the largest |s| of the launch's groups.
hipError_t launch_contract_forward_mix(const Plan& p, const MixBatch& maps, int G, int NS, hipStream_t st);
hipError_t launch_contract_inverse_mix(const Plan& p, const SpinTable& wsp, const MixBatch& maps, int G, int NS,
                                       hipStream_t st);

// Explicit quadrature (mw_quad.hip): the weights q(theta_t), t < L, into q
// (device, L doubles); the integrals of the maps of B (B.in[k]: L x nphi map,
// float64 when real, else complex128; B.out[k]: one complex128), with partial
// (device, B.n * L complex) as scratch.
hipError_t launch_quad_weights(int L, int s, double* q, hipStream_t st);
hipError_t launch_integrate(int L, int nphi, int real, const Batch& B, double2* partial, hipStream_t st);

}  // namespace mw
