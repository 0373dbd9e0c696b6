// The O(L^3) part of the MW transforms: Wigner Delta = d(pi/2) generated on the
// fly in FP64 and contracted against the Fourier coefficients.
//
// Forward, Eq.(flm_wig) folded with Eq.(Fmm_sym1):
//   f_{l,+-m} = (-1)^s i^{+-m+s} sqrt((2l+1)/4pi) sum_{n>=0} Delta^l_{n,+-m} Delta^l_{n,-s} H_{+-m,n}
// A wavefront owns 64 consecutive degrees l (one per lane) and MT orders m.
// Each lane runs the three-term recursion of row m of Delta^l along the second
// index n = l .. 0 (the beta = pi/2 recursion family of Trapani & Navaza that
// the paper compares with Risbo's, Sec. V-C):
//   sqrt((l+n)(l-n+1)) D_{m,n-1} = -2m D_{m,n} - sqrt((l-n)(l+n+1)) D_{m,n+1},
// started from the edge value D_{m,l} = 2^-l sqrt(binom(2l, l+m)).  Row |s| (the
// spin factor) runs as one more chain in the same lane.  H_{+-m,n} is the same
// for every lane and arrives through scalar loads; the sum over n accumulates
// in registers.
//
// Inverse, Eq.(Fmm):
//   F_{+-m,n} = (-1)^s i^{-(+-m+s)} sum_l sqrt((2l+1)/4pi) Delta^l_{n,+-m} Delta^l_{n,-s} f_{l,+-m}
// A wavefront owns 64 consecutive n (one per lane) and one order m.  Each lane
// runs the three-term recursion of Delta^l_{n,m} upward in the degree l from
// l0 = max(n, m), so the sum over l again accumulates in registers; the spin
// factor Delta^l_{n,|s|} runs as a second chain, started from a table.
//
// Pipelining: steps run in pairs; the uniform data of pair k-1 (scalar loads)
// and the per-lane 1/sqrt factors of pair k-1 (vector loads from a small table)
// are issued before pair k is computed, after an explicit wait on pair k's data.
// Nothing in the loop touches LDS, so the scalar-load counter only tracks the
// scalar stream.
//
// Chains whose start value is below 2^-900 (only for L > ~900) carry an extra
// exponent: the stored value is x = D * 2^(600k); while k > 0 the chain's
// contributions are masked (|D| < 2^-300) and it is rescaled when |x| > 2^300.
#include <algorithm>

#include "mw_internal.h"

namespace mw {
namespace {

__device__ __forceinline__ double2 mul_ipow(double2 z, int k)
{
    switch (k & 3) {
        case 0: return z;
        case 1: return make_double2(-z.y, z.x);
        case 2: return make_double2(-z.x, -z.y);
        default: return make_double2(z.y, -z.x);
    }
}
__device__ __forceinline__ double sgn(int k) { return (k & 1) ? -1.0 : 1.0; }
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Makes the compiler wait for a scalar-loaded value here (and, scalar loads
// returning out of order, for every scalar load issued before it).
__device__ __forceinline__ void wait_scalar(double v) { asm volatile("" ::"s"(v)); }

constexpr double EXT_UP = 0x1p300;
constexpr double EXT_DOWN = 0x1p-600;

struct alignas(64) Rec8 { double v[8]; };    // 64-byte scalar-load unit

typedef double dv2 __attribute__((ext_vector_type(2)));
typedef float fv2 __attribute__((ext_vector_type(2)));

// 1/sqrt(i) for i = j-1 .. j, read from the shifted table Rt (Rt[j] = 1/sqrt(j-1),
// Rt[0] = Rt[1] = 0), so that indices below 0 read zeros.
__device__ __forceinline__ double2 rpair(const double* __restrict__ Rt, int j)
{
    // table base in scalar registers plus a 32-bit byte offset per lane (no
    // 64-bit address arithmetic in the vector unit)
    const char* base = (const char*)Rt;
    const unsigned off = (unsigned)j * 8u;
    double2 r;
    r.x = *(const double*)(base + off);
    r.y = *(const double*)(base + off + 8u);
    return r;
}

// ===========================================================================
// Forward contraction
// ===========================================================================
// The spin rows |s_j| a chain group runs: one for the FP64 kernels, up to two
// for mixed-precision groups whose maps have two different |s| (the order
// chains Delta_{m,n} are the same for every spin and shared; Sec. V notes that
// the Wigner values need not be recomputed per spin).
template <int NS>
struct SpinSet {
    int a[NS];
};

template <int MT, bool EXT, int NS = 1>
struct FwdLane {
    double dc[MT], dn[MT];         // D_{m,n} and D_{m,n+1}
    double sc[NS], sn[NS];         // spin rows |s_j|
    double2 ap[MT][2], am[MT][2];  // accumulators for +m / -m, split by parity of n
    int k[MT], ks[NS];             // exponent levels (EXT)
    double anext;                  // sqrt((l-n)(l+n+1)) of the current step
    double q, dq;                  // Q_n = (l+n)(l-n+1) and 2(n-1), exact in FP64
    double start[MT], starts[NS];
    int startk[MT], startks[NS];
};

// Chain starts of step n (lanes whose degree l equals n start from the edge).
template <int MT, bool EXT, bool INJ, int NS, bool SPT = false>
__device__ __forceinline__ void fwd_inject(FwdLane<MT, EXT, NS>& st, int n, int l, bool& anyscaled)
{
    if (INJ) {
        if (n == l) {
#pragma unroll
            for (int c = 0; c < MT; ++c) { st.dc[c] = st.start[c]; if (EXT) st.k[c] = st.startk[c]; }
            if constexpr (!SPT) {
#pragma unroll
                for (int j = 0; j < NS; ++j) { st.sc[j] = st.starts[j]; if (EXT) st.ks[j] = st.startks[j]; }
            }
        }
        if (EXT) {
            bool sc = false;
#pragma unroll
            for (int j = 0; j < NS; ++j) sc |= st.ks[j] > 0;
#pragma unroll
            for (int c = 0; c < MT; ++c) sc |= st.k[c] > 0;
            anyscaled = __any(sc);
        }
    }
}

// Recursion from step n to n-1 with ra = 1/sqrt(Q_n):
//   D_{n-1} = -(2m D_n + a_{n+1} D_{n+1}) / a_n,  a_n = sqrt(Q_n); harmless at n = 0.
// CHK: the exponent-extended state is checked (rescaled chains); once no lane of
// the wave holds a scaled chain and none can start one (past the chain starts),
// the steps run without the checks.
template <int MT, bool EXT, int NS, bool SPT = false, bool CHK = EXT>
__device__ __forceinline__ void fwd_advance(FwdLane<MT, EXT, NS>& st, int mb, const SpinSet<NS>& as, double ra,
                                            bool& anyscaled)
{
    const double an = st.q * ra;
    const double nra = -ra;
#pragma unroll
    for (int c = 0; c < MT; ++c) {
        const double tm = 2.0 * (double)(mb + c);
        const double d = fma(tm, st.dc[c], st.anext * st.dn[c]) * nra;
        st.dn[c] = st.dc[c];
        st.dc[c] = d;
    }
    if constexpr (!SPT) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const double d = fma(2.0 * (double)as.a[j], st.sc[j], st.anext * st.sn[j]) * nra;
            st.sn[j] = st.sc[j];
            st.sc[j] = d;
        }
    }
    st.anext = an;
    st.q += st.dq;          // Q_{n-1} = Q_n + 2(n-1)
    st.dq -= 2.0;
    if (CHK && anyscaled) {
        bool still = false;
#pragma unroll
        for (int c = 0; c < MT; ++c) {
            if (st.k[c] > 0 && fabs(st.dc[c]) > EXT_UP) {
                st.dc[c] *= EXT_DOWN; st.dn[c] *= EXT_DOWN; st.k[c] -= 1;
            }
            still |= st.k[c] > 0;
        }
        if constexpr (!SPT) {
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                if (st.ks[j] > 0 && fabs(st.sc[j]) > EXT_UP) { st.sc[j] *= EXT_DOWN; st.sn[j] *= EXT_DOWN; st.ks[j] -= 1; }
                still |= st.ks[j] > 0;
            }
        }
        anyscaled = __any(still);
    }
}

// Delta_{m_c,n} * Delta_{|s_j|,n} of the current step (0 while a chain is scaled).
template <int MT, bool EXT, int NS, bool CHK = EXT>
__device__ __forceinline__ double fwd_product(const FwdLane<MT, EXT, NS>& st, int c, int j = 0)
{
    double seff = st.sc[j];
    if (CHK) seff = (st.ks[j] == 0) ? seff : 0.0;
    double d = st.dc[c];
    if (CHK) d = (st.k[c] == 0) ? d : 0.0;
    return d * seff;
}

// One step n: contributions of D_{.,n} (h = the four doubles of H at n for
// each chain), then the recursion to n-1.  The spin row's value Delta^l_{|s|,n}
// at this step is sv, read from the spin table's transposed rows.
template <int MT, bool EXT, int PAR, bool INJ, bool RL, bool SPT, bool CHK = EXT>
__device__ __forceinline__ void fwd_step(FwdLane<MT, EXT>& st, int n, int l, int mb, int as,
                                         const Rec8 (&h)[MT], double ra, double sv, bool& anyscaled)
{
    fwd_inject<MT, EXT, INJ, 1, SPT>(st, n, l, anyscaled);
#pragma unroll
    for (int c = 0; c < MT; ++c) {
        const double* hc = h[c].v + 4 * PAR;
        double pr;
        if constexpr (SPT) {
            double d = st.dc[c];
            if (CHK) d = (st.k[c] == 0) ? d : 0.0;
            pr = d * sv;
        } else {
            pr = fwd_product<MT, EXT, 1, CHK>(st, c);
        }
        st.ap[c][PAR].x = fma(pr, hc[0], st.ap[c][PAR].x);
        st.ap[c][PAR].y = fma(pr, hc[1], st.ap[c][PAR].y);
        if (!RL) {   // real maps: f_{l,-m} follows from f_{l,m}
            st.am[c][PAR].x = fma(pr, hc[2], st.am[c][PAR].x);
            st.am[c][PAR].y = fma(pr, hc[3], st.am[c][PAR].y);
        }
    }
    fwd_advance<MT, EXT, 1, SPT, CHK>(st, mb, SpinSet<1>{{as}}, ra, anyscaled);
}

template <int MT>
__device__ __forceinline__ void fwd_load_h(Rec8 (&h)[MT], const double* __restrict__ Hp, int mb, int Lp, int L,
                                           int k)
{
#pragma unroll
    for (int c = 0; c < MT; ++c) {
        // base plus a 32-bit byte offset: one scalar offset register per load
        const int m = min(mb + c, L - 1);
        const unsigned off = ((unsigned)(m * Lp) + 2u * (unsigned)k) * 32u;
        h[c] = *(const Rec8*)((const char*)Hp + off);
    }
}

// 1/sqrt factors of the pair (n = 2k+1, 2k): ra(n) = Rt'[le+n] * Rt'[le-n+1]
struct FwdR { double2 hi, lo; };
__device__ __forceinline__ FwdR fwd_load_r(const double* __restrict__ Rt, int le, int k)
{
    FwdR r;
    r.hi = rpair(Rt, le + 2 * k + 1);              // 1/sqrt(le+2k), 1/sqrt(le+2k+1)
    r.lo = rpair(Rt, max(le - 2 * k, -1) + 1);     // 1/sqrt(le-2k-1), 1/sqrt(le-2k)  (0 below 0)
    return r;
}

// The spin values of the pair's steps: sv.x at n = 2k+1, sv.y at n = 2k.
template <int MT, bool EXT, bool INJ, bool RL, bool SPT, bool CHK = EXT>
__device__ __forceinline__ void fwd_pair(FwdLane<MT, EXT>& st, int k, int l, int mb, int as,
                                         const Rec8 (&h)[MT], const FwdR& r, const double2& sv, bool& anyscaled)
{
    // n = 2k+1: 1/sqrt(l+n) = hi.y, 1/sqrt(l-n+1) = lo.x;  n = 2k: hi.x, lo.y
    fwd_step<MT, EXT, 1, INJ, RL, SPT, CHK>(st, 2 * k + 1, l, mb, as, h, r.hi.y * r.lo.x, sv.x, anyscaled);
    fwd_step<MT, EXT, 0, INJ, RL, SPT, CHK>(st, 2 * k, l, mb, as, h, r.hi.x * r.lo.y, sv.y, anyscaled);
}

// SPT: the spin values Delta^l_{|s|,n} of the lane for the pair k (rows 2k+1,
// 2k) from the transposed spin rows (svl: the lane's column, row stride L);
// without, the spin row runs as a third chain.
template <bool SPT>
__device__ __forceinline__ double2 fwd_load_sv(const double* __restrict__ svl, int L, int k)
{
    if (!SPT) return make_double2(0.0, 0.0);
    return make_double2(svl[(size_t)(2 * k + 1) * L], svl[(size_t)(2 * k) * L]);
}

// Pairs kfrom, kfrom-1, ..., kto+1 (an even count); on entry A holds pair kfrom,
// on exit A holds pair kto (pair 0 when kto < 0).
template <int MT, bool EXT, bool INJ, bool RL, bool SPT>
__device__ __forceinline__ void fwd_phase(FwdLane<MT, EXT>& st, int kfrom, int kto, int l, int le, int mb,
                                          int as, const double* __restrict__ Hp, const double* __restrict__ Rt,
                                          const double* __restrict__ svl, int Lp, int L, Rec8 (&hA)[MT],
                                          Rec8 (&hB)[MT], FwdR& rA, FwdR& rB, double2& sA, double2& sB,
                                          bool& anyscaled)
{
    auto body = [&](int k, auto chk) {
        constexpr bool C = decltype(chk)::value;
        wait_scalar(hA[0].v[0]);
        __builtin_amdgcn_sched_barrier(0);
        fwd_load_h<MT>(hB, Hp, mb, Lp, L, k - 1);
        rB = fwd_load_r(Rt, le, k - 1);
        sB = fwd_load_sv<SPT>(svl, L, k - 1);
        __builtin_amdgcn_sched_barrier(0);
        fwd_pair<MT, EXT, INJ, RL, SPT, C>(st, k, l, mb, as, hA, rA, sA, anyscaled);
        wait_scalar(hB[0].v[0]);
        __builtin_amdgcn_sched_barrier(0);
        const int k2 = max(k - 2, 0);
        fwd_load_h<MT>(hA, Hp, mb, Lp, L, k2);
        rA = fwd_load_r(Rt, le, k2);
        sA = fwd_load_sv<SPT>(svl, L, k2);
        __builtin_amdgcn_sched_barrier(0);
        fwd_pair<MT, EXT, INJ, RL, SPT, C>(st, k - 1, l, mb, as, hB, rB, sB, anyscaled);
    };
    int k = kfrom;
    if constexpr (EXT && !INJ) {
        // past the chain starts no chain becomes scaled again: once none is
        // (anyscaled is uniform over the wave), the rest runs unchecked
        for (; k > kto && anyscaled; k -= 2) body(k, std::true_type());
        for (; k > kto; k -= 2) body(k, std::false_type());
    } else {
        for (; k > kto; k -= 2) body(k, std::integral_constant<bool, EXT>());
    }
}

// Pairs ktop .. klo of one segment; pairs >= kA (kA in [klo, ktop+1]) contain
// lane starts.  Phase loops cover even pair counts; a leftover pair is peeled.
template <int MT, bool EXT, bool RL, bool SPT>
__device__ __forceinline__ void fwd_segment(FwdLane<MT, EXT>& st, int ktop, int kA, int klo, int l, int le, int mb,
                                            int as, const double* __restrict__ Hp, const double* __restrict__ Rt,
                                            const double* __restrict__ svl, int Lp, int L, bool& anyscaled)
{
    Rec8 hA[MT], hB[MT];
    FwdR rA, rB;
    double2 sA, sB;
    fwd_load_h<MT>(hA, Hp, mb, Lp, L, ktop);
    rA = fwd_load_r(Rt, le, ktop);
    sA = fwd_load_sv<SPT>(svl, L, ktop);
    int cntA = ktop - kA + 1;
    if ((cntA & 1) && kA > klo) { --kA; ++cntA; }
    if (cntA > 0) {
        const int klastA = (cntA & 1) ? kA + 1 : kA;
        fwd_phase<MT, EXT, true, RL, SPT>(st, ktop, klastA - 1, l, le, mb, as, Hp, Rt, svl, Lp, L, hA, hB, rA, rB, sA,
                                          sB, anyscaled);
        if (cntA & 1) {            // kA = klo, in A
            wait_scalar(hA[0].v[0]);
            fwd_pair<MT, EXT, true, RL, SPT>(st, kA, l, mb, as, hA, rA, sA, anyscaled);
            return;
        }
    }
    const int cntB = kA - klo;     // pairs kA-1 .. klo, A holds kA-1
    if (cntB > 0) {
        const int klastB = (cntB & 1) ? klo + 1 : klo;
        fwd_phase<MT, EXT, false, RL, SPT>(st, kA - 1, klastB - 1, l, le, mb, as, Hp, Rt, svl, Lp, L, hA, hB, rA, rB,
                                           sA, sB, anyscaled);
        if (cntB & 1) {
            wait_scalar(hA[0].v[0]);
            fwd_pair<MT, EXT, false, RL, SPT>(st, klo, l, mb, as, hA, rA, sA, anyscaled);
        }
    }
}

// Bring a (D_{n-1}, D_n) checkpoint pair with levels (k0, k1) to one level.
template <bool EXT>
__device__ __forceinline__ void ck_level(double& v0, double& v1, int k0, int k1, int& k)
{
    if (!EXT) { k = 0; return; }
    k = max(k0, k1);
    v0 = ldexp(v0, EXT_STEP * (k - k0));
    v1 = ldexp(v1, EXT_STEP * (k - k1));
}

// Segment of one wave in the forward kernels: pairs ktop..klo of the row
// recursions, with lane starts in pairs >= kA; idle waves are inactive.
struct FwdSeg { int ktop, kA, klo; bool active; };

// Chain state of wave w (rows [lo, hi)) for the group (64 degrees l0.., MT
// orders mb..): the top segment (w == nseg-1, hi = nmax+1, lo <= l0) starts
// every lane at its own n = l from the edge value; a lower segment runs n from
// hi-1 down to lo, started from the checkpoint pair of the plane at n_c = hi, a
// multiple of ckfg (every lane has l >= n_c there).
template <int MT, bool EXT, int NS>
__device__ __forceinline__ FwdSeg fwd_setup(FwdLane<MT, EXT, NS>& st, bool& anyscaled, int w, int nseg, int lo, int hi,
                                            int l0, int mb, int l, int L, const SpinSet<NS>& as, int ckfg,
                                            const double* __restrict__ edge, const int* __restrict__ edgek,
                                            const double2* __restrict__ ckf, const int2* __restrict__ ckfk)
{
    const bool valid = l < L;
    const int le = valid ? l : L - 1;
    const int nmax = min(l0 + 63, L - 1);
    const size_t T = (size_t)L * (L + 1) / 2;
#pragma unroll
    for (int c = 0; c < MT; ++c) {
        st.dc[c] = 0.0; st.dn[c] = 0.0; st.k[c] = 0; st.start[c] = 0.0; st.startk[c] = 0;
        st.ap[c][0] = st.ap[c][1] = st.am[c][0] = st.am[c][1] = make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) { st.sc[j] = 0.0; st.sn[j] = 0.0; st.ks[j] = 0; st.starts[j] = 0.0; st.startks[j] = 0; }
    st.anext = 0.0;
    st.q = 0.0; st.dq = 0.0;
    anyscaled = EXT;
    FwdSeg g{0, 0, 0, false};
    if (w == nseg - 1) {
#pragma unroll
        for (int c = 0; c < MT; ++c) {
            const int m = mb + c;
            const bool ok = valid && m <= l;
            // the table holds (-1)^(l-m) Delta^l_{m,l}
            st.start[c] = ok ? sgn(l - m) * edge[(size_t)m * L + l] : 0.0;
            st.startk[c] = (EXT && ok) ? edgek[(size_t)m * L + l] : 0;
        }
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int a = as.a[j];
            const bool oks = valid && a <= l;
            st.starts[j] = oks ? sgn(le - a) * edge[(size_t)a * L + le] : 0.0;
            st.startks[j] = (EXT && oks) ? edgek[(size_t)a * L + le] : 0;
        }
        const int ktop = nmax >> 1, ntop = 2 * ktop + 1;   // n = L (odd L) is a zero pad step
        st.q = (double)(le + ntop) * (double)(le - ntop + 1);
        st.dq = 2.0 * (double)(ntop - 1);
        g = FwdSeg{ktop, l0 >> 1, lo >> 1, true};
    } else if (w < nseg - 1) {
        const int nc = hi;
        const size_t base = (size_t)(nc / ckfg - 1) * T;
#pragma unroll
        for (int c = 0; c < MT; ++c) {
            const int m = mb + c;
            if (valid && m <= l) {
                const size_t i = base + tri_m(m, l, L);
                double2 v = ckf[i];
                int kk = 0;
                if (EXT) { const int2 kv = ckfk[i]; ck_level<EXT>(v.x, v.y, kv.x, kv.y, kk); }
                st.dc[c] = v.x; st.dn[c] = v.y; st.k[c] = kk;
            }
        }
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int a = as.a[j];
            if (valid && a <= l) {
                const size_t i = base + tri_m(a, l, L);
                double2 v = ckf[i];
                int kk = 0;
                if (EXT) { const int2 kv = ckfk[i]; ck_level<EXT>(v.x, v.y, kv.x, kv.y, kk); }
                st.sc[j] = v.x; st.sn[j] = v.y; st.ks[j] = kk;
            }
        }
        st.anext = sqrt(fmax(0.0, (double)(le + nc) * (double)(le - nc + 1)));
        const int ntop = nc - 1;
        st.q = (double)(le + ntop) * (double)(le - ntop + 1);
        st.dq = 2.0 * (double)(ntop - 1);
        if (EXT) {
            bool sc = false;
#pragma unroll
            for (int j = 0; j < NS; ++j) sc |= st.ks[j] > 0;
#pragma unroll
            for (int c = 0; c < MT; ++c) sc |= st.k[c] > 0;
            anyscaled = __any(sc);
        }
        g = FwdSeg{ntop >> 1, (ntop >> 1) + 1, lo >> 1, true};
    }
    return g;
}

// FP64 forward contraction.  One workgroup per chain group (64 degrees l0..,
// MT orders mb..); wave w runs segment w of the row recursions.  Partial sums
// are added in LDS in segment order.
template <int MT, bool EXT, bool RL, bool SPT>
__device__ __forceinline__ void contract_forward_body(
    const double* __restrict__ Hp0, size_t hstride, const Batch& B, const double* __restrict__ Rtg,
    const double* __restrict__ edge, const int* __restrict__ edgek, const double* __restrict__ cl,
    const double2* __restrict__ ckf, const int2* __restrict__ ckfk, const double* __restrict__ svf,
    const int4* __restrict__ work, int L, int Lp, int s, int ckfg)
{
    // LDS: the partial sums of upper segments, red[slot][c][k][lane].  The
    // 1/sqrt table is read from global memory (L1-resident), so the LDS of a
    // workgroup does not grow with L.
    __shared__ double2 red[SEG_MAX * MT * 4 * 64];
    const double* __restrict__ Rt = Rtg;
    const double* __restrict__ Hp = Hp0 + blockIdx.y * hstride;   // map blockIdx.y of the launch
    double2* __restrict__ flm = (double2*)B.out[blockIdx.y];
    const int slot = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // this wave's segment: see the work-list layout of the plan
    const int4 d = work[(size_t)blockIdx.x * SEG_MAX + slot];
    const int l0 = uniform(d.x), mb = uniform(d.y), code = uniform(d.z), rows = uniform(d.w);
    const bool item = l0 >= 0;
    const int w = code & 0xff, nseg = (code >> 8) & 0xff, lead = (code >> 16) & 0xff;
    const int lo = rows & 0xffff, hi = (int)((unsigned)rows >> 16);   // this segment's rows [lo, hi)
    const bool bar = (code >> 24) & 1;   // the same for every slot of the workgroup
    const int l = l0 + lane;
    const bool valid = item && l < L;
    const int le = valid ? l : L - 1;
    const int as = s < 0 ? -s : s;

    FwdLane<MT, EXT> st;
    if (item) {
        bool anyscaled;
        const FwdSeg g = fwd_setup<MT, EXT, 1>(st, anyscaled, w, nseg, lo, hi, l0, mb, l, L, SpinSet<1>{{as}}, ckfg,
                                               edge, edgek, ckf, ckfk);
        if (SPT) {   // the spin row's values come from the transposed spin rows, not a chain
            st.ks[0] = 0;
            if (EXT) {
                bool sc = false;
#pragma unroll
                for (int c = 0; c < MT; ++c) sc |= st.k[c] > 0;
                anyscaled = __any(sc);
            }
        }
        if (g.active)
            fwd_segment<MT, EXT, RL, SPT>(st, g.ktop, g.kA, g.klo, l, le, mb, as, Hp, Rt, svf + le, Lp, L, anyscaled);
    }
    if (bar) {
        // every wave of the workgroup (empty slots too) meets at this one barrier
        auto R = [&](int j, int c, int k) -> double2& { return red[((j * MT + c) * 4 + k) * 64 + lane]; };
        if (item && w > 0) {
#pragma unroll
            for (int c = 0; c < MT; ++c) {
                R(slot, c, 0) = st.ap[c][0];
                R(slot, c, 1) = st.ap[c][1];
                R(slot, c, 2) = st.am[c][0];
                R(slot, c, 3) = st.am[c][1];
            }
        }
        __syncthreads();
        if (!item || w != 0) return;
        for (int j = 1; j < nseg; ++j) {
#pragma unroll
            for (int c = 0; c < MT; ++c) {
                double2 v;
                v = R(lead + j, c, 0); st.ap[c][0].x += v.x; st.ap[c][0].y += v.y;
                v = R(lead + j, c, 1); st.ap[c][1].x += v.x; st.ap[c][1].y += v.y;
                v = R(lead + j, c, 2); st.am[c][0].x += v.x; st.am[c][0].y += v.y;
                v = R(lead + j, c, 3); st.am[c][1].x += v.x; st.am[c][1].y += v.y;
            }
        }
    } else if (!item) {
        return;
    }

    if (!valid) return;
    const double c_l = cl[l];
#pragma unroll
    for (int c = 0; c < MT; ++c) {
        const int m = mb + c;
        if (m > l) continue;
        double2 sp, sm;
        double fp, fm;
        if (s >= 0) {
            sp = make_double2(st.ap[c][0].x - st.ap[c][1].x, st.ap[c][0].y - st.ap[c][1].y);
            fp = sgn(m + l + s);
            sm = make_double2(st.am[c][0].x + st.am[c][1].x, st.am[c][0].y + st.am[c][1].y);
            fm = sgn(m + s);
        } else {
            sp = make_double2(st.ap[c][0].x + st.ap[c][1].x, st.ap[c][0].y + st.ap[c][1].y);
            fp = sgn(m + s);
            sm = make_double2(st.am[c][0].x - st.am[c][1].x, st.am[c][0].y - st.am[c][1].y);
            fm = sgn(l + m + s);
        }
        const double base = sgn(s) * c_l;
        double2 op = mul_ipow(sp, ((m + s) % 4 + 4) % 4);
        const double2 fpm = make_double2(op.x * base * fp, op.y * base * fp);
        flm[(size_t)l * l + l + m] = fpm;
        if (m > 0) {
            if (RL) {   // real scalar map: f_{l,-m} = (-1)^m conj(f_{l,m}) (Sec. IV-G)
                const double sg = sgn(m);
                flm[(size_t)l * l + l - m] = make_double2(sg * fpm.x, -sg * fpm.y);
            } else {
                double2 om = mul_ipow(sm, ((-m + s) % 4 + 4) % 4);
                flm[(size_t)l * l + l - m] = make_double2(om.x * base * fm, om.y * base * fm);
            }
        }
    }
}


// Four waves per SIMD for a complex map (five spill in the loops and are
// slower), plain or exponent-extended; a real map's plain variant fits five,
// the most its 32 KB of LDS per workgroup allows.
#define MW_FORWARD_ARGS                                                                                          \
    const double* __restrict__ Hp0, size_t hstride, Batch B, const double* __restrict__ Rtg,                    \
        const double* __restrict__ edge, const int* __restrict__ edgek, const double* __restrict__ cl,           \
        const double2* __restrict__ ckf, const int2* __restrict__ ckfk, const double* __restrict__ svf,          \
        const int4* __restrict__ work, int L, int Lp, int s, int ckfg
#define MW_FORWARD_PASS Hp0, hstride, B, Rtg, edge, edgek, cl, ckf, ckfk, svf, work, L, Lp, s, ckfg

template <int MT, bool RL, bool SPT>
__global__ __launch_bounds__(64 * SEG_MAX) __attribute__((amdgpu_waves_per_eu(4))) void k_contract_forward(
    MW_FORWARD_ARGS)
{
    contract_forward_body<MT, false, RL, SPT>(MW_FORWARD_PASS);
}

template <int MT, bool RL, bool SPT>
__global__ __launch_bounds__(64 * SEG_MAX) __attribute__((amdgpu_waves_per_eu(4))) void k_contract_forward_ext(
    MW_FORWARD_ARGS)
{
    contract_forward_body<MT, true, RL, SPT>(MW_FORWARD_PASS);
}
#undef MW_FORWARD_ARGS
#undef MW_FORWARD_PASS

// ===========================================================================
// Inverse contraction
// ===========================================================================

// Inverse coefficient stream: record (c_l sp(l) f_{l,m}, c_l sm(l) f_{l,-m}) / (h_m(l) h_|s|(l))
// at [(m*Lp + l)*4] for 0 <= m <= l < L (zero elsewhere, l < Lp), where sp and sm
// are the degree-parity factors of the +m and -m terms (Eq. for F_{m m'} with
// the order symmetries of Delta) and h the scales of the contraction's chains
// (the .y of the l-recursion table), which the division undoes.  A 32(l) x 8(m) tile is read along m (rows of
// f_lm are contiguous in m) and written along l through LDS.
constexpr int STR_L = 32, STR_M = 8;

// OUT32 = 1 writes the record as FP32 at [(m*4 + comp)*Lp + l] instead (the
// layout the mixed-precision inverse stages per order).
template <int OUT32>
__global__ __launch_bounds__(256) void k_inverse_stream(Batch B, const double* __restrict__ cl,
                                                        const double2* __restrict__ lco, int L, int Lp, int real)
{
    const int s = B.s[blockIdx.z];
    const double2* __restrict__ flm = (const double2*)B.in[blockIdx.z];
    void* __restrict__ fs = B.out[blockIdx.z];
    __shared__ double2 ta[STR_L][STR_M + 1], tb[STR_L][STR_M + 1];
    const int l0 = blockIdx.x * STR_L, m0 = blockIdx.y * STR_M;
    {
        const int i = threadIdx.x / STR_M, k = threadIdx.x % STR_M;   // read: l = l0+i, m = m0+k
        const int l = l0 + i, m = m0 + k;
        double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
        if (l < L && m <= l) {
            const size_t c = (size_t)l * l + l;
            a = flm[c + m];
            if (real) b = (m & 1) ? make_double2(-a.x, a.y) : make_double2(a.x, -a.y);
            else b = flm[c - m];
        }
        ta[i][k] = a;
        tb[i][k] = b;
    }
    __syncthreads();
    {
        const int i = threadIdx.x % STR_L, k = threadIdx.x / STR_L;   // write: l = l0+i, m = m0+k
        const int l = l0 + i, m = m0 + k;
        if (m >= L || l >= Lp) return;
        const int as = s < 0 ? -s : s;
        const double c = (l < L) ? cl[l] / (lco[(size_t)m * Lp + l].y * lco[(size_t)as * Lp + l].y) : 0.0;
        const double par = (l & 1) ? -c : c;
        const double sp = (s >= 0) ? par : c;
        const double sm = (s >= 0) ? c : par;
        const double2 a = ta[i][k], b = tb[i][k];
        if (OUT32) {
            float* r32 = (float*)fs + (size_t)m * 4 * Lp + l;
            r32[0] = (float)(sp * a.x);
            r32[(size_t)Lp] = (float)(sp * a.y);
            r32[2 * (size_t)Lp] = (float)(sm * b.x);
            r32[3 * (size_t)Lp] = (float)(sm * b.y);
        } else {
            double4* rec = (double4*)((double*)fs + ((size_t)m * Lp + l) * 4);
            *rec = make_double4(sp * a.x, sp * a.y, sm * b.x, sm * b.y);
        }
    }
}

// Coefficients of the conjugate map (Sec. IV-G): if f has spin s and
// coefficients sf_lm, conj(f) has spin -s and coefficients
// (-1)^{s+m} conj(sf_{l,-m}); under the reality condition sf* = -sf these are the
// spin -s coefficients of the same signal, obtained without a transform.  One
// thread per (l, m >= 0) reads both (l, +-m) before writing them, so out may
// equal in; entries with l < |s| are set to 0.
__global__ __launch_bounds__(256) void k_spin_flip(Batch B, int L)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;   // (l, m >= 0) in triangle order
    const int b = blockIdx.y;
    if (k >= L * (L + 1) / 2) return;
    int l = (int)((sqrt(8.0 * (double)k + 1.0) - 1.0) * 0.5);
    while ((l + 1) * (l + 2) / 2 <= k) ++l;
    while (l * (l + 1) / 2 > k) --l;
    const int m = k - l * (l + 1) / 2;
    const int s = B.s[b];
    const double2* __restrict__ in = (const double2*)B.in[b];
    double2* __restrict__ out = (double2*)B.out[b];
    const size_t c = (size_t)l * l + l;
    double2 vp = make_double2(0.0, 0.0), vm = make_double2(0.0, 0.0);
    if (l >= (s < 0 ? -s : s)) {
        const double2 a = in[c + m], z = in[c - m];
        const double sg = ((s + m) & 1) ? -1.0 : 1.0;   // (-1)^{s+m} = (-1)^{s-m}
        vp = make_double2(sg * z.x, -sg * z.y);
        vm = make_double2(sg * a.x, -sg * a.y);
    }
    out[c + m] = vp;
    if (m > 0) out[c - m] = vm;
}

// Adjoint of the real-map coefficient expansion f_{l,-m} = (-1)^m conj(f_{l,m})
// (Sec. IV-G): y_{l,m} += (-1)^m conj(y_{l,-m}) and y_{l,-m} = 0 for m > 0.
// One thread per (l, m > 0).
__global__ __launch_bounds__(256) void k_real_fold(Batch B, int L)
{
    double2* __restrict__ y = (double2*)B.out[blockIdx.z];
    const int l = blockIdx.y;
    const int m = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (l >= L || m > l) return;
    const size_t c = (size_t)l * l + l;
    const double2 a = y[c + m], b = y[c - m];
    const double sg = (m & 1) ? -1.0 : 1.0;
    y[c + m] = make_double2(a.x + sg * b.x, a.y - sg * b.y);
    y[c - m] = make_double2(0.0, 0.0);
}

struct InvR { double2 a, b; };             // 1/sqrt of l+1-n .. l+2-n and l+1+n .. l+2+n

__device__ __forceinline__ InvR inv_load_r(const double* __restrict__ Rt, int ne, int j)
{
    InvR r;
    const int l = 2 * j;
    r.a = rpair(Rt, max(l + 1 - ne, -1) + 1);   // 1/sqrt(l+1-n), 1/sqrt(l+2-n)  (0 below 0)
    r.b = rpair(Rt, l + 2 + ne);                // 1/sqrt(l+1+n), 1/sqrt(l+2+n)
    return r;
}

struct CkOff { size_t off[CKI_MAX]; };   // start of checkpoint plane k (k >= 1)

// Segment of one wave in the inverse kernels: pairs jfrom..jlast (pair j =
// degrees 2j, 2j+1), with chain starts in pairs <= jA; idle waves are inactive.
struct InvSeg { int jfrom, jA, jlast; bool active; };

// Geometry of the inverse group (64 orders n0.., order m): pairs start at the
// even degree lstart = max(n0, m) rounded down; the wave's segment covers the
// degrees [cs, ce): wave 0 from lstart (cs = lstart) up to a boundary beyond
// every chain start (all lie below lA), wave w >= 1 from the checkpoint plane at
// degree cs (a multiple of the plane spacing).
struct InvGeo { int lstart, lA, cs, ce, nseg; };

// ===========================================================================
// FP64 inverse contraction, two orders per wavefront.  The orders m0, m0+1 of a
// group share everything that depends on n and l only: X_n(l), Y_n(l), the
// exact q bookkeeping and the spin chain Delta^l_{n,|s|}; each order keeps its
// own chain Delta^l_{n,m} and sums.  The uniform data of a step (both orders'
// stream records and (Pu', h), and (Pu', h) of |s|) is 28 scalar registers, so
// it is double-buffered step by step.
// ===========================================================================
template <bool EXT, int NS = 1>
struct InvLane2 {
    double dc[2], dp[2];       // Delta^l_{n,m_c}, Delta^{l-1}_{n,m_c}
    double sc[NS], sp[NS];     // Delta^l_{n,|s_j|}, Delta^{l-1}_{n,|s_j|}
    double2 ap[2], am[2];
    int k[2], ks[NS];
    double q, dq, sprev;
    double start[2], starts[NS];
    int startk[2], startks[NS], lz[2], l0s[NS];
};

// Spin tables Delta^l_{n,|s_j|} (values, exponent levels) of the spin rows of a
// chain group.
template <int NS>
struct SpinTabs {
    const double* val[NS];
    const int* k[NS];
};

struct InvS2 { double4 f0, f1; double2 c0, c1, cs; };   // one step l

// Rows of the uniform data of a group: stream records of both orders, their
// (Pu', h) factors and those of |s|, each indexed by the degree l.  Addresses
// are a base pointer plus a 32-bit byte offset (scalar loads take the offset
// in a register, so a row costs one register instead of a 64-bit pointer).
struct Inv2Rows {
    const char* f;   // stream records, 32 bytes per (m, l)
    const char* c;   // (Pu', h), 16 bytes per (m, l)
    unsigned f0, f1, c0, c1, cs, cs2;   // byte offsets of the rows at l = 0 (cs2: a second spin row)
};

__device__ __forceinline__ Inv2Rows inv2_rows(const double* __restrict__ fs, const double2* __restrict__ lco, int m0,
                                              int as, int Lp, int L, int as2 = -1)
{
    const int m1 = min(m0 + 1, L - 1);   // order L (odd L) never starts; any row will do
    return Inv2Rows{(const char*)fs, (const char*)lco, (unsigned)(m0 * Lp) * 32u, (unsigned)(m1 * Lp) * 32u,
                    (unsigned)(m0 * Lp) * 16u, (unsigned)(m1 * Lp) * 16u, (unsigned)(as * Lp) * 16u,
                    (unsigned)((as2 < 0 ? as : as2) * Lp) * 16u};
}

__device__ __forceinline__ void inv2_load(InvS2& u, const Inv2Rows& w, int l)
{
    const unsigned lf = (unsigned)l * 32u, lc = (unsigned)l * 16u;
    u.f0 = *(const double4*)(w.f + (w.f0 + lf));
    u.f1 = *(const double4*)(w.f + (w.f1 + lf));
    u.c0 = *(const double2*)(w.c + (w.c0 + lc));
    u.c1 = *(const double2*)(w.c + (w.c1 + lc));
    u.cs = *(const double2*)(w.c + (w.cs + lc));
}


// Brings the first lines of a segment's uniform rows into the L2 before its
// loop: lane i reads one dword of line i of each row (stream records, 32 bytes
// per degree; (Pu', h) rows, 16 bytes), starting at degree l0 and clamped to
// degree lend.  Waves of one order pair start their segments at the same
// degrees, so without this every new line of the loop would be a miss beyond
// the L2 for all of them at once; the values feed only a register use.
__device__ __forceinline__ unsigned inv2_touch(const Inv2Rows& w, int l0, int lend, int lane)
{
    const unsigned df = (unsigned)min(l0 + 2 * lane, lend), dc = (unsigned)min(l0 + 4 * lane, lend);
    unsigned t = *(const unsigned*)(w.f + (w.f0 + df * 32u));
    t += *(const unsigned*)(w.f + (w.f1 + df * 32u));
    t += *(const unsigned*)(w.c + (w.c0 + dc * 16u));
    t += *(const unsigned*)(w.c + (w.c1 + dc * 16u));
    t += *(const unsigned*)(w.c + (w.cs + dc * 16u));
    return t;
}

// One step l of both orders' chains and the spin chain: injections, the
// products pr[c] = e^l_{n,m_c} e^l_{n,|s|} of this step (scaled chains, e = h Delta;
// the coefficient records carry 1/(h_m h_|s|)), then the recursion to l+1.
// (c0, c1, cs): (Pu', h) of the two orders and of |s| at l.
template <bool EXT, int NS>
__device__ __forceinline__ bool inv2_scaled(const InvLane2<EXT, NS>& st)
{
    bool any = st.k[0] > 0 || st.k[1] > 0;
#pragma unroll
    for (int j = 0; j < NS; ++j) any |= st.ks[j] > 0;
    return any;
}

// dd: the chain values of this step as they enter the products (0 while scaled).
// SPT: the spin values e^l_{n,|s_j|} of this step are svt[j], read from the
// spin tables' scaled rows, instead of chains.
// CHK: the exponent-extended state is checked; past the chain starts, once no
// lane of the wave holds a scaled chain, the steps run without the checks.
template <bool EXT, bool INJ, int NS, bool SPT = false, bool CHK = EXT>
__device__ __forceinline__ void inv2_core_d(InvLane2<EXT, NS>& st, int l, int lstart, double nd, const double2& c0,
                                            const double2& c1, const double2 (&cs)[NS], double rs,
                                            double (&pr)[2][NS], double (&dd)[2], bool& anyscaled,
                                            const double* svt = nullptr)
{
    if (INJ) {
#pragma unroll
        for (int c = 0; c < 2; ++c)
            if (l == st.lz[c]) { st.dc[c] = st.start[c]; if (EXT) st.k[c] = st.startk[c]; }
        if constexpr (!SPT) {
#pragma unroll
            for (int j = 0; j < NS; ++j)
                if (l == st.l0s[j] && st.l0s[j] > lstart) { st.sc[j] = st.starts[j]; if (EXT) st.ks[j] = st.startks[j]; }
        }
        if (EXT) anyscaled = __any(inv2_scaled(st));
    }
    double sv[NS];
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        if constexpr (SPT) {
            sv[j] = svt[j];
        } else {
            sv[j] = st.sc[j];
            if (CHK) sv[j] = (st.ks[j] == 0) ? sv[j] : 0.0;
        }
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        double d = st.dc[c];
        if (CHK) d = (st.k[c] == 0) ? d : 0.0;
        dd[c] = d;
#pragma unroll
        for (int j = 0; j < NS; ++j) pr[c][j] = d * sv[j];
    }
    // X_n(l) = n/sqrt((l+1)^2-n^2), Y_n(l) = sqrt(l^2-n^2)/sqrt((l+1)^2-n^2); harmless at l = L-1
    const double xn = nd * rs;
    const double yn = st.sprev * rs;
    st.sprev = st.q * rs;
    st.q += st.dq;
    st.dq += 2.0;
    // scaled chains: the Delta^{l-1} term has coefficient 1 (.x = Pu'_m(l))
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const double2 pq = c ? c1 : c0;
        const double dn = fma(pq.x * xn, st.dc[c], yn * st.dp[c]);
        st.dp[c] = st.dc[c];
        st.dc[c] = dn;
    }
    if constexpr (!SPT) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const double sn = fma(cs[j].x * xn, st.sc[j], yn * st.sp[j]);
            st.sp[j] = st.sc[j];
            st.sc[j] = sn;
        }
    }
    if (CHK && anyscaled) {
#pragma unroll
        for (int c = 0; c < 2; ++c)
            if (st.k[c] > 0 && fabs(st.dc[c]) > EXT_UP) { st.dc[c] *= EXT_DOWN; st.dp[c] *= EXT_DOWN; st.k[c] -= 1; }
        if constexpr (!SPT) {
#pragma unroll
            for (int j = 0; j < NS; ++j)
                if (st.ks[j] > 0 && fabs(st.sc[j]) > EXT_UP) { st.sc[j] *= EXT_DOWN; st.sp[j] *= EXT_DOWN; st.ks[j] -= 1; }
        }
        anyscaled = __any(inv2_scaled(st));
    }
}

template <bool EXT, bool INJ, int NS>
__device__ __forceinline__ void inv2_core(InvLane2<EXT, NS>& st, int l, int lstart, double nd, const double2& c0,
                                          const double2& c1, const double2 (&cs)[NS], double rs,
                                          double (&pr)[2][NS], bool& anyscaled)
{
    double dd[2];
    inv2_core_d<EXT, INJ, NS>(st, l, lstart, nd, c0, c1, cs, rs, pr, dd, anyscaled);
}

template <bool EXT, bool INJ, bool RL, bool CHK = EXT>
__device__ __forceinline__ void inv2_step(InvLane2<EXT>& st, int l, int lstart, double nd, const InvS2& u, double rs,
                                          double sv, bool& anyscaled)
{
    double pr[2][1], dd[2];
    const double2 cs[1] = {u.cs};
    inv2_core_d<EXT, INJ, 1, true, CHK>(st, l, lstart, nd, u.c0, u.c1, cs, rs, pr, dd, anyscaled, &sv);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const double4 f = c ? u.f1 : u.f0;
        st.ap[c].x = fma(pr[c][0], f.x, st.ap[c].x);
        st.ap[c].y = fma(pr[c][0], f.y, st.ap[c].y);
        if (!RL) {
            st.am[c].x = fma(pr[c][0], f.z, st.am[c].x);
            st.am[c].y = fma(pr[c][0], f.w, st.am[c].y);
        }
    }
}

// Pairs jfrom .. jlast (pair j = steps 2j, 2j+1); A holds even steps, B odd ones.
// The 1/sqrt factors alternate between two register sets over pairs (two pairs
// per iteration, an odd last pair peeled); r holds those of pair jfrom on entry
// and of pair jlast+1 on return.
// The spin values of the lane come from the scaled spin rows sv[l*L + n]
// (svb: the lane's row base), loaded one step ahead beside the uniform records
// (svA with uA, svB with uB).
template <bool EXT, bool INJ, bool RL>
__device__ __forceinline__ void inv2_phase(InvLane2<EXT>& st, int jfrom, int jlast, int lend, int lstart, int ne,
                                           double nd, const Inv2Rows& rows, const double* __restrict__ Rt,
                                           const double* __restrict__ svb, int L, InvS2& uA, InvS2& uB, double& svA,
                                           double& svB, InvR& r, bool& anyscaled)
{
    const int jr = lend >> 1;   // last pair whose factors exist
    InvR rB;
    auto halfc = [&](int l, const InvR& rc, auto chk) {   // steps l (in A) and l+1 (in B)
        constexpr bool C = decltype(chk)::value;
        wait_scalar(uA.f0.x);
        __builtin_amdgcn_sched_barrier(0);
        inv2_load(uB, rows, l + 1);
        svB = svb[(size_t)(l + 1) * L];
        __builtin_amdgcn_sched_barrier(0);
        inv2_step<EXT, INJ, RL, C>(st, l, lstart, nd, uA, rc.a.x * rc.b.x, svA, anyscaled);
        wait_scalar(uB.f0.x);
        __builtin_amdgcn_sched_barrier(0);
        const int l2 = min(l + 2, lend);
        inv2_load(uA, rows, l2);
        svA = svb[(size_t)l2 * L];
        __builtin_amdgcn_sched_barrier(0);
        inv2_step<EXT, INJ, RL, C>(st, l + 1, lstart, nd, uB, rc.a.y * rc.b.y, svB, anyscaled);
    };
    auto half = [&](int l, const InvR& rc) { halfc(l, rc, std::integral_constant<bool, EXT>()); };
    if constexpr (EXT) {
        // the exponent-extended variant keeps one pair per iteration: unrolled,
        // it needs more registers than its wave budget leaves.  Past the chain
        // starts no chain becomes scaled again: once none is (anyscaled is
        // uniform over the wave), the rest runs unchecked.
        int j = jfrom;
        if constexpr (!INJ) {
            for (; j <= jlast && anyscaled; ++j) {
                rB = inv_load_r(Rt, ne, min(j + 1, jr));
                halfc(2 * j, r, std::true_type());
                r = rB;
            }
        }
        for (; j <= jlast; ++j) {
            rB = inv_load_r(Rt, ne, min(j + 1, jr));
            if constexpr (INJ) halfc(2 * j, r, std::true_type());
            else halfc(2 * j, r, std::false_type());
            r = rB;
        }
    } else {
        int j = jfrom;
        for (; j < jlast; j += 2) {
            rB = inv_load_r(Rt, ne, min(j + 1, jr));
            half(2 * j, r);
            r = inv_load_r(Rt, ne, min(j + 2, jr));
            half(2 * j + 2, rB);
        }
        if (j == jlast) {
            rB = inv_load_r(Rt, ne, min(j + 1, jr));
            half(2 * j, r);
            r = rB;
        }
    }
}

// Start values are scaled by h_m(l) (the .y of the l-recursion table) at their
// degree, so that the chains run as e = h Delta.
template <bool EXT, int NS>
__device__ __forceinline__ InvSeg inv2_setup(InvLane2<EXT, NS>& st, bool& anyscaled, const InvGeo& geo, int w, int n,
                                             int m0, int L, int Lp, const SpinSet<NS>& sset, int ckg,
                                             const double2* __restrict__ lco, const double* __restrict__ edge,
                                             const int* __restrict__ edgek, const SpinTabs<NS>& tabs,
                                             const double2* __restrict__ cki, const int2* __restrict__ ckik,
                                             const CkOff& ckoff)
{
    const bool valid = n < L;
    const int ne = valid ? n : L - 1;
    const int lstart = geo.lstart;
    const int jend = (Lp >> 1) - 1;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        st.dc[c] = 0.0; st.dp[c] = 0.0; st.k[c] = 0; st.start[c] = 0.0; st.startk[c] = 0;
        st.ap[c] = st.am[c] = make_double2(0.0, 0.0);
        st.lz[c] = max(n, m0 + c);
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        st.sc[j] = 0.0; st.sp[j] = 0.0; st.ks[j] = 0; st.starts[j] = 0.0; st.startks[j] = 0;
        st.l0s[j] = max(n, sset.a[j]);
    }
    st.sprev = 0.0; st.q = 0.0; st.dq = 0.0;
    anyscaled = EXT;
    InvSeg g{0, 0, -1, false};
    if (w == 0) {
        if (valid) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int m = m0 + c;
                if (m >= L) continue;
                st.start[c] = edge[(size_t)m * L + n] * lco[(size_t)m * Lp + st.lz[c]].y;
                if (EXT) st.startk[c] = edgek[(size_t)m * L + n];
            }
            // spin chains: from the table at lstart when already running, else injected
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                const int as = sset.a[j];
                const double* __restrict__ stab = tabs.val[j];
                const int* __restrict__ stabk = tabs.k[j];
                if (st.l0s[j] <= lstart) {
                    double v1 = stab[(size_t)lstart * L + n], v0 = 0.0;
                    int k1 = EXT ? stabk[(size_t)lstart * L + n] : 0, k0 = k1;
                    v1 *= lco[(size_t)as * Lp + lstart].y;
                    if (lstart >= 1) {
                        v0 = stab[(size_t)(lstart - 1) * L + n] * lco[(size_t)as * Lp + lstart - 1].y;
                        k0 = EXT ? stabk[(size_t)(lstart - 1) * L + n] : 0;
                    }
                    int kk;
                    ck_level<EXT>(v0, v1, k0, k1, kk);
                    st.sc[j] = v1; st.sp[j] = v0; st.ks[j] = kk;
                } else if (st.l0s[j] < L) {
                    st.starts[j] = stab[(size_t)st.l0s[j] * L + n] * lco[(size_t)as * Lp + st.l0s[j]].y;
                    st.startks[j] = EXT ? stabk[(size_t)st.l0s[j] * L + n] : 0;
                }
            }
        }
        st.sprev = (lstart >= ne) ? sqrt((double)(lstart - ne) * (double)(lstart + ne)) : 0.0;
        st.q = (double)(lstart + 1 - ne) * (double)(lstart + 1 + ne);
        st.dq = 2.0 * (double)lstart + 3.0;
        const int jlast = min(geo.ce >> 1, jend + 1) - 1;
        const int jA = min(jlast, (geo.lA - 1) >> 1);
        g = InvSeg{lstart >> 1, jA, jlast, true};
    } else if (w < geo.nseg) {
        // segment from degree cdeg (> m0+1), started from its checkpoint plane
        const int cdeg = geo.cs;
        const int jj = cdeg / ckg;
        if (valid) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const int m = m0 + c;
                if (m >= L) continue;
                const size_t i = ckoff.off[jj] + (size_t)m * (cdeg + 1) + n;
                double2 v = cki[i];
                v.x *= lco[(size_t)m * Lp + cdeg - 1].y;
                v.y *= lco[(size_t)m * Lp + cdeg].y;
                int kk = 0;
                if (EXT) { const int2 kv = ckik[i]; ck_level<EXT>(v.x, v.y, kv.x, kv.y, kk); }
                st.dp[c] = v.x; st.dc[c] = v.y; st.k[c] = kk;
            }
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                const int as = sset.a[j];
                const double* __restrict__ stab = tabs.val[j];
                const int* __restrict__ stabk = tabs.k[j];
                double v1 = stab[(size_t)cdeg * L + n] * lco[(size_t)as * Lp + cdeg].y;
                double v0 = stab[(size_t)(cdeg - 1) * L + n] * lco[(size_t)as * Lp + cdeg - 1].y;
                int k1 = EXT ? stabk[(size_t)cdeg * L + n] : 0, k0 = EXT ? stabk[(size_t)(cdeg - 1) * L + n] : 0;
                int kk;
                ck_level<EXT>(v0, v1, k0, k1, kk);
                st.sc[j] = v1; st.sp[j] = v0; st.ks[j] = kk;
            }
        }
        st.sprev = sqrt(fmax(0.0, (double)(cdeg - ne) * (double)(cdeg + ne)));
        st.q = (double)(cdeg + 1 - ne) * (double)(cdeg + 1 + ne);
        st.dq = 2.0 * (double)cdeg + 3.0;
        if (EXT) anyscaled = __any(inv2_scaled(st));
        const int jlast = min(geo.ce >> 1, jend + 1) - 1;
        g = InvSeg{cdeg >> 1, (cdeg >> 1) - 1, jlast, true};
    }
    return g;
}

template <bool EXT, bool RL>
__device__ __forceinline__ void contract_inverse2_body(
    const double* __restrict__ fs0, size_t fstride, const Batch& B, const double* __restrict__ Rtg,
    const double* __restrict__ edge, const int* __restrict__ edgek, const double2* __restrict__ lco,
    const double* __restrict__ stab, const int* __restrict__ stabk, const double* __restrict__ svt,
    const double2* __restrict__ cki, const int2* __restrict__ ckik, CkOff ckoff, const int4* __restrict__ work,
    int L, int Lp, int s, int ckg)
{
    // LDS: the partial sums of later segments, red[slot][c][2][lane].  The 1/sqrt
    // table is read from global memory (L1-resident), so the LDS of a workgroup
    // stays small and does not grow with L.
    __shared__ double2 red[SEGI_MAX * 2 * 2 * 64];
    const double* __restrict__ Rt = Rtg;
    const double* __restrict__ fs = fs0 + blockIdx.y * fstride;   // map blockIdx.y of the launch
    double2* __restrict__ F = (double2*)B.out[blockIdx.y];
    const int slot = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // this wave's segment: see the work-list layout of the spin table
    const int4 d = work[(size_t)blockIdx.x * SEGI_MAX + slot];
    const int n0 = uniform(d.x), m0 = uniform(d.y), code = uniform(d.z), bounds = uniform(d.w);
    const bool item = n0 >= 0;
    const int w = code & 0xff, nseg = (code >> 8) & 0xff, lead = (code >> 16) & 0xff;
    const bool bar = (code >> 24) & 1;   // the same for every slot of the workgroup
    const int n = n0 + lane;
    const bool valid = item && n < L;
    const int ne = valid ? n : L - 1;
    const int as = s < 0 ? -s : s;
    const double nd = (double)ne;
    const int lend = Lp - 1;

    InvLane2<EXT> st;
    if (item) {
        InvGeo geo;
        geo.lstart = max(n0, m0) & ~1;
        geo.lA = max(max(n0 + 64, m0 + 2), as + 1);   // every chain start of both orders lies below lA
        geo.cs = bounds & 0xffff;
        geo.ce = (int)((unsigned)bounds >> 16);
        geo.nseg = nseg;
        const Inv2Rows rows = inv2_rows(fs, lco, m0, as, Lp, L);
        const unsigned touched = inv2_touch(rows, geo.cs, lend, lane);
        bool anyscaled;
        const InvSeg g = inv2_setup<EXT, 1>(st, anyscaled, geo, w, n, m0, L, Lp, SpinSet<1>{{as}}, ckg, lco, edge,
                                            edgek, SpinTabs<1>{{stab}, {stabk}}, cki, ckik, ckoff);
        st.ks[0] = 0;   // the spin values come from the scaled rows, not a chain
        if (EXT) anyscaled = __any(inv2_scaled(st));
        asm volatile("" ::"v"(touched));
        if (g.active) {
            const double* __restrict__ svb = svt + ne;
            InvS2 uA, uB;
            inv2_load(uA, rows, 2 * g.jfrom);
            double svA = svb[(size_t)(2 * g.jfrom) * L], svB;
            InvR r = inv_load_r(Rt, ne, g.jfrom);
            const int jA = min(g.jA, g.jlast);
            if (g.jfrom <= jA)
                inv2_phase<EXT, true, RL>(st, g.jfrom, jA, lend, geo.lstart, ne, nd, rows, Rt, svb, L, uA, uB, svA, svB,
                                          r, anyscaled);
            if (max(g.jfrom, jA + 1) <= g.jlast)
                inv2_phase<EXT, false, RL>(st, max(g.jfrom, jA + 1), g.jlast, lend, geo.lstart, ne, nd, rows, Rt, svb,
                                           L, uA, uB, svA, svB, r, anyscaled);
        }
    }

    if (bar) {
        // every wave of the workgroup (empty slots too) meets at this one barrier
        auto R = [&](int k, int c, int h) -> double2& { return red[((k * 2 + c) * 2 + h) * 64 + lane]; };
        if (item && w > 0) {
#pragma unroll
            for (int c = 0; c < 2; ++c) { R(slot, c, 0) = st.ap[c]; R(slot, c, 1) = st.am[c]; }
        }
        __syncthreads();
        if (!item || w != 0) return;
        for (int k = 1; k < nseg; ++k)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const double2 a = R(lead + k, c, 0), b = R(lead + k, c, 1);
                st.ap[c].x += a.x; st.ap[c].y += a.y;
                st.am[c].x += b.x; st.am[c].y += b.y;
            }
    } else if (!item) {
        return;
    }

    if (!valid) return;
    const double fsp = sgn(s) * ((s >= 0) ? sgn(n) : 1.0);
    const double fsm = sgn(s) * ((s < 0) ? sgn(n) : 1.0);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int m = m0 + c;
        if (m >= L) continue;
        const double2 op = mul_ipow(st.ap[c], ((-(m + s)) % 4 + 4) % 4);
        F[(size_t)(L - 1 + m) * L + n] = make_double2(op.x * fsp, op.y * fsp);
        if (!RL && m > 0) {
            const double2 om = mul_ipow(st.am[c], ((m - s) % 4 + 4) % 4);
            F[(size_t)(L - 1 - m) * L + n] = make_double2(om.x * fsm, om.y * fsm);
        }
    }
}

#define MW_INVERSE2_ARGS                                                                                         \
    const double* __restrict__ fs0, size_t fstride, Batch B, const double* __restrict__ Rtg,                    \
        const double* __restrict__ edge, const int* __restrict__ edgek, const double2* __restrict__ lco,         \
        const double* __restrict__ stab, const int* __restrict__ stabk, const double* __restrict__ svt,         \
        const double2* __restrict__ cki, const int2* __restrict__ ckik, CkOff ckoff,                            \
        const int4* __restrict__ work, int L, int Lp, int s, int ckg
#define MW_INVERSE2_PASS fs0, fstride, B, Rtg, edge, edgek, lco, stab, stabk, svt, cki, ckik, ckoff, work, L, Lp, s, ckg

// Register budgets: a real map keeps no -m sums, which leaves room for one more
// wave per SIMD (seven plain, six exponent-extended) without spills in the loops.
template <bool RL>
__global__ __launch_bounds__(64 * SEGI_MAX) __attribute__((amdgpu_waves_per_eu(RL ? 7 : 6))) void k_contract_inverse2(
    MW_INVERSE2_ARGS)
{
    contract_inverse2_body<false, RL>(MW_INVERSE2_PASS);
}

template <bool RL>
__global__ __launch_bounds__(64 * SEGI_MAX) __attribute__((amdgpu_waves_per_eu(RL ? 6 : 4))) void k_contract_inverse2_ext(
    MW_INVERSE2_ARGS)
{
    contract_inverse2_body<true, RL>(MW_INVERSE2_PASS);
}
#undef MW_INVERSE2_ARGS
#undef MW_INVERSE2_PASS

// ===========================================================================
// FP64 inverse contraction over the triangle n >= m.  By the symmetry
// Delta^l_{m,n} = (-1)^{m+n} Delta^l_{n,m} (Sec. III-C), the chain Delta^l_{n,m}
// of a lane n >= m serves two sums:
//   normal      F_{+-m,n}: the stream record of order m (uniform over the wave)
//               times the lane's spin chain Delta^l_{n,|s|}, as in the
//               two-order kernel above;
//   transposed  F_{+-n,m}: the lane's own coefficients f_{l,+-n}, read from
//               f_lm (64 consecutive n of one degree are one contiguous run),
//               times the uniform factor c_l Delta^l_{m,|s|} / h_m(l), which
//               the spin table's lcos rows carry beside the chain factor of
//               order m (the division undoes the chain's scale h_m).
// With also Delta^l_{m,-n} = (-1)^{l+m} Delta^l_{m,n} and Delta^l_{m,-s} =
// (-1)^{l+m} Delta^l_{m,|s|} for s >= 0, the transposed sums take the degree
// signs of the normal ones (sp(l) on the +n sum, sm(l) on the -n sum: (-1)^l
// and 1 for s >= 0, 1 and (-1)^l for s < 0; SNEG = s < 0 fixes them per step
// parity at compile time) and the output signs (-1)^{s+n} (order +n) and
// (-1)^{s+n+m} (order -n) for s >= 0, (-1)^{s+n+m} and (-1)^{s+n} for s < 0.
// Lanes n < m of a group on the diagonal run no chain (their pairs are the
// transposed sums of another group); lane n = m writes the normal sums only.
// Only the groups with n0 + 63 >= m0 run (the spin table's wtri): about half
// the chain steps of the square kernel, at four more FMAs per step and order
// and two coalesced 16-byte reads per lane and step (one for real maps).
// ===========================================================================
template <bool EXT>
struct InvLane3 {
    InvLane2<EXT> b;
    double2 at[2], atm[2];   // transposed sums: orders +n, -n at rows m0, m0+1
};

// f_{l,+n} and f_{l,-n} of the lane at byte offsets op = 16 (l^2 + l + n) and
// op - 32 n of f_lm, through a buffer resource of L^2 records: offsets past the
// end (degree L, or l^2 + l - n < 0 as an unsigned offset) read zeros.
template <bool RL>
__device__ __forceinline__ double4 f_load(__amdgpu_buffer_rsrc_t rs, unsigned op, unsigned n32)
{
    const double2 a = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, op, 0, 0));
    if (RL) return make_double4(a.x, a.y, 0.0, 0.0);
    const double2 b = __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, op - n32, 0, 0));
    return make_double4(a.x, a.y, b.x, b.y);
}

// PAR: parity of l (the transposed sums' degree signs).
template <bool EXT, bool INJ, bool RL, bool SNEG, bool SPT, int PAR, bool CHK = EXT>
__device__ __forceinline__ void inv3_step(InvLane3<EXT>& st, int l, int lstart, double nd, const InvS2& u,
                                          const double4& g, double rs, double sv, bool& anyscaled)
{
    double pr[2][1], dd[2];
    const double2 cs[1] = {u.cs};
    inv2_core_d<EXT, INJ, 1, SPT, CHK>(st.b, l, lstart, nd, u.c0, u.c1, cs, rs, pr, dd, anyscaled, &sv);
    constexpr double sgp = (PAR && !SNEG) ? -1.0 : 1.0;   // sp(l)
    constexpr double sgm = (PAR && SNEG) ? -1.0 : 1.0;    // sm(l)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const double4 f = c ? u.f1 : u.f0;
        st.b.ap[c].x = fma(pr[c][0], f.x, st.b.ap[c].x);
        st.b.ap[c].y = fma(pr[c][0], f.y, st.b.ap[c].y);
        if (!RL) {
            st.b.am[c].x = fma(pr[c][0], f.z, st.b.am[c].x);
            st.b.am[c].y = fma(pr[c][0], f.w, st.b.am[c].y);
        }
        const double pt = dd[c] * (c ? u.c1.y : u.c0.y);
        st.at[c].x = fma(sgp * pt, g.x, st.at[c].x);
        st.at[c].y = fma(sgp * pt, g.y, st.at[c].y);
        if (!RL) {
            st.atm[c].x = fma(sgm * pt, g.z, st.atm[c].x);
            st.atm[c].y = fma(sgm * pt, g.w, st.atm[c].y);
        }
    }
}

// Pairs jfrom .. jlast as in inv2_phase; the lane's coefficients (and with SPT
// its spin values, else a third chain) are loaded one step ahead beside the
// uniform records (gA, svA with uA; gB, svB with uB).  op: the lane's f_lm
// offset at degree 2 jfrom on entry, advanced by 32 (l+1) per step.
template <bool EXT, bool INJ, bool RL, bool SNEG, bool SPT>
__device__ __forceinline__ void inv3_phase(InvLane3<EXT>& st, int jfrom, int jlast, int lend, int lstart, int ne,
                                           double nd, const Inv2Rows& rows, const double* __restrict__ Rt,
                                           __amdgpu_buffer_rsrc_t frs, unsigned& op, unsigned n32,
                                           const double* __restrict__ svb, int L, InvS2& uA, InvS2& uB, double4& gA,
                                           double4& gB, double& svA, double& svB, InvR& r, bool& anyscaled)
{
    const int jr = lend >> 1;   // last pair whose factors exist
    InvR rB;
    auto half = [&](int l, const InvR& rc, auto chk) {   // steps l (in A) and l+1 (in B)
        constexpr bool C = decltype(chk)::value;
        wait_scalar(uA.f0.x);
        __builtin_amdgcn_sched_barrier(0);
        inv2_load(uB, rows, l + 1);
        op += 32u * (unsigned)(l + 1);   // degree l+1
        gB = f_load<RL>(frs, op, n32);
        if (SPT) svB = svb[(size_t)(l + 1) * L];
        __builtin_amdgcn_sched_barrier(0);
        inv3_step<EXT, INJ, RL, SNEG, SPT, 0, C>(st, l, lstart, nd, uA, gA, rc.a.x * rc.b.x, svA, anyscaled);
        wait_scalar(uB.f0.x);
        __builtin_amdgcn_sched_barrier(0);
        const int l2 = min(l + 2, lend);
        inv2_load(uA, rows, l2);
        op += 32u * (unsigned)(l + 2);   // degree l+2 (past lend: beyond f_lm, reads zeros)
        gA = f_load<RL>(frs, op, n32);
        if (SPT) svA = svb[(size_t)l2 * L];
        __builtin_amdgcn_sched_barrier(0);
        inv3_step<EXT, INJ, RL, SNEG, SPT, 1, C>(st, l + 1, lstart, nd, uB, gB, rc.a.y * rc.b.y, svB, anyscaled);
    };
    int j = jfrom;
    if constexpr (EXT && !INJ) {
        // past the chain starts: checked while a chain of the wave is scaled
        // (anyscaled is uniform), unchecked after
        for (; j <= jlast && anyscaled; ++j) {
            rB = inv_load_r(Rt, ne, min(j + 1, jr));
            half(2 * j, r, std::true_type());
            r = rB;
        }
        for (; j <= jlast; ++j) {
            rB = inv_load_r(Rt, ne, min(j + 1, jr));
            half(2 * j, r, std::false_type());
            r = rB;
        }
    } else {
        for (; j <= jlast; ++j) {
            rB = inv_load_r(Rt, ne, min(j + 1, jr));
            half(2 * j, r, std::integral_constant<bool, EXT>());
            r = rB;
        }
    }
}

template <bool EXT, bool RL, bool SNEG, bool SPT>
__device__ __forceinline__ void contract_inverse_tri_body(
    const double* __restrict__ fs0, size_t fstride, const Batch& B, const double* __restrict__ Rtg,
    const double* __restrict__ edge, const int* __restrict__ edgek, const double2* __restrict__ lco,
    const double2* __restrict__ lcos, const double* __restrict__ stab, const int* __restrict__ stabk,
    const double* __restrict__ svt, const double2* __restrict__ cki, const int2* __restrict__ ckik, CkOff ckoff,
    const int4* __restrict__ work, int L, int Lp, int s, int ckg)
{
    // LDS: the partial sums of later segments, red[slot][c][acc][lane] with acc =
    // ap, at (and am, atm for complex maps)
    constexpr int NACC = RL ? 2 : 4;
    __shared__ double2 red[SEGT_MAX * 2 * NACC * 64];
    const double* __restrict__ Rt = Rtg;
    const double* __restrict__ fs = fs0 + blockIdx.y * fstride;   // map blockIdx.y of the launch
    const __amdgpu_buffer_rsrc_t frs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)B.in[blockIdx.y], (short)0, (int)((unsigned)L * (unsigned)L * 16u), 0x00020000);
    double2* __restrict__ F = (double2*)B.out[blockIdx.y];
    const int slot = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int4 d = work[(size_t)blockIdx.x * SEGT_MAX + slot];
    const int n0 = uniform(d.x), m0 = uniform(d.y), code = uniform(d.z), bounds = uniform(d.w);
    const bool item = n0 >= 0;
    const int w = code & 0xff, nseg = (code >> 8) & 0xff, lead = (code >> 16) & 0xff;
    const bool bar = (code >> 24) & 1;   // the same for every slot of the workgroup
    const int n = n0 + lane;
    const bool valid = item && n < L;
    const int ne = valid ? n : L - 1;
    const int as = s < 0 ? -s : s;
    const double nd = (double)ne;
    const int lend = Lp - 1;

    InvLane3<EXT> st;
#pragma unroll
    for (int c = 0; c < 2; ++c) st.at[c] = st.atm[c] = make_double2(0.0, 0.0);
    if (item) {
        InvGeo geo;
        geo.lstart = max(n0, m0) & ~1;
        geo.lA = max(max(n0 + 64, m0 + 2), as + 1);   // every chain start of both orders lies below lA
        geo.cs = bounds & 0xffff;
        geo.ce = (int)((unsigned)bounds >> 16);
        geo.nseg = nseg;
        // uniform rows: stream records of both orders; (Pu', spin factor) of
        // both orders and (Pu', -) of |s|, all from lcos
        const Inv2Rows rows = inv2_rows(fs, lcos, m0, as, Lp, L);
        const unsigned touched = inv2_touch(rows, geo.cs, lend, lane);
        bool anyscaled;
        const InvSeg g = inv2_setup<EXT, 1>(st.b, anyscaled, geo, w, n, m0, L, Lp, SpinSet<1>{{as}}, ckg, lco, edge,
                                            edgek, SpinTabs<1>{{stab}, {stabk}}, cki, ckik, ckoff);
        // lanes n < m run no chain of order m
#pragma unroll
        for (int c = 0; c < 2; ++c)
            if (n < m0 + c) {
                st.b.start[c] = 0.0; st.b.startk[c] = 0;
                st.b.dc[c] = 0.0; st.b.dp[c] = 0.0; st.b.k[c] = 0;
            }
        if (SPT) st.b.ks[0] = 0;   // the spin values come from the scaled rows, not a chain
        if (EXT) anyscaled = __any(inv2_scaled(st.b));
        asm volatile("" ::"v"(touched));
        if (g.active) {
            const unsigned l0 = 2u * (unsigned)g.jfrom, n32 = 32u * (unsigned)ne;
            unsigned op = 16u * (l0 * l0 + l0 + (unsigned)ne);
            const double* __restrict__ svb = svt + ne;
            InvS2 uA, uB;
            double4 gA, gB;
            inv2_load(uA, rows, 2 * g.jfrom);
            gA = f_load<RL>(frs, op, n32);
            double svA = SPT ? svb[(size_t)l0 * L] : 0.0, svB = 0.0;
            InvR r = inv_load_r(Rt, ne, g.jfrom);
            const int jA = min(g.jA, g.jlast);
            if (g.jfrom <= jA)
                inv3_phase<EXT, true, RL, SNEG, SPT>(st, g.jfrom, jA, lend, geo.lstart, ne, nd, rows, Rt, frs, op, n32,
                                                     svb, L, uA, uB, gA, gB, svA, svB, r, anyscaled);
            if (max(g.jfrom, jA + 1) <= g.jlast)
                inv3_phase<EXT, false, RL, SNEG, SPT>(st, max(g.jfrom, jA + 1), g.jlast, lend, geo.lstart, ne, nd, rows,
                                                      Rt, frs, op, n32, svb, L, uA, uB, gA, gB, svA, svB, r, anyscaled);
        }
    }

    if (bar) {
        // every wave of the workgroup (empty slots too) meets at this one barrier
        auto R = [&](int k, int c, int h) -> double2& { return red[((k * 2 + c) * NACC + h) * 64 + lane]; };
        if (item && w > 0) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                R(slot, c, 0) = st.b.ap[c];
                R(slot, c, 1) = st.at[c];
                if (!RL) { R(slot, c, NACC - 2) = st.b.am[c]; R(slot, c, NACC - 1) = st.atm[c]; }
            }
        }
        __syncthreads();
        if (!item || w != 0) return;
        for (int k = 1; k < nseg; ++k)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const double2 a = R(lead + k, c, 0), t = R(lead + k, c, 1);
                st.b.ap[c].x += a.x; st.b.ap[c].y += a.y;
                st.at[c].x += t.x; st.at[c].y += t.y;
                if (!RL) {
                    const double2 b = R(lead + k, c, NACC - 2), u = R(lead + k, c, NACC - 1);
                    st.b.am[c].x += b.x; st.b.am[c].y += b.y;
                    st.atm[c].x += u.x; st.atm[c].y += u.y;
                }
            }
    } else if (!item) {
        return;
    }

    if (!valid) return;
    const double ss = sgn(s), sn = sgn(n);
    const double fsp = ss * ((s >= 0) ? sn : 1.0);
    const double fsm = ss * ((s < 0) ? sn : 1.0);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int m = m0 + c;
        if (m >= L || n < m) continue;
        const double2 op = mul_ipow(st.b.ap[c], ((-(m + s)) % 4 + 4) % 4);
        F[(size_t)(L - 1 + m) * L + n] = make_double2(op.x * fsp, op.y * fsp);
        if (!RL && m > 0) {
            const double2 om = mul_ipow(st.b.am[c], ((m - s) % 4 + 4) % 4);
            F[(size_t)(L - 1 - m) * L + n] = make_double2(om.x * fsm, om.y * fsm);
        }
        if (n == m) continue;
        const double sgm = sgn(m);
        const double tsp = ss * sn * ((s >= 0) ? 1.0 : sgm);
        const double2 tp = mul_ipow(st.at[c], ((-(n + s)) % 4 + 4) % 4);
        F[(size_t)(L - 1 + n) * L + m] = make_double2(tp.x * tsp, tp.y * tsp);
        if (!RL) {
            const double tsm = ss * sn * ((s >= 0) ? sgm : 1.0);
            const double2 tm = mul_ipow(st.atm[c], ((n - s) % 4 + 4) % 4);
            F[(size_t)(L - 1 - n) * L + m] = make_double2(tm.x * tsm, tm.y * tsm);
        }
    }
}

#define MW_INVTRI_ARGS                                                                                           \
    const double* __restrict__ fs0, size_t fstride, Batch B, const double* __restrict__ Rtg,                    \
        const double* __restrict__ edge, const int* __restrict__ edgek, const double2* __restrict__ lco,         \
        const double2* __restrict__ lcos, const double* __restrict__ stab, const int* __restrict__ stabk,       \
        const double* __restrict__ svt, const double2* __restrict__ cki, const int2* __restrict__ ckik,         \
        CkOff ckoff, const int4* __restrict__ work, int L, int Lp, int s, int ckg
#define MW_INVTRI_PASS \
    fs0, fstride, B, Rtg, edge, edgek, lco, lcos, stab, stabk, svt, cki, ckik, ckoff, work, L, Lp, s, ckg

template <bool RL, bool SNEG, bool SPT>
__global__ __launch_bounds__(64 * SEGT_MAX) __attribute__((amdgpu_waves_per_eu(RL ? 5 : 4))) void
k_contract_inverse_tri(MW_INVTRI_ARGS)
{
    contract_inverse_tri_body<false, RL, SNEG, SPT>(MW_INVTRI_PASS);
}

template <bool RL, bool SNEG, bool SPT>
__global__ __launch_bounds__(64 * SEGT_MAX) __attribute__((amdgpu_waves_per_eu(4))) void
k_contract_inverse_tri_ext(MW_INVTRI_ARGS)
{
    contract_inverse_tri_body<true, RL, SNEG, SPT>(MW_INVTRI_PASS);
}
#undef MW_INVTRI_ARGS
#undef MW_INVTRI_PASS

// ===========================================================================
// Mixed precision (MW_FP32C): the same FP64 chains; each step's products
// Delta * Delta are rounded to FP32 and accumulated by the matrix cores with
// v_mfma_f32_4x4x1_16b_f32 (16 blocks of a 4x4 outer product per wave).  Block
// b of the instruction owns lanes 4b..4b+3; with lane i holding its own chain
// product as the B operand and component (i mod 4) of the uniform data as the A
// operand, accumulator register v of lane i receives sum_k comp_v(k) * K_i(k):
// every lane keeps its own four sums and nothing moves between lanes.  Several
// maps of one spin share the chains: each adds one instruction per step.  The
// uniform data (FP32, signs of the parity split folded in) is staged in LDS per
// workgroup; partial sums of the segments are added in FP64.
// ===========================================================================
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ v4f mfma4(float a, float b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}

// The staged FP32 data reaches the matrix cores through a per-wave window in
// LDS of WIN steps, refilled at each window boundary from registers that were
// loaded from global memory one window earlier (a wave reads only the window
// it wrote, so no barrier is needed).
constexpr int WIN = 32;                  // steps (n or l values) per window; 16 pairs
// LDS floats per window row: two more than WIN, so that the four component rows
// one step reads (one address each, broadcast to their lanes) start on banks 2
// apart instead of all on one bank.
constexpr int WROW = WIN + 2;

// Forward window q (n in [WIN*q, WIN*q + WIN)): rows (b, c, comp) of WIN floats,
// 8G rows, held as 2G float2 values per lane of the wave (in LDS, rows of WROW).
template <int G>
struct FwdWin { fv2 v[2 * G]; };

template <int G>
__device__ __forceinline__ void fwd_win_load(FwdWin<G>& r, const MixMaps& maps, int mb, int q, int lane)
{
#pragma unroll
    for (int t = 0; t < 2 * G; ++t) {
        const int e = lane + 64 * t;                  // float2 index in the window, 16 per row
        const int row = e >> 4, n = WIN * q + 2 * (e & 15);
        const int comp = row & 3, c = (row >> 2) & 1, b = row >> 3;
        r.v[t] = fv2{0.0f, 0.0f};
        if (b < mix_n(maps)) {
            const int Lb = maps.L[b], m = mb + c;
            // rows hold Lp_b entries, the pad n = L_b (odd L_b) zero
            if (m < Lb && n < Lb)
                r.v[t] = *(const fv2*)(maps.src[b] + ((size_t)m * 4 + comp) * (size_t)(Lb + (Lb & 1)) + n);
        }
    }
}

template <int G>
__device__ __forceinline__ void win_store(float* __restrict__ win, const fv2* v, int lane)
{
#pragma unroll
    for (int t = 0; t < G; ++t) {
        const int e = lane + 64 * t;   // float2 index in the window, 16 per row
        ((fv2*)win)[(e >> 4) * (WROW / 2) + (e & 15)] = v[t];
    }
}

// Maps of a group take the products of their own spin row: sj[b] in [0, NS).
// SPT: the spin rows' values of the pair (rows 2k+1, 2k) come from the spin
// tables' transposed rows (sv.v[j] = (row 2k+1, row 2k)), not chains.
template <int NS>
struct SvPairF { double2 v[NS]; };

template <bool SPT, int NS>
__device__ __forceinline__ void fwd_mix_load_sv(SvPairF<NS>& sv, const double* const (&svl)[NS], int L, int k)
{
    if constexpr (SPT) {
#pragma unroll
        for (int j = 0; j < NS; ++j)
            sv.v[j] = make_double2(svl[j][(size_t)(2 * k + 1) * L], svl[j][(size_t)(2 * k) * L]);
    }
}

template <bool EXT, int NS, bool CHK = EXT>
__device__ __forceinline__ double fwd_chain_value(const FwdLane<2, EXT, NS>& st, int c)
{
    double d = st.dc[c];
    if (CHK) d = (st.k[c] == 0) ? d : 0.0;
    return d;
}

// CHK: the exponent-extended state is checked (as in fwd_advance).
template <bool EXT, bool INJ, int G, int NS, bool SPT, bool CHK = EXT>
__device__ __forceinline__ void fwd_mix_pair(FwdLane<2, EXT, NS>& st, v4f (&acc)[2][G], int k, int l, int mb,
                                             const SpinSet<NS>& as, const MixMaps& maps,
                                             const float* __restrict__ win, int comp, const FwdR& r,
                                             const SvPairF<NS>& sv, bool& anyscaled)
{
    float k1[2][NS], k0[2][NS];
    fwd_inject<2, EXT, INJ, NS, SPT>(st, 2 * k + 1, l, anyscaled);
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        if constexpr (SPT) {
            k1[0][j] = (float)(fwd_chain_value<EXT, NS, CHK>(st, 0) * sv.v[j].x);
            k1[1][j] = (float)(fwd_chain_value<EXT, NS, CHK>(st, 1) * sv.v[j].x);
        } else {
            k1[0][j] = (float)fwd_product<2, EXT, NS, CHK>(st, 0, j);
            k1[1][j] = (float)fwd_product<2, EXT, NS, CHK>(st, 1, j);
        }
    }
    fwd_advance<2, EXT, NS, SPT, CHK>(st, mb, as, r.hi.y * r.lo.x, anyscaled);
    fwd_inject<2, EXT, INJ, NS, SPT>(st, 2 * k, l, anyscaled);
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        if constexpr (SPT) {
            k0[0][j] = (float)(fwd_chain_value<EXT, NS, CHK>(st, 0) * sv.v[j].y);
            k0[1][j] = (float)(fwd_chain_value<EXT, NS, CHK>(st, 1) * sv.v[j].y);
        } else {
            k0[0][j] = (float)fwd_product<2, EXT, NS, CHK>(st, 0, j);
            k0[1][j] = (float)fwd_product<2, EXT, NS, CHK>(st, 1, j);
        }
    }
    fwd_advance<2, EXT, NS, SPT, CHK>(st, mb, as, r.hi.x * r.lo.y, anyscaled);
    const int off = 2 * k - WIN * (k / (WIN / 2));   // n = 2k within its window
#pragma unroll
    for (int b = 0; b < G; ++b) {
        const bool second = NS > 1 && mix_row(maps, b) != 0;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const fv2 a = *(const fv2*)(win + ((b * 2 + c) * 4 + comp) * WROW + off);   // n = 2k, 2k+1
            acc[c][b] = mfma4(a.y, second ? k1[c][NS - 1] : k1[c][0], acc[c][b]);
            acc[c][b] = mfma4(a.x, second ? k0[c][NS - 1] : k0[c][0], acc[c][b]);
        }
    }
}

// Pairs k .. kto (descending; INJ: pairs with lane starts), window by window:
// on entering window q the window loaded one window earlier is stored to LDS and
// window q-1 requested; the pairs of a window then run two at a time with the
// 1/sqrt factors alternating between the A and B register sets (A holds pair k
// on entry and on return).  EXIT: return before entering a window once no chain
// of the wave is scaled (k then names the next pair; the caller continues
// unchecked, CHK = false).
template <bool EXT, bool INJ, int G, int NS, bool SPT, bool CHK = EXT, bool EXIT = false>
__device__ __forceinline__ void fwd_mix_run(FwdLane<2, EXT, NS>& st, v4f (&acc)[2][G], const FwdSeg& g, int& k, int kto,
                                            int l, int le, int mb, const SpinSet<NS>& as, const double* __restrict__ Rt,
                                            const double* const (&svl)[NS], int L, float* __restrict__ win,
                                            const MixMaps& maps, int lane, FwdWin<G>& nxt, FwdR& rA, SvPairF<NS>& sA,
                                            bool& anyscaled)
{
    constexpr int PW = WIN / 2;   // pairs per window
    const int comp = lane & 3;
    FwdR rB;
    SvPairF<NS> sB;
    while (k >= kto) {
        if constexpr (EXIT) {
            if (!anyscaled) return;
        }
        if (k == g.ktop || (k % PW) == PW - 1) {       // entering window k / PW
            win_store<2 * G>(win, nxt.v, lane);
            if (k / PW > g.klo / PW) fwd_win_load<G>(nxt, maps, mb, k / PW - 1, lane);
        }
        const int kw = max(kto, (k / PW) * PW);        // lowest pair of this window in range
        for (; k > kw; k -= 2) {
            rB = fwd_load_r(Rt, le, max(k - 1, 0));
            fwd_mix_load_sv<SPT>(sB, svl, L, max(k - 1, 0));
            fwd_mix_pair<EXT, INJ, G, NS, SPT, CHK>(st, acc, k, l, mb, as, maps, win, comp, rA, sA, anyscaled);
            rA = fwd_load_r(Rt, le, max(k - 2, 0));
            fwd_mix_load_sv<SPT>(sA, svl, L, max(k - 2, 0));
            fwd_mix_pair<EXT, INJ, G, NS, SPT, CHK>(st, acc, k - 1, l, mb, as, maps, win, comp, rB, sB, anyscaled);
        }
        if (k == kw) {                                 // odd pair left in the window
            rB = fwd_load_r(Rt, le, max(k - 1, 0));
            fwd_mix_load_sv<SPT>(sB, svl, L, max(k - 1, 0));
            fwd_mix_pair<EXT, INJ, G, NS, SPT, CHK>(st, acc, k, l, mb, as, maps, win, comp, rA, sA, anyscaled);
            rA = rB;
            sA = sB;
            --k;
        }
    }
}

template <bool EXT, int G, int NS, bool SPT>
__device__ __forceinline__ void fwd_mix_segment(FwdLane<2, EXT, NS>& st, v4f (&acc)[2][G], const FwdSeg& g, int l,
                                                int le, int mb, const SpinSet<NS>& as, const double* __restrict__ Rt,
                                                const double* const (&svl)[NS], int L, float* __restrict__ win,
                                                const MixMaps& maps, int lane, bool& anyscaled)
{
    constexpr int PW = WIN / 2;
    FwdWin<G> nxt;
    fwd_win_load<G>(nxt, maps, mb, g.ktop / PW, lane);
    FwdR rA = fwd_load_r(Rt, le, g.ktop);
    SvPairF<NS> sA;
    fwd_mix_load_sv<SPT>(sA, svl, L, g.ktop);
    int k = g.ktop;
    fwd_mix_run<EXT, true, G, NS, SPT>(st, acc, g, k, max(g.kA, g.klo), l, le, mb, as, Rt, svl, L, win, maps, lane,
                                       nxt, rA, sA, anyscaled);   // pairs with lane starts
    if constexpr (EXT) {
        // past the chain starts: checked while a chain of the wave is scaled,
        // unchecked from the next window on
        fwd_mix_run<EXT, false, G, NS, SPT, true, true>(st, acc, g, k, g.klo, l, le, mb, as, Rt, svl, L, win, maps,
                                                        lane, nxt, rA, sA, anyscaled);
        fwd_mix_run<EXT, false, G, NS, SPT, false>(st, acc, g, k, g.klo, l, le, mb, as, Rt, svl, L, win, maps, lane,
                                                   nxt, rA, sA, anyscaled);
    } else {
        fwd_mix_run<EXT, false, G, NS, SPT>(st, acc, g, k, g.klo, l, le, mb, as, Rt, svl, L, win, maps, lane, nxt, rA,
                                            sA, anyscaled);
    }
}

// Forward contraction of a group of up to G maps with at most NS different |s|
// (band-limits maps.L[b] <= L, the plan's; spin mix_spin(MB, maps, b), whose |s|
// is the launch's spin row mix_row(maps, b)).  maps.src[b]: H of map b in FP32 at
// [(m*4 + comp)*Lp_b + n], comp = (Re, Im) of sigma_+(n) H_{m,n} and of
// sigma_-(n) H_{-m,n}, where sigma_+ = (-1)^n for s >= 0 (else 1) and sigma_- =
// (-1)^n for s < 0 (else 1); maps.dst[b]: f_lm of map b.
// LDS floats per wave slot of the mixed forward: its window, later its partial
// sums (a v4f per order, map and lane).
__host__ __device__ constexpr int fwdm_slot_floats(int G)
{
    return (G * 8 * WROW > 2 * G * 64 * 4) ? G * 8 * WROW : 2 * G * 64 * 4;
}

// Wave budgets as for the mixed inverse: five waves per SIMD for one map (96
// VGPRs, the accumulators in ordinary VGPRs), four for two, three for four;
// with a second spin row one wave less for one or two maps (no spills).
template <bool EXT, int G, int NS, bool SPT>
__global__ __launch_bounds__(64 * SEG_MAX) __attribute__((amdgpu_waves_per_eu(
    G == 8 ? 2 : (NS == 1 ? (G == 1 ? 5 : (G == 4 ? 3 : 4)) : (G == 1 ? 4 : 3))))) void k_contract_forward_mix(
    MixBatch MB, const double* __restrict__ Rtg, const double* __restrict__ edge, const int* __restrict__ edgek,
    const double* __restrict__ cl, const double2* __restrict__ ckf, const int2* __restrict__ ckfk,
    const int4* __restrict__ work, int L, int ckfg)
{
    extern __shared__ double smem[];
    const MixMaps& maps = MB.g[blockIdx.y];
    const int slot = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // this wave's segment: see the work-list layout of the plan
    const int4 d = work[(size_t)blockIdx.x * SEG_MAX + slot];
    const int l0 = uniform(d.x), mb = uniform(d.y), code = uniform(d.z), rows = uniform(d.w);
    const bool item = l0 >= 0;
    const int w = code & 0xff, nseg = (code >> 8) & 0xff, lead = (code >> 16) & 0xff;
    const int lo = rows & 0xffff, hi = (int)((unsigned)rows >> 16);   // this segment's rows [lo, hi)
    const bool bar = (code >> 24) & 1;   // the same for every slot of the workgroup
    bool any = false;                    // does any map of the group have this (l0, mb) block?
    for (int b = 0; b < mix_n(maps); ++b) any |= (l0 < maps.L[b] && mb < maps.L[b]);
    const double* __restrict__ Rt = Rtg;               // 1/sqrt table, L1-resident
    float* region = (float*)smem + slot * fwdm_slot_floats(G);
    const int l = l0 + lane;
    const bool valid = item && l < L;
    const int le = valid ? l : L - 1;
    SpinSet<NS> as;
#pragma unroll
    for (int j = 0; j < NS; ++j) as.a[j] = MB.as[j];

    v4f acc[2][G];
#pragma unroll
    for (int b = 0; b < G; ++b) acc[0][b] = acc[1][b] = v4f{0.f, 0.f, 0.f, 0.f};
    if (item && any) {
        FwdLane<2, EXT, NS> st;
        bool anyscaled;
        const FwdSeg g =
            fwd_setup<2, EXT, NS>(st, anyscaled, w, nseg, lo, hi, l0, mb, l, L, as, ckfg, edge, edgek, ckf, ckfk);
        const double* svl[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) svl[j] = SPT ? MB.ssvf[j] + le : nullptr;
        if (SPT) {   // the spin rows' values come from the tables' transposed rows, not chains
#pragma unroll
            for (int j = 0; j < NS; ++j) st.ks[j] = 0;
            if (EXT) anyscaled = __any(st.k[0] > 0 || st.k[1] > 0);
        }
        if (g.active)
            fwd_mix_segment<EXT, G, NS, SPT>(st, acc, g, l, le, mb, as, Rt, svl, L, region, maps, lane, anyscaled);
    }

    if (bar) {
        // every wave of the workgroup (empty slots too) meets at this one barrier;
        // a wave's partial sums overwrite its own window, which it no longer reads
        if (item && w > 0) {
            v4f* red = (v4f*)region;
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int b = 0; b < G; ++b) red[(c * G + b) * 64 + lane] = acc[c][b];
        }
        __syncthreads();
        if (!item || w != 0) return;
    } else if (!item) {
        return;
    }
    if (!valid) return;
    // one (map, order) at a time: its FP32 sums in FP64, plus those of the later
    // segments in segment order
    const int nadd = bar ? nseg : 1;
#pragma unroll
    for (int b = 0; b < G; ++b) {
        if (b >= mix_n(maps) || l >= maps.L[b]) continue;
        const int s = mix_spin(MB, maps, b);
        const double base = sgn(s) * cl[l];
        double2* flm = maps.dst[b];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int m = mb + c;
            if (m > l || m >= maps.L[b]) continue;
            double sum[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) sum[q] = (double)acc[c][b][q];
            for (int k = 1; k < nadd; ++k) {
                const v4f v = ((const v4f*)((const float*)smem + (lead + k) * fwdm_slot_floats(G)))[(c * G + b) * 64 + lane];
#pragma unroll
                for (int q = 0; q < 4; ++q) sum[q] += (double)v[q];
            }
            const double fp = (s >= 0) ? sgn(m + l + s) : sgn(m + s);
            const double fm = (s >= 0) ? sgn(m + s) : sgn(l + m + s);
            const double2 op = mul_ipow(make_double2(sum[0], sum[1]), ((m + s) % 4 + 4) % 4);
            flm[(size_t)l * l + l + m] = make_double2(op.x * base * fp, op.y * base * fp);
            if (m > 0) {
                const double2 om = mul_ipow(make_double2(sum[2], sum[3]), ((-m + s) % 4 + 4) % 4);
                flm[(size_t)l * l + l - m] = make_double2(om.x * base * fm, om.y * base * fm);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Mixed-precision inverse contraction, two orders per wavefront: the chains of
// the FP64 two-order kernel (inv2_core), with each step's products rounded to
// FP32 and accumulated by v_mfma_f32_4x4x1_16b_f32 against the FP32 stream of
// every map of the group (windows of WIN degrees in LDS, as in the one-order
// kernel).  Work list: the packed segment list of the spin table.
// pair (l, l+1): (Pu', h) of m0, of m0+1 and of the spin rows |s_j|
template <int NS>
struct InvC2 { double4 c0, c1, cs[NS]; };

template <int NS>
__device__ __forceinline__ void inv2m_load_c(InvC2<NS>& u, const Inv2Rows& w, int j)
{
    const unsigned lc = (unsigned)(2 * j) * 16u;
    u.c0 = *(const double4*)(w.c + (w.c0 + lc));
    u.c1 = *(const double4*)(w.c + (w.c1 + lc));
    u.cs[0] = *(const double4*)(w.c + (w.cs + lc));
    if constexpr (NS > 1) u.cs[NS - 1] = *(const double4*)(w.c + (w.cs2 + lc));
}

// Window q of the group: rows r = (b*2 + c)*4 + comp (map b, order m0+c, stream
// component comp) of WIN floats; each lane holds 2G float2 of them.
template <int G>
struct InvWin2 { fv2 v[2 * G]; };

template <int G>
__device__ __forceinline__ void inv2m_win_load(InvWin2<G>& r, const MixMaps& maps, int m0, int q, int lane)
{
#pragma unroll
    for (int t = 0; t < 2 * G; ++t) {
        const int e = lane + 64 * t;                  // float2 index in the window, 16 per row
        const int row = e >> 4, l = WIN * q + 2 * (e & 15);
        const int comp = row & 3, c = (row >> 2) & 1, b = row >> 3;
        const int m = m0 + c;
        r.v[t] = fv2{0.0f, 0.0f};
        if (b < mix_n(maps)) {
            const int Lb = maps.L[b];
            if (m < Lb && l < Lb)
                r.v[t] = *(const fv2*)(maps.src[b] + ((size_t)m * 4 + comp) * (size_t)(Lb + (Lb & 1)) + l);
        }
    }
}

// Spin values of a pair (degrees 2j, 2j+1) of the lane, one double2 per spin
// row, from the scaled spin rows (row stride L).
template <int NS>
struct SvPair { double2 v[NS]; };

template <int NS>
__device__ __forceinline__ void inv2m_load_sv(SvPair<NS>& sv, const double* const (&svl)[NS], int L, int j)
{
#pragma unroll
    for (int q = 0; q < NS; ++q) sv.v[q] = make_double2(svl[q][(size_t)(2 * j) * L], svl[q][(size_t)(2 * j + 1) * L]);
}

template <bool EXT, bool INJ, int G, int NS, bool CHK = EXT>
__device__ __forceinline__ void inv2m_pair(InvLane2<EXT, NS>& st, v4f (&acc)[2][G], int j, int lstart, double nd,
                                           const InvC2<NS>& u, const InvR& r, const SvPair<NS>& sp,
                                           const MixMaps& maps, const float* __restrict__ win, int comp,
                                           bool& anyscaled)
{
    const int l = 2 * j;
    double p0[2][NS], p1[2][NS], dd[2], s0[NS], s1[NS];
    double2 cs0[NS], cs1[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        cs0[q] = make_double2(u.cs[q].x, u.cs[q].y);
        cs1[q] = make_double2(u.cs[q].z, u.cs[q].w);
        s0[q] = sp.v[q].x;
        s1[q] = sp.v[q].y;
    }
    inv2_core_d<EXT, INJ, NS, true, CHK>(st, l, lstart, nd, make_double2(u.c0.x, u.c0.y),
                                         make_double2(u.c1.x, u.c1.y), cs0, r.a.x * r.b.x, p0, dd, anyscaled, s0);
    inv2_core_d<EXT, INJ, NS, true, CHK>(st, l + 1, lstart, nd, make_double2(u.c0.z, u.c0.w),
                                         make_double2(u.c1.z, u.c1.w), cs1, r.a.y * r.b.y, p1, dd, anyscaled, s1);
    const int off = l - WIN * (j / (WIN / 2));   // degree l within its window
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        float k0[NS], k1[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) { k0[q] = (float)p0[c][q]; k1[q] = (float)p1[c][q]; }
#pragma unroll
        for (int b = 0; b < G; ++b) {
            const bool second = NS > 1 && mix_row(maps, b) != 0;
            const fv2 a = *(const fv2*)(win + ((b * 2 + c) * 4 + comp) * WROW + off);   // degrees l, l+1
            acc[c][b] = mfma4(a.x, second ? k0[NS - 1] : k0[0], acc[c][b]);
            acc[c][b] = mfma4(a.y, second ? k1[NS - 1] : k1[0], acc[c][b]);
        }
    }
}

// Pairs j .. jto of a segment (INJ: pairs with chain starts), window by window:
// on entering window q the window loaded one window earlier is stored to LDS and
// window q+1 requested; the pairs of a window then run two at a time with the
// uniform data and 1/sqrt factors alternating between the A and B register sets
// (A holds pair j on entry and on return).  EXIT: return before entering a
// window once no chain of the wave is scaled (the caller continues unchecked).
template <bool EXT, bool INJ, int G, int NS, bool CHK = EXT, bool EXIT = false>
__device__ __forceinline__ void inv2m_run(InvLane2<EXT, NS>& st, v4f (&acc)[2][G], const InvSeg& g, int& j, int jto,
                                          int jend, int lstart, int ne, double nd, int m0, const Inv2Rows& rows,
                                          const double* __restrict__ Rt, const double* const (&svl)[NS], int L,
                                          float* __restrict__ win, const MixMaps& maps, int lane, InvWin2<G>& nxt,
                                          InvC2<NS>& uA, InvR& rA, SvPair<NS>& sA, bool& anyscaled)
{
    constexpr int PW = WIN / 2;   // pairs per window
    const int comp = lane & 3;
    InvC2<NS> uB;
    InvR rB;
    SvPair<NS> sB;
    while (j <= jto) {
        if constexpr (EXIT) {
            if (!anyscaled) return;
        }
        if (j == g.jfrom || (j % PW) == 0) {          // entering window j / PW
            win_store<2 * G>(win, nxt.v, lane);
            if (j / PW < g.jlast / PW) inv2m_win_load<G>(nxt, maps, m0, j / PW + 1, lane);
        }
        const int jw = min(jto, (j / PW) * PW + PW - 1);   // last pair of this window in range
        for (; j < jw; j += 2) {
            wait_scalar(uA.c0.x);
            inv2m_load_c(uB, rows, min(j + 1, jend));
            rB = inv_load_r(Rt, ne, min(j + 1, jend));
            inv2m_load_sv(sB, svl, L, min(j + 1, jend));
            inv2m_pair<EXT, INJ, G, NS, CHK>(st, acc, j, lstart, nd, uA, rA, sA, maps, win, comp, anyscaled);
            wait_scalar(uB.c0.x);
            inv2m_load_c(uA, rows, min(j + 2, jend));
            rA = inv_load_r(Rt, ne, min(j + 2, jend));
            inv2m_load_sv(sA, svl, L, min(j + 2, jend));
            inv2m_pair<EXT, INJ, G, NS, CHK>(st, acc, j + 1, lstart, nd, uB, rB, sB, maps, win, comp, anyscaled);
        }
        if (j == jw) {                                 // odd pair left in the window
            wait_scalar(uA.c0.x);
            inv2m_load_c(uB, rows, min(j + 1, jend));
            rB = inv_load_r(Rt, ne, min(j + 1, jend));
            inv2m_load_sv(sB, svl, L, min(j + 1, jend));
            inv2m_pair<EXT, INJ, G, NS, CHK>(st, acc, j, lstart, nd, uA, rA, sA, maps, win, comp, anyscaled);
            uA = uB;
            rA = rB;
            sA = sB;
            ++j;
        }
    }
}

template <bool EXT, int G, int NS>
__device__ __forceinline__ void inv2m_segment(InvLane2<EXT, NS>& st, v4f (&acc)[2][G], const InvSeg& g, int jend,
                                              int lstart, int ne, double nd, int m0, const Inv2Rows& rows,
                                              const double* __restrict__ Rt, const double* const (&svl)[NS], int L,
                                              float* __restrict__ win, const MixMaps& maps, int lane,
                                              bool& anyscaled)
{
    constexpr int PW = WIN / 2;
    InvWin2<G> nxt;
    inv2m_win_load<G>(nxt, maps, m0, g.jfrom / PW, lane);
    InvC2<NS> uA;
    inv2m_load_c<NS>(uA, rows, g.jfrom);
    InvR rA = inv_load_r(Rt, ne, g.jfrom);
    SvPair<NS> sA;
    inv2m_load_sv(sA, svl, L, g.jfrom);
    int j = g.jfrom;
    inv2m_run<EXT, true, G, NS>(st, acc, g, j, min(g.jA, g.jlast), jend, lstart, ne, nd, m0, rows, Rt, svl, L, win,
                                maps, lane, nxt, uA, rA, sA, anyscaled);   // pairs with chain starts
    if constexpr (EXT) {
        // past the chain starts: checked while a chain of the wave is scaled,
        // unchecked from the next window on
        inv2m_run<EXT, false, G, NS, true, true>(st, acc, g, j, g.jlast, jend, lstart, ne, nd, m0, rows, Rt, svl, L,
                                                 win, maps, lane, nxt, uA, rA, sA, anyscaled);
        inv2m_run<EXT, false, G, NS, false>(st, acc, g, j, g.jlast, jend, lstart, ne, nd, m0, rows, Rt, svl, L, win,
                                            maps, lane, nxt, uA, rA, sA, anyscaled);
    } else {
        inv2m_run<EXT, false, G, NS>(st, acc, g, j, g.jlast, jend, lstart, ne, nd, m0, rows, Rt, svl, L, win, maps,
                                     lane, nxt, uA, rA, sA, anyscaled);
    }
}

// LDS floats per wave slot: its window, later its partial sums (a v4f per
// order, map and lane).
__host__ __device__ constexpr int inv2m_slot_floats(int G)
{
    return (2 * G * 4 * WROW > 2 * G * 64 * 4) ? 2 * G * 4 * WROW : 2 * G * 64 * 4;
}

// Groups of four maps hold three waves per SIMD (136 VGPRs beside the 32 AGPRs of
// their accumulators); left alone the allocator can take two more and drop to two.
// Groups whose maps have two different |s| (NS = 2) run both spin rows beside
// the shared order chains, started from the launch's spin tables (MB.stab);
// the work list is that of the larger |s| (its first segment reaches past every
// chain start of both spin rows).  Each map's records carry the scale of its
// own spin row.
template <bool EXT, int G, int NS>
__global__ __launch_bounds__(64 * SEGI_MAX) __attribute__((amdgpu_waves_per_eu(G == 8 ? 2 : (G == 4 ? 3 : 4)))) void k_contract_inverse2_mix(
    MixBatch MB, const double* __restrict__ Rtg, const double* __restrict__ edge, const int* __restrict__ edgek,
    const double2* __restrict__ lco, const double2* __restrict__ cki, const int2* __restrict__ ckik, CkOff ckoff,
    const int4* __restrict__ work, int L, int Lp, int ckg)
{
    extern __shared__ double smem[];
    const MixMaps& maps = MB.g[blockIdx.y];
    const int slot = uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    // this wave's segment: see the work-list layout of the spin table
    const int4 d = work[(size_t)blockIdx.x * SEGI_MAX + slot];
    const int n0 = uniform(d.x), m0 = uniform(d.y), code = uniform(d.z), bounds = uniform(d.w);
    const bool item = n0 >= 0;
    const int w = code & 0xff, nseg = (code >> 8) & 0xff, lead = (code >> 16) & 0xff;
    const bool bar = (code >> 24) & 1;   // the same for every slot of the workgroup
    bool any = false;                    // does any map of the group have this (n0, m0) block?
    for (int b = 0; b < mix_n(maps); ++b) any |= (n0 < maps.L[b] && m0 < maps.L[b]);
    const double* __restrict__ Rt = Rtg;               // 1/sqrt table, L1-resident
    float* region = (float*)smem + slot * inv2m_slot_floats(G);
    SpinSet<NS> sset;
    SpinTabs<NS> tj;
    int asmax = 0;
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        sset.a[j] = MB.as[j];
        asmax = max(asmax, MB.as[j]);
        tj.val[j] = MB.stab[j];
        tj.k[j] = MB.stabk[j];
    }
    const int n = n0 + lane;
    const bool valid = item && n < L;
    const int ne = valid ? n : L - 1;
    const double nd = (double)ne;
    const int jend = (Lp >> 1) - 1;

    v4f acc[2][G];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < G; ++b) acc[c][b] = v4f{0.f, 0.f, 0.f, 0.f};
    if (item && any) {
        InvGeo geo;
        geo.lstart = max(n0, m0) & ~1;
        geo.lA = max(max(n0 + 64, m0 + 2), asmax + 1);   // every chain start lies below lA
        geo.cs = bounds & 0xffff;
        geo.ce = (int)((unsigned)bounds >> 16);
        geo.nseg = nseg;
        InvLane2<EXT, NS> st;
        bool anyscaled;
        const InvSeg g = inv2_setup<EXT, NS>(st, anyscaled, geo, w, n, m0, L, Lp, sset, ckg, lco, edge, edgek, tj, cki,
                                             ckik, ckoff);
        // the spin values come from the scaled spin rows, not chains
        const double* svl[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) { st.ks[q] = 0; svl[q] = MB.ssv[q] + ne; }
        if (EXT) anyscaled = __any(inv2_scaled(st));
        if (g.active)
            inv2m_segment<EXT, G, NS>(st, acc, g, jend, geo.lstart, ne, nd, m0,
                                      inv2_rows(nullptr, lco, m0, sset.a[0], Lp, L, sset.a[NS - 1]), Rt, svl, L,
                                      region, maps, lane, anyscaled);
    }

    if (bar) {
        // every wave of the workgroup (empty slots too) meets at this one barrier;
        // a wave's partial sums overwrite its own window, which it no longer reads
        if (item && w > 0) {
            v4f* red = (v4f*)region;
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int b = 0; b < G; ++b) red[(c * G + b) * 64 + lane] = acc[c][b];
        }
        __syncthreads();
        if (!item || w != 0) return;
    } else if (!item) {
        return;
    }
    if (!valid) return;
    // one (order, map) at a time: its FP32 sums in FP64, plus those of the later
    // segments in segment order
    const int nadd = bar ? nseg : 1;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int m = m0 + c;
#pragma unroll
        for (int b = 0; b < G; ++b) {
            if (b >= mix_n(maps)) continue;
            const int s = mix_spin(MB, maps, b);
            const double fsp = sgn(s) * ((s >= 0) ? sgn(n) : 1.0);
            const double fsm = sgn(s) * ((s < 0) ? sgn(n) : 1.0);
            const int Lb = maps.L[b];
            if (n >= Lb || m >= Lb) continue;
            double sum[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) sum[q] = (double)acc[c][b][q];
            for (int k = 1; k < nadd; ++k) {
                const v4f v = ((const v4f*)((const float*)smem + (lead + k) * inv2m_slot_floats(G)))[(c * G + b) * 64 + lane];
#pragma unroll
                for (int q = 0; q < 4; ++q) sum[q] += (double)v[q];
            }
            double2* F = maps.dst[b];
            const double2 op = mul_ipow(make_double2(sum[0], sum[1]), ((-(m + s)) % 4 + 4) % 4);
            F[(size_t)(Lb - 1 + m) * Lb + n] = make_double2(op.x * fsp, op.y * fsp);
            if (m > 0) {
                const double2 om = mul_ipow(make_double2(sum[2], sum[3]), ((m - s) % 4 + 4) % 4);
                F[(size_t)(Lb - 1 - m) * Lb + n] = make_double2(om.x * fsm, om.y * fsm);
            }
        }
    }
}

}  // namespace

namespace {
template <bool EXT, bool RL, bool SPT>
hipError_t fwd_go(const Plan& p, const SpinTable& sp, int s, const double* in0, size_t stride, const Batch& B,
                  hipStream_t st)
{
    const dim3 grid(p.nworkf4, B.n), block(64 * SEG_MAX);
    if (EXT)
        hipLaunchKernelGGL((k_contract_forward_ext<MT_FWD, RL, SPT>), grid, block, 0, st, in0, stride, B, p.rtab,
                           p.edge, p.edgek, p.cl, p.ckf, p.ckfk, sp.svalf, p.workf4, p.L, p.Lp, s, p.ckfg);
    else
        hipLaunchKernelGGL((k_contract_forward<MT_FWD, RL, SPT>), grid, block, 0, st, in0, stride, B, p.rtab, p.edge,
                           p.edgek, p.cl, p.ckf, p.ckfk, sp.svalf, p.workf4, p.L, p.Lp, s, p.ckfg);
    return hipGetLastError();
}

template <bool EXT, bool SPT>
hipError_t fwd_go_r(const Plan& p, const SpinTable& sp, int s, int real, const double* in0, size_t stride,
                    const Batch& B, hipStream_t st)
{
    return real ? fwd_go<EXT, true, SPT>(p, sp, s, in0, stride, B, st)
                : fwd_go<EXT, false, SPT>(p, sp, s, in0, stride, B, st);
}
}  // namespace

// From L = FWD_SPT_MIN_L the spin row's values come from the spin table's
// transposed rows; below, the third chain is faster (measured at L = 256 and
// 512: 6-25% slower with the table, at L = 1024 and 2048 5-7% faster).
hipError_t launch_contract_forward(const Plan& p, const SpinTable& sp, int s, int real, const double* in0,
                                   size_t stride, const Batch& B, hipStream_t st)
{
    const bool spt = p.L >= FWD_SPT_MIN_L;
    if (p.ext)
        return spt ? fwd_go_r<true, true>(p, sp, s, real, in0, stride, B, st)
                   : fwd_go_r<true, false>(p, sp, s, real, in0, stride, B, st);
    return spt ? fwd_go_r<false, true>(p, sp, s, real, in0, stride, B, st)
               : fwd_go_r<false, false>(p, sp, s, real, in0, stride, B, st);
}

hipError_t launch_spin_flip(int L, const Batch& B, hipStream_t st)
{
    const int n = L * (L + 1) / 2;
    hipLaunchKernelGGL(k_spin_flip, dim3((n + 255) / 256, B.n), dim3(256), 0, st, B, L);
    return hipGetLastError();
}

hipError_t launch_real_fold(int L, const Batch& B, hipStream_t st)
{
    const dim3 grid((L + 255) / 256, L, B.n);
    hipLaunchKernelGGL(k_real_fold, grid, dim3(256), 0, st, B, L);
    return hipGetLastError();
}

hipError_t launch_inverse_stream(const Plan& p, int real, const Batch& B, int out32, hipStream_t st)
{
    const dim3 grid((p.Lp + STR_L - 1) / STR_L, (p.L + STR_M - 1) / STR_M, B.n);
    if (out32) hipLaunchKernelGGL(k_inverse_stream<1>, grid, dim3(256), 0, st, B, p.cl, p.lco, p.L, p.Lp, real);
    else hipLaunchKernelGGL(k_inverse_stream<0>, grid, dim3(256), 0, st, B, p.cl, p.lco, p.L, p.Lp, real);
    return hipGetLastError();
}

namespace {
template <bool EXT, bool RL, bool SNEG, bool SPT = false>
hipError_t inv_tri_go(const Plan& p, const SpinTable& sp, int s, const double* in0, size_t stride, const Batch& B,
                      hipStream_t st)
{
    CkOff off;
    for (int j = 0; j < CKI_MAX; ++j) off.off[j] = p.cki_off[j];
    const dim3 grid(sp.nwtri, B.n), block(64 * SEGT_MAX);
    if (EXT)
        hipLaunchKernelGGL((k_contract_inverse_tri_ext<RL, SNEG, SPT>), grid, block, 0, st, in0, stride, B, p.rtab, p.edge,
                           p.edgek, p.lco, sp.lcos, sp.val, sp.k, sp.sval, p.cki, p.ckik, off, sp.wtri, p.L, p.Lp, s,
                           p.ckg);
    else
        hipLaunchKernelGGL((k_contract_inverse_tri<RL, SNEG, SPT>), grid, block, 0, st, in0, stride, B, p.rtab, p.edge,
                           p.edgek, p.lco, sp.lcos, sp.val, sp.k, sp.sval, p.cki, p.ckik, off, sp.wtri, p.L, p.Lp, s,
                           p.ckg);
    return hipGetLastError();
}

template <bool EXT, bool RL>
hipError_t inv_sq_go(const Plan& p, const SpinTable& sp, int s, const double* in0, size_t stride, const Batch& B,
                     hipStream_t st)
{
    CkOff off;
    for (int j = 0; j < CKI_MAX; ++j) off.off[j] = p.cki_off[j];
    const dim3 grid(sp.nwinv, B.n), block(64 * SEGI_MAX);
    if (EXT)
        hipLaunchKernelGGL((k_contract_inverse2_ext<RL>), grid, block, 0, st, in0, stride, B, p.rtab, p.edge,
                           p.edgek, p.lco, sp.val, sp.k, sp.sval, p.cki, p.ckik, off, sp.winv, p.L, p.Lp, s, p.ckg);
    else
        hipLaunchKernelGGL((k_contract_inverse2<RL>), grid, block, 0, st, in0, stride, B, p.rtab, p.edge, p.edgek,
                           p.lco, sp.val, sp.k, sp.sval, p.cki, p.ckik, off, sp.winv, p.L, p.Lp, s, p.ckg);
    return hipGetLastError();
}

template <bool EXT>
hipError_t inv_go(const Plan& p, const SpinTable& sp, int s, int real, const double* in0, size_t stride,
                  const Batch& B, hipStream_t st)
{
    // real maps have s = 0; from L = INV_TRI_SPT_MIN_L their spin values come from
    // the scaled spin rows (below, and for complex maps, the extra per-lane read
    // cost more than the chain it replaces: real L = 320..896 8-13% slower,
    // complex L = 1024 and 2048 6-10% slower; real L = 1024 6% and 2048 12% faster)
    if (real) {
        if (p.L >= INV_TRI_SPT_MIN_L) return inv_tri_go<EXT, true, false, true>(p, sp, s, in0, stride, B, st);
        return inv_tri_go<EXT, true, false>(p, sp, s, in0, stride, B, st);
    }
    if (p.L >= INV_TRI_MIN_L || g_inv_tri_all)
        return s < 0 ? inv_tri_go<EXT, false, true>(p, sp, s, in0, stride, B, st)
                     : inv_tri_go<EXT, false, false>(p, sp, s, in0, stride, B, st);
    return inv_sq_go<EXT, false>(p, sp, s, in0, stride, B, st);
}
}  // namespace

int g_inv_tri_all = 0;

// The triangle kernel runs real maps at every band-limit and complex maps from
// L = INV_TRI_MIN_L: below, a complex map's two coefficient reads per lane and
// step and its four waves per SIMD (against six for the square kernel) cost more
// than the halved chain work saves (measured at L = 256 and 512, one map and
// batches: 2-16% slower; equal at L = 1024, 17% faster at L = 2048).
hipError_t launch_contract_inverse(const Plan& p, const SpinTable& sp, int s, int real, const double* in0,
                                   size_t stride, const Batch& B, hipStream_t st)
{
    if (p.ext) return inv_go<true>(p, sp, s, real, in0, stride, B, st);
    return inv_go<false>(p, sp, s, real, in0, stride, B, st);
}

// ---- mixed precision launchers ------------------------------------------
namespace {

size_t mix_lds_forward(int G) { return (size_t)SEG_MAX * fwdm_slot_floats(G) * sizeof(float); }

template <class K>
hipError_t mix_attr(K kernel, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <bool EXT, int G, int NS, bool SPT>
hipError_t fwd_mix_go2(const Plan& p, const MixBatch& maps, hipStream_t st)
{
    const size_t lds = mix_lds_forward(G);
    hipError_t e = mix_attr(k_contract_forward_mix<EXT, G, NS, SPT>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_contract_forward_mix<EXT, G, NS, SPT>), dim3(p.nworkf4, maps.ng), dim3(64 * SEG_MAX), lds,
                       st, maps, p.rtab, p.edge, p.edgek, p.cl, p.ckf, p.ckfk, p.workf4, p.L, p.ckfg);
    return hipGetLastError();
}

// From L = FWD_SPT_MIN_L (the launch carrying its spin tables) the spin rows'
// values come from the tables, as in the FP64 forward.
template <bool EXT, int G, int NS>
hipError_t fwd_mix_go(const Plan& p, const MixBatch& maps, hipStream_t st)
{
    bool spt = p.L >= FWD_SPT_MIN_L;
    for (int j = 0; j < NS; ++j) spt = spt && maps.ssvf[j] != nullptr;
    return spt ? fwd_mix_go2<EXT, G, NS, true>(p, maps, st) : fwd_mix_go2<EXT, G, NS, false>(p, maps, st);
}

template <bool EXT, int G, int NS>
hipError_t inv_mix_go(const Plan& p, const SpinTable& wsp, const MixBatch& maps, hipStream_t st)
{
    CkOff off;
    for (int j = 0; j < CKI_MAX; ++j) off.off[j] = p.cki_off[j];
    const size_t lds = (size_t)SEGI_MAX * inv2m_slot_floats(G) * sizeof(float);
    hipError_t e = mix_attr(k_contract_inverse2_mix<EXT, G, NS>, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_contract_inverse2_mix<EXT, G, NS>), dim3(wsp.nwinv, maps.ng), dim3(64 * SEGI_MAX), lds, st,
                       maps, p.rtab, p.edge, p.edgek, p.lco, p.cki, p.ckik, off, wsp.winv, p.L, p.Lp, p.ckg);
    return hipGetLastError();
}

template <bool EXT, int NS>
hipError_t fwd_mix_g(const Plan& p, const MixBatch& maps, int G, hipStream_t st)
{
    if (G == 1) return fwd_mix_go<EXT, 1, NS>(p, maps, st);
    if (G == 2) return fwd_mix_go<EXT, 2, NS>(p, maps, st);
    if (G == 4) return fwd_mix_go<EXT, 4, NS>(p, maps, st);
    return fwd_mix_go<EXT, 8, NS>(p, maps, st);
}

template <bool EXT, int NS>
hipError_t inv_mix_g(const Plan& p, const SpinTable& wsp, const MixBatch& maps, int G, hipStream_t st)
{
    if (G == 1) return inv_mix_go<EXT, 1, NS>(p, wsp, maps, st);
    if (G == 2) return inv_mix_go<EXT, 2, NS>(p, wsp, maps, st);
    if (G == 4) return inv_mix_go<EXT, 4, NS>(p, wsp, maps, st);
    return inv_mix_go<EXT, 8, NS>(p, wsp, maps, st);
}

}  // namespace

int mix_group_max()
{
    for (int G = GMAX; G > 1; G >>= 1)
        if (mix_lds_forward(G) <= 160 * 1024 && (size_t)SEGI_MAX * inv2m_slot_floats(G) * 4 <= 160 * 1024)
            return G;
    return 1;
}

// Groups of one launch: 1..G maps each; ns in [1, NS] spin rows, every map's
// row below ns.
bool mix_ok(const MixBatch& maps, int G, int NS)
{
    if (maps.ng < 1 || maps.ng > MIXG || G > GMAX || NS < 1 || NS > NSMAX || maps.ns < 1 || maps.ns > NS)
        return false;
    for (int g = 0; g < maps.ng; ++g) {
        const MixMaps& m = maps.g[g];
        if (mix_n(m) < 1 || mix_n(m) > G) return false;
        for (int b = 0; b < mix_n(m); ++b)
            if (mix_row(m, b) >= maps.ns) return false;
    }
    return true;
}

hipError_t launch_contract_forward_mix(const Plan& p, const MixBatch& maps, int G, int NS, hipStream_t st)
{
    if (!mix_ok(maps, G, NS)) return hipErrorInvalidValue;
    if (p.ext) return NS == 2 ? fwd_mix_g<true, 2>(p, maps, G, st) : fwd_mix_g<true, 1>(p, maps, G, st);
    return NS == 2 ? fwd_mix_g<false, 2>(p, maps, G, st) : fwd_mix_g<false, 1>(p, maps, G, st);
}

hipError_t launch_contract_inverse_mix(const Plan& p, const SpinTable& wsp, const MixBatch& maps, int G, int NS,
                                       hipStream_t st)
{
    if (!mix_ok(maps, G, NS)) return hipErrorInvalidValue;
    if (p.ext) return NS == 2 ? inv_mix_g<true, 2>(p, wsp, maps, G, st) : inv_mix_g<true, 1>(p, wsp, maps, G, st);
    return NS == 2 ? inv_mix_g<false, 2>(p, wsp, maps, G, st) : inv_mix_g<false, 1>(p, wsp, maps, G, st);
}

}  // namespace mw
