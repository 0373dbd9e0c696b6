// The O(L^3) part of the MW transforms: Wigner Delta = d(pi/2) generated on the
// fly in FP64 and contracted against the Fourier coefficients.
//
// Forward, Eq.(flm_wig) folded with Eq.(Fmm_sym1):
//   f_{l,+-m} = (-1)^s i^{+-m+s} sqrt((2l+1)/4pi) sum_{n>=0} Delta^l_{n,+-m} Delta^l_{n,-s} H_{+-m,n}
// A wavefront owns 64 consecutive degrees l (one per lane) and MT orders m.
// Each lane runs the three-term recursion of row m of Delta^l along the second
// index n = l .. 0 (beta = pi/2 member of the recursion family of Trapani &
// Navaza, Sec. V-C):
//   sqrt((l+n)(l-n+1)) D_{m,n-1} = -2m D_{m,n} - sqrt((l-n)(l+n+1)) D_{m,n+1},
// started from the edge value D_{m,l} = 2^-l sqrt(binom(2l, l+m)).  The row |s|
// (the spin factor) runs as one more chain in the same lane.  H_{+-m,n} is the
// same for all lanes (scalar loads), the sqrt factors come from an LDS table,
// and the sum over n accumulates in registers.
//
// Inverse, Eq.(Fmm):
//   F_{+-m,n} = (-1)^s i^{-(+-m+s)} sum_l sqrt((2l+1)/4pi) Delta^l_{n,+-m} Delta^l_{n,-s} f_{l,+-m}
// A wavefront owns 64 consecutive n (one per lane) and MT orders m.  Each lane
// runs the three-term recursion of Delta^l_{n,m} in the degree l (upward from
// l0 = max(n, m)), so the sum over l again accumulates in registers; the spin
// factor Delta^l_{n,|s|} runs as one more chain, started from a table.
//
// Chains whose start value is below 2^-900 (only for L > ~900) carry an extra
// exponent: the stored value is x = D * 2^(600k); while k > 0 the chain's
// contributions are masked (|D| < 2^-300) and it is rescaled when |x| > 2^300.
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

constexpr double EXT_UP = 0x1p300;
constexpr double EXT_DOWN = 0x1p-600;

// ===========================================================================
// Forward contraction
// ===========================================================================
template <int MT, bool EXT>
struct FwdLane {
    double dc[MT], dn[MT];      // D_{m,n} and D_{m,n+1}
    double sc, sn;              // spin row |s|
    double2 ap[MT][2], am[MT][2];  // accumulators for +m / -m, split by parity of n
    int k[MT], ks;              // exponent levels (EXT)
    double anext;               // sqrt((l-n)(l+n+1)) of the current step
};

template <int MT, bool EXT, int PAR>
__device__ __forceinline__ void fwd_step(FwdLane<MT, EXT>& st, int n, int le, int L, int mb, int as,
                                         const double2* __restrict__ H, const double2* sq, bool& anyscaled)
{
    // contributions of D_{.,n}
    double seff = st.sc;
    if (EXT) seff = (st.ks == 0) ? seff : 0.0;
#pragma unroll
    for (int c = 0; c < MT; ++c) {
        const int mrow = min(mb + c, L - 1);
        const double2 hp = H[(size_t)(L - 1 + mrow) * L + n];
        const double2 hm = H[(size_t)(L - 1 - mrow) * L + n];
        double d = st.dc[c];
        if (EXT) d = (st.k[c] == 0) ? d : 0.0;
        const double pr = d * seff;
        st.ap[c][PAR].x = fma(pr, hp.x, st.ap[c][PAR].x);
        st.ap[c][PAR].y = fma(pr, hp.y, st.ap[c][PAR].y);
        st.am[c][PAR].x = fma(pr, hm.x, st.am[c][PAR].x);
        st.am[c][PAR].y = fma(pr, hm.y, st.am[c][PAR].y);
    }
    if (n == 0) return;
    // advance every chain from (n, n+1) to (n-1, n)
    const double2 t1 = sq[le + n];
    const double2 t2 = sq[max(le - n + 1, 0)];
    const double an = t1.x * t2.x;
    const double nra = -(t1.y * t2.y);
#pragma unroll
    for (int c = 0; c < MT; ++c) {
        const double tm = 2.0 * (double)(mb + c);
        const double d = fma(tm, st.dc[c], st.anext * st.dn[c]) * nra;
        st.dn[c] = st.dc[c];
        st.dc[c] = d;
    }
    {
        const double d = fma(2.0 * (double)as, st.sc, st.anext * st.sn) * nra;
        st.sn = st.sc;
        st.sc = d;
    }
    st.anext = an;
    if (EXT && anyscaled) {
        bool still = false;
#pragma unroll
        for (int c = 0; c < MT; ++c) {
            if (st.k[c] > 0 && fabs(st.dc[c]) > EXT_UP) {
                st.dc[c] *= EXT_DOWN; st.dn[c] *= EXT_DOWN; st.k[c] -= 1;
            }
            still |= st.k[c] > 0;
        }
        if (st.ks > 0 && fabs(st.sc) > EXT_UP) { st.sc *= EXT_DOWN; st.sn *= EXT_DOWN; st.ks -= 1; }
        still |= st.ks > 0;
        anyscaled = __any(still);
    }
}

template <int MT, bool EXT>
__global__ __launch_bounds__(256) void k_contract_forward(
    const double2* __restrict__ H, double2* __restrict__ flm, const double2* __restrict__ sqtab,
    const double* __restrict__ edge, const int* __restrict__ edgek, const double* __restrict__ cl,
    const int2* __restrict__ work, int nwork, int L, int s)
{
    extern __shared__ double2 sq[];
    for (int i = threadIdx.x; i < 2 * L + 3; i += blockDim.x) sq[i] = sqtab[i];
    __syncthreads();
    const int wv = uniform(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    if (wv >= nwork) return;
    const int lane = threadIdx.x & 63;
    const int l0 = uniform(work[wv].x), mb = uniform(work[wv].y);
    const int l = l0 + lane;
    const bool valid = l < L;
    const int le = valid ? l : L - 1;
    const int as = s < 0 ? -s : s;

    FwdLane<MT, EXT> st;
    double start[MT];
    int startk[MT];
#pragma unroll
    for (int c = 0; c < MT; ++c) {
        const int m = mb + c;
        const bool ok = valid && m <= l;
        start[c] = ok ? edge[(size_t)l * (l + 1) / 2 + m] : 0.0;
        startk[c] = (EXT && ok) ? edgek[(size_t)l * (l + 1) / 2 + m] : 0;
        st.dc[c] = 0.0; st.dn[c] = 0.0; st.k[c] = 0;
        st.ap[c][0] = st.ap[c][1] = st.am[c][0] = st.am[c][1] = make_double2(0.0, 0.0);
    }
    const bool oks = valid && as <= l;
    const double starts = oks ? edge[(size_t)le * (le + 1) / 2 + as] : 0.0;
    const int startks = (EXT && oks) ? edgek[(size_t)le * (le + 1) / 2 + as] : 0;
    st.sc = 0.0; st.sn = 0.0; st.ks = 0; st.anext = 0.0;
    bool anyscaled = EXT;

    const int nmax = min(l0 + 63, L - 1);
    int n = nmax;
    // phase A: lanes start at their own n = l
    for (; n >= l0; --n) {
        if (n == l) {
#pragma unroll
            for (int c = 0; c < MT; ++c) { st.dc[c] = start[c]; st.k[c] = startk[c]; }
            st.sc = starts; st.ks = startks;
        }
        if (EXT) {
            bool sc = false;
#pragma unroll
            for (int c = 0; c < MT; ++c) sc |= st.k[c] > 0;
            sc |= st.ks > 0;
            anyscaled = __any(sc) || (n > l0);
        }
        if (n & 1) fwd_step<MT, EXT, 1>(st, n, le, L, mb, as, H, sq, anyscaled);
        else fwd_step<MT, EXT, 0>(st, n, le, L, mb, as, H, sq, anyscaled);
    }
    // phase B: every lane running
    for (; n >= 1; n -= 2) {
        if (n & 1) {
            fwd_step<MT, EXT, 1>(st, n, le, L, mb, as, H, sq, anyscaled);
            fwd_step<MT, EXT, 0>(st, n - 1, le, L, mb, as, H, sq, anyscaled);
        } else {
            fwd_step<MT, EXT, 0>(st, n, le, L, mb, as, H, sq, anyscaled);
            fwd_step<MT, EXT, 1>(st, n - 1, le, L, mb, as, H, sq, anyscaled);
        }
    }
    if (n == 0) fwd_step<MT, EXT, 0>(st, 0, le, L, mb, as, H, sq, anyscaled);

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
        flm[(size_t)l * l + l + m] = make_double2(op.x * base * fp, op.y * base * fp);
        if (m > 0) {
            double2 om = mul_ipow(sm, ((-m + s) % 4 + 4) % 4);
            flm[(size_t)l * l + l - m] = make_double2(om.x * base * fm, om.y * base * fm);
        }
    }
}

// ===========================================================================
// Inverse contraction
// ===========================================================================
template <int MT, bool EXT>
struct InvLane {
    double dc[MT], dp[MT];     // Delta^l_{n,m}, Delta^{l-1}_{n,m}
    double sc, sp;             // Delta^l_{n,|s|}, Delta^{l-1}_{n,|s|}
    double2 ap[MT], am[MT];
    int k[MT], ks;
    double sprev;              // sqrt(l^2 - n^2) of the current step
};

template <int MT, bool EXT, int PAR>
__device__ __forceinline__ void inv_step(InvLane<MT, EXT>& st, int l, int ne, int L, int mb, int as,
                                         int s, int real, const double2* __restrict__ flm,
                                         const double2* __restrict__ lco, const double* __restrict__ cl,
                                         const double2* sq, bool& anyscaled)
{
    // contributions at degree l
    double seff = st.sc * cl[l];
    if (EXT) seff = (st.ks == 0) ? seff : 0.0;
#pragma unroll
    for (int c = 0; c < MT; ++c) {
        const int m = min(mb + c, l);   // orders above l contribute nothing (chain is 0)
        double2 fpv = flm[(size_t)l * l + l + m];
        double2 fmv;
        if (real) fmv = (m & 1) ? make_double2(-fpv.x, fpv.y) : make_double2(fpv.x, -fpv.y);
        else fmv = flm[(size_t)l * l + l - m];
        // (-1)^l on the +m sum for s >= 0, on the -m sum for s < 0
        if (PAR) {
            if (s >= 0) fpv = make_double2(-fpv.x, -fpv.y);
            else fmv = make_double2(-fmv.x, -fmv.y);
        }
        double d = st.dc[c];
        if (EXT) d = (st.k[c] == 0) ? d : 0.0;
        const double pr = d * seff;
        st.ap[c].x = fma(pr, fpv.x, st.ap[c].x);
        st.ap[c].y = fma(pr, fpv.y, st.ap[c].y);
        st.am[c].x = fma(pr, fmv.x, st.am[c].x);
        st.am[c].y = fma(pr, fmv.y, st.am[c].y);
    }
    if (l + 1 >= L) return;
    // n-dependent factors X_n(l) = n / sqrt((l+1)^2 - n^2), Y_n(l) = sqrt(l^2-n^2)/sqrt((l+1)^2-n^2)
    const double2 t1 = sq[max(l + 1 - ne, 0)];
    const double2 t2 = sq[l + 1 + ne];
    const double rs = t1.y * t2.y;
    const double snew = t1.x * t2.x;
    const double xn = (double)ne * rs;
    const double yn = st.sprev * rs;
    st.sprev = snew;
#pragma unroll
    for (int c = 0; c < MT; ++c) {
        const double2 pq = lco[(size_t)min(mb + c, L - 1) * L + l];
        const double d = fma(pq.x * xn, st.dc[c], (pq.y * yn) * st.dp[c]);
        st.dp[c] = st.dc[c];
        st.dc[c] = d;
    }
    {
        const double2 pq = lco[(size_t)as * L + l];
        const double d = fma(pq.x * xn, st.sc, (pq.y * yn) * st.sp);
        st.sp = st.sc;
        st.sc = d;
    }
    if (EXT && anyscaled) {
        bool still = false;
#pragma unroll
        for (int c = 0; c < MT; ++c) {
            if (st.k[c] > 0 && fabs(st.dc[c]) > EXT_UP) {
                st.dc[c] *= EXT_DOWN; st.dp[c] *= EXT_DOWN; st.k[c] -= 1;
            }
            still |= st.k[c] > 0;
        }
        if (st.ks > 0 && fabs(st.sc) > EXT_UP) { st.sc *= EXT_DOWN; st.sp *= EXT_DOWN; st.ks -= 1; }
        still |= st.ks > 0;
        anyscaled = __any(still);
    }
}

template <int MT, bool EXT>
__global__ __launch_bounds__(256) void k_contract_inverse(
    const double2* __restrict__ flm, double2* __restrict__ F, const double2* __restrict__ sqtab,
    const double* __restrict__ edge, const int* __restrict__ edgek, const double2* __restrict__ lco,
    const double* __restrict__ cl, const double* __restrict__ stab, const int* __restrict__ stabk,
    const int2* __restrict__ work, int nwork, int L, int s, int real)
{
    extern __shared__ double2 sq[];
    for (int i = threadIdx.x; i < 2 * L + 3; i += blockDim.x) sq[i] = sqtab[i];
    __syncthreads();
    const int wv = uniform(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    if (wv >= nwork) return;
    const int lane = threadIdx.x & 63;
    const int n0 = uniform(work[wv].x), mb = uniform(work[wv].y);
    const int n = n0 + lane;
    const bool valid = n < L;
    const int ne = valid ? n : L - 1;
    const int as = s < 0 ? -s : s;
    const int lstart = max(n0, mb);

    InvLane<MT, EXT> st;
    double start[MT];
    int startk[MT], lz[MT];
#pragma unroll
    for (int c = 0; c < MT; ++c) {
        const int m = mb + c;
        const bool ok = valid && m < L;
        lz[c] = max(n, m);
        double v = 0.0;
        int kk = 0;
        if (ok) {
            if (n >= m) {
                const size_t i = (size_t)n * (n + 1) / 2 + m;
                v = ((n - m) & 1) ? -edge[i] : edge[i];
                if (EXT) kk = edgek[i];
            } else {
                const size_t i = (size_t)m * (m + 1) / 2 + n;
                v = edge[i];
                if (EXT) kk = edgek[i];
            }
        }
        start[c] = v; startk[c] = kk;
        st.dc[c] = 0.0; st.dp[c] = 0.0; st.k[c] = 0;
        st.ap[c] = st.am[c] = make_double2(0.0, 0.0);
    }
    // spin chain: from the table at lstart (and lstart-1) when already running,
    // else injected at its own start l0s = max(n, |s|)
    const int l0s = max(n, as);
    st.sc = 0.0; st.sp = 0.0; st.ks = 0;
    double starts = 0.0;
    int startks = 0;
    if (valid) {
        if (l0s <= lstart) {
            double v1 = stab[(size_t)lstart * L + n];
            int k1 = EXT ? stabk[(size_t)lstart * L + n] : 0;
            double v0 = 0.0;
            int k0 = k1;
            if (lstart >= 1) {
                v0 = stab[(size_t)(lstart - 1) * L + n];
                k0 = EXT ? stabk[(size_t)(lstart - 1) * L + n] : 0;
            }
            if (EXT) {
                // bring both to the deeper scale level
                const int kk = max(k0, k1);
                v1 = ldexp(v1, 600 * (kk - k1));
                v0 = ldexp(v0, 600 * (kk - k0));
                st.ks = kk;
            }
            st.sc = v1; st.sp = v0;
        } else if (l0s < L) {
            starts = stab[(size_t)l0s * L + n];
            startks = EXT ? stabk[(size_t)l0s * L + n] : 0;
        }
    }
    st.sprev = sq[max(lstart - ne, 0)].x * sq[lstart + ne].x;
    bool anyscaled = EXT;
    // phase A: injections happen while l < lA
    const int lA = min(L, max(max(n0 + 64, mb + MT), as + 1));
    int l = lstart;
    for (; l < lA; ++l) {
#pragma unroll
        for (int c = 0; c < MT; ++c)
            if (l == lz[c]) { st.dc[c] = start[c]; st.k[c] = startk[c]; }
        if (l == l0s && l0s > lstart) { st.sc = starts; st.ks = startks; }
        if (EXT) {
            bool sc = false;
#pragma unroll
            for (int c = 0; c < MT; ++c) sc |= st.k[c] > 0;
            sc |= st.ks > 0;
            anyscaled = __any(sc) || true;
        }
        if (l & 1) inv_step<MT, EXT, 1>(st, l, ne, L, mb, as, s, real, flm, lco, cl, sq, anyscaled);
        else inv_step<MT, EXT, 0>(st, l, ne, L, mb, as, s, real, flm, lco, cl, sq, anyscaled);
    }
    for (; l + 1 < L; l += 2) {
        if (l & 1) {
            inv_step<MT, EXT, 1>(st, l, ne, L, mb, as, s, real, flm, lco, cl, sq, anyscaled);
            inv_step<MT, EXT, 0>(st, l + 1, ne, L, mb, as, s, real, flm, lco, cl, sq, anyscaled);
        } else {
            inv_step<MT, EXT, 0>(st, l, ne, L, mb, as, s, real, flm, lco, cl, sq, anyscaled);
            inv_step<MT, EXT, 1>(st, l + 1, ne, L, mb, as, s, real, flm, lco, cl, sq, anyscaled);
        }
    }
    if (l < L) {
        if (l & 1) inv_step<MT, EXT, 1>(st, l, ne, L, mb, as, s, real, flm, lco, cl, sq, anyscaled);
        else inv_step<MT, EXT, 0>(st, l, ne, L, mb, as, s, real, flm, lco, cl, sq, anyscaled);
    }

    if (!valid) return;
#pragma unroll
    for (int c = 0; c < MT; ++c) {
        const int m = mb + c;
        if (m >= L) continue;
        const double fsp = sgn(s) * ((s >= 0) ? sgn(n) : 1.0);
        const double fsm = sgn(s) * ((s < 0) ? sgn(n) : 1.0);
        double2 op = mul_ipow(st.ap[c], ((-(m + s)) % 4 + 4) % 4);
        F[(size_t)(L - 1 + m) * L + n] = make_double2(op.x * fsp, op.y * fsp);
        if (m > 0) {
            double2 om = mul_ipow(st.am[c], ((m - s) % 4 + 4) % 4);
            F[(size_t)(L - 1 - m) * L + n] = make_double2(om.x * fsm, om.y * fsm);
        }
    }
}

template <class K>
hipError_t set_lds(K kernel, size_t bytes)
{
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

hipError_t launch_contract_forward(const Plan& p, int s, int real, const double2* H, double2* flm,
                                   hipStream_t st)
{
    (void)real;
    const size_t lds = (size_t)(2 * p.L + 3) * sizeof(double2);
    const int threads = 256, wpb = threads / 64;
    const dim3 grid((p.nworkf + wpb - 1) / wpb);
    hipError_t e;
    if (p.ext) {
        auto k = k_contract_forward<MT_FWD, true>;
        if ((e = set_lds(k, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k, grid, dim3(threads), lds, st, H, flm, p.sqtab, p.edge, p.edgek, p.cl,
                           p.workf, p.nworkf, p.L, s);
    } else {
        auto k = k_contract_forward<MT_FWD, false>;
        if ((e = set_lds(k, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k, grid, dim3(threads), lds, st, H, flm, p.sqtab, p.edge, p.edgek, p.cl,
                           p.workf, p.nworkf, p.L, s);
    }
    return hipGetLastError();
}

hipError_t launch_contract_inverse(const Plan& p, const SpinTable& sp, int s, int real,
                                   const double2* flm, double2* F, hipStream_t st)
{
    const size_t lds = (size_t)(2 * p.L + 3) * sizeof(double2);
    const int threads = 256, wpb = threads / 64;
    const dim3 grid((p.nworki + wpb - 1) / wpb);
    hipError_t e;
    if (p.ext) {
        auto k = k_contract_inverse<MT_INV, true>;
        if ((e = set_lds(k, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k, grid, dim3(threads), lds, st, flm, F, p.sqtab, p.edge, p.edgek, p.lco,
                           p.cl, sp.val, sp.k, p.worki, p.nworki, p.L, s, real);
    } else {
        auto k = k_contract_inverse<MT_INV, false>;
        if ((e = set_lds(k, lds)) != hipSuccess) return e;
        hipLaunchKernelGGL(k, grid, dim3(threads), lds, st, flm, F, p.sqtab, p.edge, p.edgek, p.lco,
                           p.cl, sp.val, sp.k, p.worki, p.nworki, p.L, s, real);
    }
    return hipGetLastError();
}

}  // namespace mw
