// Host-side construction of the per-band-limit tables (long double arithmetic,
// rounded once to double when uploaded).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "mw_internal.h"

namespace mw {

namespace {

using ld = long double;
using cld = std::complex<long double>;
const ld PI_L = 3.141592653589793238462643383279502884L;

int next_pow2(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// In-place iterative radix-2 DFT, X_j = sum_k x_k exp(-2 pi i j k / N).
void host_fft(std::vector<cld>& a)
{
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        for (size_t i = 0; i < n; i += len) {
            for (size_t k = 0; k < len / 2; ++k) {
                ld ang = -2.0L * PI_L * (ld)k / (ld)len;
                cld w(cosl(ang), sinl(ang));
                cld u = a[i + k], v = a[i + k + len / 2] * w;
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
        }
    }
}

// Split a positive value into mantissa * 2^(-EXT_STEP k) with the mantissa
// kept above 2^-EXT_LIMIT whenever k > 0.
void split_ext(ld v, double& x, int& k)
{
    if (v == 0.0L) { x = 0.0; k = 0; return; }
    int e = ilogbl(v);
    k = 0;
    if (e < -EXT_LIMIT) k = (-EXT_LIMIT - e + EXT_STEP - 1) / EXT_STEP;
    x = (double)ldexpl(v, EXT_STEP * k);
}

// Delta^l_{m,l} = 2^-l sqrt(binom(2l, l+m)) for 0 <= m <= l < L, by the exact
// ratio recurrences in long double (no underflow for l < 8192).
std::vector<ld> edge_values(int L)
{
    std::vector<ld> E((size_t)L * (L + 1) / 2);
    ld e0 = 1.0L;
    for (int l = 0; l < L; ++l) {
        if (l > 0) e0 *= sqrtl((2.0L * l - 1.0L) / (2.0L * l));
        size_t base = (size_t)l * (l + 1) / 2;
        ld v = e0;
        E[base] = v;
        for (int m = 1; m <= l; ++m) {
            v *= sqrtl((ld)(l - m + 1) / (ld)(l + m));
            E[base + m] = v;
        }
    }
    return E;
}

// Delta^l_{a,b} for l = max(a,b) .. L-1 by the upward degree recursion at beta = pi/2
// (symmetric in a, b), started from the edge value; out[l] (0 for l < max(a,b)).
void degree_chain(const std::vector<ld>& E, int L, int a, int b, std::vector<ld>& out)
{
    out.assign(L, 0.0L);
    const int l0 = std::max(a, b);
    if (l0 >= L) return;
    auto edge = [&](int l, int k) { return E[(size_t)l * (l + 1) / 2 + k]; };
    ld dcur = (a >= b) ? ((((a - b) & 1) ? -1.0L : 1.0L) * edge(a, b)) : edge(b, a);
    ld dprev = 0.0L;
    for (int l = l0; l < L; ++l) {
        out[l] = dcur;
        if (l + 1 >= L) break;
        ld dnext = 0.0L;
        if (l > 0) {
            ld num = -(2.0L * l + 1.0L) * (ld)a * (ld)b * dcur -
                     (ld)(l + 1) * sqrtl(((ld)l * l - (ld)a * a) * ((ld)l * l - (ld)b * b)) * dprev;
            ld den = (ld)l * sqrtl(((ld)(l + 1) * (l + 1) - (ld)a * a) * ((ld)(l + 1) * (l + 1) - (ld)b * b));
            dnext = num / den;
        }
        dprev = dcur;
        dcur = dnext;
    }
}

// Row m of Delta^c by the three-term recursion in the second index from the edge:
// out[n] = Delta^c_{m,n}, n = 0..c.
void row_chain(const std::vector<ld>& E, int c, int m, std::vector<ld>& out)
{
    out.assign(c + 1, 0.0L);
    ld dn = E[(size_t)c * (c + 1) / 2 + m], dn1 = 0.0L;
    out[c] = dn;
    for (int n = c; n >= 1; --n) {
        ld an = sqrtl((ld)(c + n) * (ld)(c - n + 1));
        ld an1 = sqrtl((ld)(c - n) * (ld)(c + n + 1));
        ld dm1 = -(2.0L * m * dn + an1 * dn1) / an;
        dn1 = dn;
        dn = dm1;
        out[n - 1] = dn;
    }
}

void split_signed(ld v, double& x, int& k)
{
    split_ext(fabsl(v), x, k);
    if (v < 0) x = -x;
}

template <class T>
int upload(const std::vector<T>& h, T** d, size_t& bytes, std::string& err)
{
    size_t nb = h.size() * sizeof(T);
    if (nb == 0) nb = sizeof(T);
    if (hipMalloc((void**)d, nb) != hipSuccess) { err = "hipMalloc of plan table failed"; return -2; }
    if (!h.empty() && hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
        err = "hipMemcpy of plan table failed";
        return -3;
    }
    bytes += nb;
    return 0;
}

}  // namespace

static std::vector<int4> forward_work(const Plan& p);   // below

int g_split_min_n2 = 16384;

// Slot of frequency j in the stored kernel spectra (bhat, what, whatc): j
// itself, or on a split plan (N2 larger than the 8192-point transforms the LDS
// holds, L > 2048) the de-interleaved order [even j | odd j] that the
// half-length convolutions of the Fourier kernels read.
static int spectrum_slot(int j, int N2, bool split)
{
    if (!split) return j;
    return (j & 1) ? N2 / 2 + (j >> 1) : (j >> 1);
}

// Chain segmentation for band-limit L: up to smax waves of a workgroup share
// each chain, in segments of seg (a multiple of 64) degrees or rows, nseg of
// them over the whole range; false if more than smax would be needed.
static bool segment_chains(int L, int smax, int& seg, int& nseg)
{
    const int sz = 64 * std::max(1, (L + 64 * smax - 1) / (64 * smax));
    seg = (sz < L) ? sz : (L + 63) / 64 * 64 + 64;
    nseg = (seg < L) ? (L + seg - 1) / seg : 1;
    return nseg <= smax;
}

// Grid of the checkpoint planes for segments of length seg: c = k*g, 0 < c < L,
// k < n.  Up to L = 1024 the planes are four times denser than the segments
// (at least 16 apart, at most 15 planes), so that a chain group can choose
// boundaries that split its own range evenly; above, one plane per segment
// length (the planes hold O(L^2) values each).
static void ck_grid(int L, int seg, int& g, int& n)
{
    g = (L <= 1024) ? std::max(16, seg / 4) : seg;
    n = (L - 1) / g + 1;
}

// l-recursion factors at beta = pi/2, split into an m part (this table) and an
// n part formed in the kernel:
//  Delta^{l+1} = Pu_m(l) X_n(l) Delta^l + Qu_m(l) Y_n(l) Delta^{l-1}
//  Pu_m(l) = -(2l+1) m / (l sqrt((l+1)^2 - m^2)),  Qu_m(l) = -(l+1)/l sqrt((l^2-m^2)/((l+1)^2-m^2))
// The inverse runs the chains scaled, e_l = h_m(l) Delta^l, with h_m(m) =
// h_m(m+1) = 1 and h_m(l+1) = h_m(l-1) / Qu_m(l), so that the Delta^{l-1} term
// has coefficient 1:  e_{l+1} = Pu'_m(l) X_n(l) e_l + Y_n(l) e_{l-1},
// Pu'_m(l) = Pu_m(l) h_m(l+1) / h_m(l).  |Qu_m(l)| is close to 1 away from
// l = m, so h stays in [1, 5] up to L = 2048.  Entry [m*Lp + l] holds
// (Pu'_m(l), h_m(l)); h = 1 where the chain does not exist (l < m, l >= L).
static std::vector<double2> lrec_factors(int L, int Lp)
{
    std::vector<double2> lco((size_t)L * Lp, make_double2(0.0, 1.0));
    for (int m = 0; m < L; ++m) {
        ld hprev = 1.0L, hcur = 1.0L;   // h_m(l-1), h_m(l) at l = m
        for (int l = m; l < L; ++l) {
            const ld a = (ld)(l + 1) * (l + 1) - (ld)m * m;
            const ld pu = (l == 0) ? 0.0L : -(2.0L * l + 1.0L) * (ld)m / ((ld)l * sqrtl(a));
            ld hnext = 1.0L;   // h_m(l+1)
            if (l > m) {
                const ld b = (ld)l * l - (ld)m * m;
                const ld qu = -((ld)(l + 1) / (ld)l) * sqrtl(b / a);
                hnext = hprev / qu;
            }
            lco[(size_t)m * Lp + l] = make_double2((double)(pu * hnext / hcur), (double)hcur);
            hprev = hcur;
            hcur = hnext;
        }
    }
    return lco;
}

int build_plan(int L, Plan& p, std::string& err)
{
    p = Plan();
    p.L = L;
    p.N1 = 2 * L - 1;
    p.Lp = L + (L & 1);
    p.N2 = std::max(16, next_pow2(4 * L - 3));
    p.logN2 = 0;
    while ((1 << p.logN2) < p.N2) ++p.logN2;
    p.split = p.N2 >= g_split_min_n2;
    const int N1 = p.N1, N2 = p.N2;
    int rc;

    // 1/sqrt table, shifted: rt[j] = 1/sqrt(j-1), rt[0] = rt[1] = 0
    std::vector<double> rt(2 * L + 8, 0.0);
    for (int j = 2; j < (int)rt.size(); ++j) rt[j] = (double)(1.0L / sqrtl((ld)(j - 1)));
    if ((rc = upload(rt, &p.rtab, p.bytes, err))) return rc;

    // edge table
    std::vector<ld> E = edge_values(L);
    std::vector<double> ex(E.size());
    std::vector<int> ek(E.size());
    for (size_t i = 0; i < E.size(); ++i) {
        split_ext(E[i], ex[i], ek[i]);
        if (ek[i]) p.ext = true;
    }
    {
        std::vector<double> sq2((size_t)L * L);
        std::vector<int> sk2((size_t)L * L);
        for (int m = 0; m < L; ++m)
            for (int n = 0; n < L; ++n) {
                const size_t i = (n >= m) ? (size_t)n * (n + 1) / 2 + m : (size_t)m * (m + 1) / 2 + n;
                const bool neg = n >= m && ((n - m) & 1);
                sq2[(size_t)m * L + n] = neg ? -ex[i] : ex[i];
                sk2[(size_t)m * L + n] = ek[i];
            }
        if ((rc = upload(sq2, &p.edge, p.bytes, err))) return rc;
        if ((rc = upload(sk2, &p.edgek, p.bytes, err))) return rc;
    }

    const std::vector<double2> lco = lrec_factors(L, p.Lp);
    if ((rc = upload(lco, &p.lco, p.bytes, err))) return rc;

    std::vector<double> cl(L);
    for (int l = 0; l < L; ++l) cl[l] = (double)sqrtl((2.0L * l + 1.0L) / (4.0L * PI_L));
    if ((rc = upload(cl, &p.cl, p.bytes, err))) return rc;

    // Fourier tables
    std::vector<double2> tw(N2);
    for (int e = 0; e < N2; ++e) {
        ld a = -2.0L * PI_L * (ld)e / (ld)N2;
        tw[e] = make_double2((double)cosl(a), (double)sinl(a));
    }
    if ((rc = upload(tw, &p.tw, p.bytes, err))) return rc;

    std::vector<cld> c(N1);
    std::vector<double2> chirp(N1);
    for (int j = 0; j < N1; ++j) {
        long long r = ((long long)j * j) % (2LL * N1);
        ld a = -PI_L * (ld)r / (ld)N1;
        c[j] = cld(cosl(a), sinl(a));
        chirp[j] = make_double2((double)c[j].real(), (double)c[j].imag());
    }
    if ((rc = upload(chirp, &p.chirp, p.bytes, err))) return rc;

    std::vector<cld> bv(N2, cld(0, 0));
    for (int k = 0; k < N1; ++k) {
        bv[k] = std::conj(c[k]);
        if (k) bv[N2 - k] = std::conj(c[k]);
    }
    host_fft(bv);
    std::vector<double2> bh(N2);
    for (int j = 0; j < N2; ++j) {
        cld v = bv[j] / (ld)N2;
        bh[(size_t)spectrum_slot(j, N2, p.split)] = make_double2((double)v.real(), (double)v.imag());
    }
    if ((rc = upload(bh, &p.bhat, p.bytes, err))) return rc;

    // weights of the theta convolution (Sec. IV-D): w(+-1) = +-i pi/2, 0 for other
    // odd k, 2/(1-k^2) for even k; placed at k mod N2 for |k| <= 2(L-1).
    std::vector<cld> wv(N2, cld(0, 0));
    for (int k = -2 * (L - 1); k <= 2 * (L - 1); ++k) {
        cld w;
        if (k == 1) w = cld(0, PI_L / 2);
        else if (k == -1) w = cld(0, -PI_L / 2);
        else if (k % 2 != 0) w = cld(0, 0);
        else w = cld(2.0L / (1.0L - (ld)k * (ld)k), 0);
        wv[((k % N2) + N2) % N2] += w;
    }
    host_fft(wv);
    std::vector<double2> wh(N2);
    for (int j = 0; j < N2; ++j) {
        cld v = wv[j] * (2.0L * PI_L / (ld)N2);
        wh[(size_t)spectrum_slot(j, N2, p.split)] = make_double2((double)v.real(), (double)v.imag());
    }
    if ((rc = upload(wh, &p.what, p.bytes, err))) return rc;
    for (auto& v : wh) v.y = -v.y;   // conjugate spectrum, for the adjoint's correlation
    if ((rc = upload(wh, &p.whatc, p.bytes, err))) return rc;
    {
        // the even part w_e(k) = (w(k) + w(-k))/2 of the weights (2/(1-k^2) at even
        // k, zero at odd k), for the paired theta stage, in frequency order, and the
        // sum of w_e over |k| <= L-1
        std::vector<cld> we(N2, cld(0, 0));
        ld sum = 0.0L;
        for (int k = -2 * (L - 1); k <= 2 * (L - 1); k += 2) {
            const ld v = 2.0L / (1.0L - (ld)k * (ld)k);
            we[((k % N2) + N2) % N2] += cld(v, 0);
            if (k >= -(L - 1) && k <= L - 1) sum += v;
        }
        host_fft(we);
        std::vector<double2> wes(N2);
        for (int j = 0; j < N2; ++j) {
            const cld v = we[j] * (2.0L * PI_L / (ld)N2);
            wes[j] = make_double2((double)v.real(), (double)v.imag());
        }
        if ((rc = upload(wes, &p.whate, p.bytes, err))) return rc;
        p.wsum_e = (double)sum;
    }

    std::vector<double2> th(N1);
    for (int k = 0; k < N1; ++k) {
        int mp = (k <= L - 1) ? k : k - N1;
        ld a = -PI_L * (ld)mp / (ld)N1;
        ld sc = 1.0L / (2.0L * PI_L * (ld)N1);
        th[k] = make_double2((double)(cosl(a) * sc), (double)(sinl(a) * sc));
    }
    if ((rc = upload(th, &p.thtw, p.bytes, err))) return rc;
    {
        // e^{-i m' pi/N1} chirp_k, rounded once (the theta stages' chirp and twiddle product)
        std::vector<double2> wc(N1);
        for (int k = 0; k < N1; ++k) {
            const int mp = (k <= L - 1) ? k : k - N1;
            const ld a = -PI_L * (ld)mp / (ld)N1;
            const cld v = cld(cosl(a), sinl(a)) * c[k];
            wc[k] = make_double2((double)v.real(), (double)v.imag());
        }
        if ((rc = upload(wc, &p.thwc, p.bytes, err))) return rc;
        p.thsc = (double)(1.0L / (2.0L * PI_L * (ld)N1));
    }

    // chain segmentation (segment_chains), the checkpoints at the boundaries
    // (O(L^2) each, by the degree recursion or the row recursion in long double)
    // restarting the later segments
    {
        if (!segment_chains(L, SEG_MAX, p.segf, p.nsegf) || !segment_chains(L, SEGI_MAX, p.segi, p.nsegi)) {
            err = "segmentation exceeds the waves of a workgroup";
            return -3;
        }
        const size_t T = (size_t)L * (L + 1) / 2;
        ck_grid(L, p.segf, p.ckfg, p.nckf);
        if (p.nckf > 1) {
            std::vector<double2> ck((size_t)(p.nckf - 1) * T, make_double2(0.0, 0.0));
            std::vector<int2> ckk((size_t)(p.nckf - 1) * T, make_int2(0, 0));
            std::vector<ld> c0, c1;
            for (int j = 1; j < p.nckf; ++j) {
                const int nc = j * p.ckfg;
                for (int m = 0; m < L; ++m) {
                    degree_chain(E, L, m, nc - 1, c0);
                    degree_chain(E, L, m, nc, c1);
                    for (int l = std::max(m, nc - 1); l < L; ++l) {
                        double x0, x1;
                        int k0, k1;
                        split_signed(c0[l], x0, k0);
                        split_signed(c1[l], x1, k1);
                        const size_t i = (size_t)(j - 1) * T + tri_m(m, l, L);
                        ck[i] = make_double2(x0, x1);
                        ckk[i] = make_int2(k0, k1);
                    }
                }
            }
            if ((rc = upload(ck, &p.ckf, p.bytes, err))) return rc;
            if ((rc = upload(ckk, &p.ckfk, p.bytes, err))) return rc;
        }
        ck_grid(L, p.segi, p.ckg, p.nck);
        if (p.nck > 1) {
            size_t tot = 0;
            for (int j = 1; j < p.nck; ++j) {
                const int c = j * p.ckg;
                p.cki_off[j] = tot;
                tot += (size_t)(c + 1) * (c + 1);
            }
            std::vector<double2> ck(tot, make_double2(0.0, 0.0));
            std::vector<int2> ckk(tot, make_int2(0, 0));
            std::vector<ld> r0, r1;
            for (int j = 1; j < p.nck; ++j) {
                const int c = j * p.ckg;
                for (int m = 0; m <= c; ++m) {
                    row_chain(E, c, m, r1);                    // Delta^c_{m,n}
                    if (m <= c - 1) row_chain(E, c - 1, m, r0);  // Delta^{c-1}_{m,n}
                    for (int n = 0; n <= c; ++n) {
                        // Delta_{n,m} = (-1)^{n-m} Delta_{m,n}
                        const ld sg = ((n - m) & 1) ? -1.0L : 1.0L;
                        const ld v1 = sg * r1[n];
                        const ld v0 = (m <= c - 1 && n <= c - 1) ? sg * r0[n] : 0.0L;
                        double x0, x1;
                        int k0, k1;
                        split_signed(v0, x0, k0);
                        split_signed(v1, x1, k1);
                        ck[p.cki_off[j] + (size_t)m * (c + 1) + n] = make_double2(x0, x1);
                        ckk[p.cki_off[j] + (size_t)m * (c + 1) + n] = make_int2(k0, k1);
                    }
                }
            }
            if ((rc = upload(ck, &p.cki, p.bytes, err))) return rc;
            if ((rc = upload(ckk, &p.ckik, p.bytes, err))) return rc;
        }
    }

    // Work list of the forward contractions (FP64 and mixed): packed segments,
    // see forward_work.
    {
        const std::vector<int4> wf4 = forward_work(p);
        p.nworkf4 = (int)(wf4.size() / SEG_MAX);
        if ((rc = upload(wf4, &p.workf4, p.bytes, err))) return rc;
    }
    return 0;
}

void free_plan(Plan& p)
{
    void* ptrs[] = {p.rtab, p.edge, p.edgek, p.lco, p.cl, p.tw, p.chirp, p.bhat, p.what, p.whatc, p.whate, p.thtw, p.thwc,
                    p.workf4, p.ckf, p.ckfk, p.cki, p.ckik};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    p = Plan();
}

// Packing of the segments of chain groups into workgroups of `slots` wave slots
// (layout of the resulting work list in mw_internal.h).  items[x] are the
// groups dealt to XCD x, (a, b) = (first lane index, first order), with their
// segment count, the length that orders them (the longest segment for the
// forward, the whole chain for the inverse) and each segment's descriptor word.
// Groups of one segment go four to a workgroup with no barrier (every wave
// exits when done); groups of several segments are placed first-fit into the
// last few open workgroups, so that waves meeting at the reduction barrier
// have similar lengths.  Workgroups are dealt round-robin over the 8 XCDs
// (workgroup k*8 + x is the k-th of XCD x); per XCD they are ordered as in
// balance_cus when at most `resident` per compute unit are needed (the launch
// fits at once, or nearly), else longest first, which is what dynamic dispatch
// wants.
// work: the group's steps summed over its segments, plus a start-up cost per
// segment.
// dw: the descriptor's last word for each segment (see the work-list layouts).
constexpr int SEG_CAP = SEGT_MAX > SEGI_MAX ? (SEGT_MAX > SEG_MAX ? SEGT_MAX : SEG_MAX) : (SEGI_MAX > SEG_MAX ? SEGI_MAX : SEG_MAX);
struct SegItem { int a, b, nseg, len, work; int dw[SEG_CAP]; };

// Workgroups per compute unit up to which a work list is laid out for the
// round-robin placement (balance_cus) rather than longest first.  The FP64
// inverse holds four to seven waves per SIMD (complex or real map, plain or
// exponent-extended), the forward four or five, the mixed kernels two to four;
// lists a little longer than what fits at once still gain from the balanced
// layout (their last workgroups start as others finish), measured at L = 512
// with 203 inverse and 137 forward workgroups per XCD.
constexpr int RESIDENT_INV = 7;
constexpr int RESIDENT_TRI = 7;
constexpr int RESIDENT_FWD = 5;

// Order of the workgroups of one XCD when all of them are resident at once:
// the dispatcher then fills the 32 compute units of an XCD round-robin, so its
// k-th and (k+32)-th workgroups share a compute unit.  The workgroups are
// assigned, heaviest first, to the least-loaded of the 32 position classes
// k mod 32 (each taking as many as it has positions) and laid out class by
// class.  Plain longest-first order would give the unit at position 0 the
// heaviest workgroup of every block of 32.
template <class G>
static void balance_cus(std::vector<G>& gs)
{
    constexpr int C = 32;
    const int n = (int)gs.size();
    std::stable_sort(gs.begin(), gs.end(), [](const G& u, const G& v) { return u.work > v.work; });
    std::vector<std::vector<int>> bin(C);
    std::vector<long> load(C, 0);
    for (int i = 0; i < n; ++i) {
        int best = -1;
        for (int c = 0; c < C; ++c) {
            const int cap = n / C + (c < n % C ? 1 : 0);
            if ((int)bin[c].size() < cap && (best < 0 || load[c] < load[best])) best = c;
        }
        bin[best].push_back(i);
        load[best] += gs[i].work;
    }
    std::vector<G> out;
    out.reserve(n);
    for (int k = 0; k < n; ++k) out.push_back(gs[bin[k % C][k / C]]);
    gs.swap(out);
}

static std::vector<int4> pack_segments(std::vector<std::vector<SegItem>>& items, int slots, int resident)
{
    struct Group { int used, len; long work; bool bar; int4 slot[SEG_CAP]; };
    std::vector<std::vector<Group>> per(items.size());
    for (size_t x = 0; x < items.size(); ++x) {
        std::vector<SegItem>& it = items[x];
        std::stable_sort(it.begin(), it.end(), [](const SegItem& u, const SegItem& v) { return u.len > v.len; });
        std::vector<Group>& gs = per[x];
        std::vector<int> open;   // groups with free slots, oldest first
        constexpr int WINDOW = 4;
        for (const SegItem& t : it) {
            const bool bar = t.nseg > 1;
            int g = -1;
            for (int k = (int)open.size() - 1; k >= 0 && g < 0; --k) {
                const Group& c = gs[open[k]];
                if (c.bar == bar && slots - c.used >= t.nseg) g = open[k];
            }
            if (g < 0) {
                Group c;
                c.used = 0;
                c.len = t.len;
                c.work = 0;
                c.bar = bar;
                for (int i = 0; i < slots; ++i) c.slot[i] = make_int4(-1, 0, bar ? 1 << 24 : 0, 0);
                gs.push_back(c);
                g = (int)gs.size() - 1;
                open.push_back(g);
                if ((int)open.size() > WINDOW) open.erase(open.begin());
            }
            Group& c = gs[g];
            for (int w = 0; w < t.nseg; ++w)
                c.slot[c.used + w] =
                    make_int4(t.a, t.b, w | (t.nseg << 8) | (c.used << 16) | (bar ? 1 << 24 : 0), t.dw[w]);
            c.used += t.nseg;
            c.work += t.work;
            if (c.used == slots)
                for (size_t k = 0; k < open.size(); ++k)
                    if (open[k] == g) { open.erase(open.begin() + k); break; }
        }
    }
    size_t n = 0;   // workgroups of the busiest XCD
    for (auto& v : per) n = std::max(n, v.size());
    for (auto& gs : per) {
        if (n <= (size_t)32 * resident) balance_cus(gs);
        else std::stable_sort(gs.begin(), gs.end(), [](const Group& u, const Group& v) { return u.len > v.len; });
    }
    std::vector<int4> out;
    out.reserve(n * per.size() * slots);
    for (size_t g = 0; g < n; ++g)
        for (auto& v : per)
            for (int i = 0; i < slots; ++i) out.push_back(g < v.size() ? v[g].slot[i] : make_int4(-1, 0, 0, 0));
    return out;
}

// Segments of a chain over the steps [l0, end) whose first segment must reach
// lmin (every chain start lies before it): at most smax segments with
// boundaries among the ascending candidates cand, the longest as short as
// possible.  bnd[0] = l0, bnd[nseg] = end; returns nseg.
static int split_chain(int l0, int end, int lmin, const std::vector<int>& cand, int smax, int* bnd)
{
    // fewest segments no longer than T, boundaries as far out as allowed
    auto greedy = [&](int T, int* b) {
        int k = 0;
        b[0] = l0;
        while (end - b[k] > T) {
            int c = -1;
            for (const int cj : cand)
                if (cj > b[k] && cj <= b[k] + T && (k > 0 || cj >= lmin)) c = cj;
            if (c < 0 || k + 1 >= smax) return -1;
            b[++k] = c;
        }
        b[k + 1] = end;
        return k + 1;
    };
    int lo = 1, hi = end - l0;   // hi is always feasible (one segment)
    while (lo < hi) {
        const int mid = (lo + hi) / 2;
        int b[(SEG_CAP) + 1];
        if (greedy(mid, b) > 0) hi = mid;
        else lo = mid + 1;
    }
    return greedy(hi, bnd);
}

// FP64 inverse contraction: group (n0, m0) starts its pairs at lstart =
// max(n0, m0) rounded down to even; every chain start (n, m or |s|) lies below
// lA, so its first segment runs to a boundary >= max(lA, lstart+2); the
// boundaries (split_chain) make the group's longest segment as short as the
// planes allow.  Descriptor word: segment start | end << 16 (degrees).  Dealt
// to XCDs by order pair.
static std::vector<int4> inverse_work(const Plan& p, int as)
{
    const int L = p.L, Lp = p.Lp;
    std::vector<int> cand;   // the checkpoint planes
    for (int k = 1; k < p.nck; ++k) cand.push_back(k * p.ckg);
    std::vector<std::vector<SegItem>> items(8);
    for (int n0 = 0; n0 < L; n0 += 64)
        for (int m0 = 0; m0 < L; m0 += 2) {
            const int lstart = std::max(n0, m0) & ~1;
            const int lA = std::max(std::max(n0 + 64, m0 + 2), as + 1);
            int bnd[SEGI_MAX + 1];
            const int nseg = split_chain(lstart, Lp, std::max(lA, lstart + 2), cand, SEGI_MAX, bnd);
            SegItem t{n0, m0, nseg, Lp - lstart, Lp - lstart + 16 * nseg, {}};
            for (int w = 0; w < nseg; ++w) t.dw[w] = bnd[w] | (bnd[w + 1] << 16);
            items[(m0 / 2) & 7].push_back(t);
        }
    return pack_segments(items, SEGI_MAX, RESIDENT_INV);
}

// The same groups restricted to those that meet n >= m (m0 <= n0 + 63), for the
// FP64 inverse that runs each chain with n >= m once for (m, n) and (n, m).
// Dealt to XCDs by chunks of four order pairs, back and forth: the uniform rows
// of an order stay in one L2, a 128-byte line of F holds eight orders of one
// row in the transposed outputs, and the alternating direction evens out the
// work, which falls with m0.  (Contiguous runs of (n0, m0) per XCD, which keep
// each lane's coefficient rows in one L2 instead, were slower: the uniform
// rows of every order then meet in every L2.)
static std::vector<int4> inverse_work_tri(const Plan& p, int as)
{
    const int L = p.L, Lp = p.Lp;
    std::vector<int> cand;   // the checkpoint planes
    for (int k = 1; k < p.nck; ++k) cand.push_back(k * p.ckg);
    std::vector<std::vector<SegItem>> items(8);
    for (int n0 = 0; n0 < L; n0 += 64)
        for (int m0 = 0; m0 < L && m0 <= n0 + 63; m0 += 2) {
            const int lstart = std::max(n0, m0) & ~1;
            const int lA = std::max(std::max(n0 + 64, m0 + 2), as + 1);
            int bnd[SEGT_MAX + 1];
            const int nseg = split_chain(lstart, Lp, std::max(lA, lstart + 2), cand, SEGT_MAX, bnd);
            SegItem t{n0, m0, nseg, Lp - lstart, Lp - lstart + 16 * nseg, {}};
            for (int w = 0; w < nseg; ++w) t.dw[w] = bnd[w] | (bnd[w + 1] << 16);
            const int chunk = m0 >> 3, pos = chunk & 7;
            items[((chunk >> 3) & 1) ? 7 - pos : pos].push_back(t);
        }
    return pack_segments(items, SEGT_MAX, RESIDENT_TRI);
}

// FP64 forward contraction: group (l0, mb) runs the row recursions from nmax =
// min(l0+63, L-1) down to 0 in at most SEG_MAX segments: segment w covers the
// rows [lo, hi) (w = 0 the lowest); the top one (w = nseg-1) runs from nmax and
// starts the lanes, so it reaches down to l0 at least, and each lower one
// starts from the checkpoint plane at row hi.  The boundaries make the group's
// longest segment as short as the planes allow (split_chain on the rows counted
// from the top).  Descriptor word: lo | hi << 16.  Dealt to XCDs by chunks of
// eight orders (for L >= 256), so that the waves writing the f_lm of one line
// (orders m..m+7 at one degree) meet in one L2.
static std::vector<int4> forward_work(const Plan& p)
{
    const int L = p.L;
    std::vector<std::vector<SegItem>> items(8);
    for (int l0 = 0; l0 < L; l0 += 64) {
        const int nmax = std::min(l0 + 63, L - 1), R = nmax + 1;
        // rows counted from the top: r = R - n; planes at rows k*ckfg <= nmax
        std::vector<int> cand;
        for (int k = p.nckf - 1; k >= 1; --k)
            if (k * p.ckfg <= nmax) cand.push_back(R - k * p.ckfg);
        int bnd[SEG_MAX + 1];
        const int nseg = split_chain(0, R, R - l0, cand, SEG_MAX, bnd);
        int len = 0;
        for (int k = 0; k < nseg; ++k) len = std::max(len, bnd[k + 1] - bnd[k]);
        for (int mb = 0; mb <= nmax; mb += MT_FWD) {
            // orders in chunks of 8 (one 128-byte line of f_lm per degree), dealt
            // to the XCDs back and forth so every XCD gets low and high orders;
            // below L = 256 (fewer than four rounds of chunks) the XCDs would get
            // unequal shares, and order pairs are dealt round-robin instead
            const int chunk = mb >> 3, pos = chunk & 7;
            const int x = (L < 256) ? (mb / MT_FWD) & 7 : (((chunk >> 3) & 1) ? 7 - pos : pos);
            SegItem t{l0, mb, nseg, len, nmax + 1 + 16 * nseg, {}};
            for (int w = 0; w < nseg; ++w) {   // w = 0 lowest: top-down segment k = nseg-1-w
                const int k = nseg - 1 - w;
                t.dw[w] = (R - bnd[k + 1]) | ((R - bnd[k]) << 16);
            }
            items[x].push_back(t);
        }
    }
    return pack_segments(items, SEG_MAX, RESIDENT_FWD);
}

// Delta^l_{n,|s|} for n <= l < L by the upward l-recursion in long double,
// started at l0 = max(n, |s|) from the edge value.
int build_spin_table(const Plan& p, int as, SpinTable& t, std::string& err)
{
    const int L = p.L;
    t = SpinTable();
    t.L = L;
    t.as = as;
    std::vector<ld> E = edge_values(L);
    auto edge = [&](int l, int m) { return E[(size_t)l * (l + 1) / 2 + m]; };
    std::vector<double> val((size_t)L * L, 0.0);
    std::vector<int> kk((size_t)L * L, 0);
    // (Pu'_m(l), c_l Delta^l_{m,|s|} / h_m(l)) for the FP64 inverse's transposed sums
    std::vector<double2> lcos = lrec_factors(L, p.Lp);
    for (double2& v : lcos) v.y = 0.0;
    const std::vector<double2> hs = lrec_factors(L, p.Lp);
    // the scaled spin values h_|s|(l) Delta^l_{n,|s|} (zero below 2^-900 and in
    // the pad row l = L of an odd L), the FP64 inverses' spin rows
    std::vector<double> sval((size_t)p.Lp * L, 0.0);
    // the forward's spin values Delta^l_{|s|,n} = (-1)^{n+|s|} Delta^l_{n,|s|},
    // transposed (64 consecutive l of one row n are one read)
    std::vector<double> svalf((size_t)p.Lp * L, 0.0);
    for (int n = 0; n < L; ++n) {
        int l0 = std::max(n, as);
        if (l0 >= L) continue;
        ld dcur = (n >= as) ? (((n - as) % 2) ? -edge(n, as) : edge(n, as)) : edge(as, n);
        ld dprev = 0.0L;
        for (int l = l0; l < L; ++l) {
            double x;
            int k;
            ld a = fabsl(dcur);
            split_ext(a, x, k);
            val[(size_t)l * L + n] = (dcur < 0) ? -x : x;
            kk[(size_t)l * L + n] = k;
            if (a > 0x1p-900L) {
                sval[(size_t)l * L + n] = (double)(dcur * (ld)hs[(size_t)as * p.Lp + l].y);
                svalf[(size_t)n * L + l] = (double)(((n + as) & 1) ? -dcur : dcur);
            }
            if (a > 0x1p-900L)
                lcos[(size_t)n * p.Lp + l].y =
                    (double)(sqrtl((2.0L * l + 1.0L) / (4.0L * PI_L)) * dcur / (ld)hs[(size_t)n * p.Lp + l].y);
            if (l + 1 >= L) break;
            ld dnext;
            if (l == 0) {
                dnext = 0.0L;
            } else {
                ld num = -(2.0L * l + 1.0L) * (ld)as * (ld)n * dcur -
                         (ld)(l + 1) * sqrtl(((ld)l * l - (ld)as * as) * ((ld)l * l - (ld)n * n)) * dprev;
                ld den = (ld)l * sqrtl(((ld)(l + 1) * (l + 1) - (ld)as * as) * ((ld)(l + 1) * (l + 1) - (ld)n * n));
                dnext = num / den;
            }
            dprev = dcur;
            dcur = dnext;
        }
    }
    int rc;
    if ((rc = upload(val, &t.val, t.bytes, err))) return rc;
    if ((rc = upload(kk, &t.k, t.bytes, err))) return rc;
    const std::vector<int4> w = inverse_work(p, as);
    t.nwinv = (int)(w.size() / SEGI_MAX);
    if ((rc = upload(w, &t.winv, t.bytes, err))) return rc;
    if ((rc = upload(lcos, &t.lcos, t.bytes, err))) return rc;
    if ((rc = upload(sval, &t.sval, t.bytes, err))) return rc;
    if ((rc = upload(svalf, &t.svalf, t.bytes, err))) return rc;
    const std::vector<int4> wt = inverse_work_tri(p, as);
    t.nwtri = (int)(wt.size() / SEGT_MAX);
    if ((rc = upload(wt, &t.wtri, t.bytes, err))) return rc;
    return 0;
}

void free_spin_table(SpinTable& t)
{
    if (t.val) (void)hipFree(t.val);
    if (t.k) (void)hipFree(t.k);
    if (t.winv) (void)hipFree(t.winv);
    if (t.lcos) (void)hipFree(t.lcos);
    if (t.sval) (void)hipFree(t.sval);
    if (t.svalf) (void)hipFree(t.svalf);
    if (t.wtri) (void)hipFree(t.wtri);
    t = SpinTable();
}

}  // namespace mw
