// Host-only checks of the contraction work lists that the plan builder packs
// (inverse_work, inverse_work_tri, forward_work in mw_plan.cpp): every segment of every chain
// group appears exactly once, the segments of a group sit in consecutive slots
// of one workgroup with a consistent lead slot, barrier flags match the groups
// a workgroup holds, restart boundaries lie where checkpoints exist, and a list
// that fits the GPU at once spreads its steps evenly over the compute units.
// Built and run by tests/test_host_plan.py; prints one line per failure.
#include "../../paper_1110_6298_amd/csrc/mw_plan.cpp"

#include <cstdio>
#include <map>
#include <tuple>

using namespace mw;

static long bad = 0;
#define CHECK(c, ...)                        \
    do {                                     \
        if (!(c)) {                          \
            ++bad;                           \
            if (bad < 20) printf(__VA_ARGS__); \
        }                                    \
    } while (0)

// Steps of each slot and the per-CU totals when workgroup k*8 + x runs on CU
// (x, k mod 32) of XCD x: the spread must stay within one workgroup's steps of
// the mean whenever the list fits at once.
static void check_balance(const char* tag, int L, const std::vector<int4>& w, int slots, int resident,
                          const std::vector<long>& steps)
{
    const size_t nwg = w.size() / slots;
    if ((nwg + 7) / 8 > (size_t)32 * resident) return;
    std::vector<long> cu(256, 0);
    long heaviest = 0, total = 0;
    for (size_t g = 0; g < nwg; ++g) {
        long wg = 0;
        for (int i = 0; i < slots; ++i) wg += steps[g * slots + i];
        cu[(g % 8) * 32 + (g / 8) % 32] += wg;
        heaviest = std::max(heaviest, wg);
        total += wg;
    }
    long mx = 0;
    for (long c : cu) mx = std::max(mx, c);
    CHECK(mx <= total / 256 + heaviest, "%s L=%d: busiest CU %ld steps, mean %ld, heaviest workgroup %ld\n", tag, L,
          mx, total / 256, heaviest);
}

// tri: the list of the FP64 inverse over the triangle n >= m (inverse_work_tri,
// SEGT_MAX slots, only the groups with m0 <= n0 + 63).
static void check_inverse(int L, int as, bool tri)
{
    Plan p;
    p.L = L;
    p.Lp = L + (L & 1);
    CHECK(segment_chains(L, SEGI_MAX, p.segi, p.nsegi), "inverse L=%d: segmentation\n", L);
    ck_grid(L, p.segi, p.ckg, p.nck);
    CHECK(p.nck <= CKI_MAX && p.ckg % 2 == 0, "inverse L=%d: plane grid\n", L);
    auto plane = [&](int c) { return c > 0 && c < L && c % p.ckg == 0 && c / p.ckg < p.nck; };
    const int S = tri ? SEGT_MAX : SEGI_MAX;
    const std::vector<int4> w = tri ? inverse_work_tri(p, as) : inverse_work(p, as);
    CHECK(w.size() % S == 0, "inverse L=%d: size\n", L);
    std::map<std::tuple<int, int, int>, int> seen;
    std::vector<long> steps(w.size(), 0);
    for (size_t g = 0; g < w.size() / S; ++g) {
        const int4* s = &w[g * S];
        const int bar = (s[0].z >> 24) & 1;
        int anymulti = 0, items = 0;
        for (int i = 0; i < S; ++i) {
            CHECK(((s[i].z >> 24) & 1) == bar, "inverse L=%d s=%d: barrier flag differs within workgroup %zu\n", L,
                  as, g);
            if (s[i].x < 0) continue;
            ++items;
            const int n0 = s[i].x, m0 = s[i].y, seg = s[i].z & 0xff, nseg = (s[i].z >> 8) & 0xff;
            const int lead = (s[i].z >> 16) & 0xff;
            const int cs = s[i].w & 0xffff, ce = (int)((unsigned)s[i].w >> 16);
            anymulti |= nseg > 1;
            CHECK(n0 % 64 == 0 && n0 < L && m0 % 2 == 0 && m0 < L, "inverse L=%d: group (%d, %d)\n", L, n0, m0);
            CHECK(!tri || m0 <= n0 + 63, "inverse L=%d: group (%d, %d) above the triangle\n", L, n0, m0);
            CHECK(lead + seg == i && lead + nseg <= S, "inverse L=%d: slot layout\n", L);
            for (int k = 0; k < nseg && lead + k < S; ++k) {
                const int4 o = s[lead + k];
                CHECK(o.x == n0 && o.y == m0 && (o.z & 0xff) == k && ((o.z >> 8) & 0xff) == nseg,
                      "inverse L=%d: sibling segment\n", L);
                // consecutive segments of the group meet at their common boundary
                if (k + 1 < nseg && lead + k + 1 < S)
                    CHECK(((unsigned)o.w >> 16) == (unsigned)(s[lead + k + 1].w & 0xffff),
                          "inverse L=%d: segments not contiguous\n", L);
            }
            // every chain start (n, m or |s|) lies below lA: the first segment starts at
            // lstart and reaches past lA; later ones restart at checkpoint planes; the
            // last one ends with the degrees
            const int lstart = std::max(n0, m0) & ~1;
            const int lA = std::max(std::max(n0 + 64, m0 + 2), as + 1);
            if (seg == 0) CHECK(cs == lstart, "inverse L=%d: first segment start\n", L);
            if (seg == 0 && nseg > 1)
                CHECK(ce >= std::max(lA, lstart + 2) && plane(ce), "inverse L=%d s=%d: first boundary %d\n", L, as, ce);
            if (seg >= 1) CHECK(plane(cs) && cs >= lA, "inverse L=%d s=%d: restart degree %d\n", L, as, cs);
            if (seg == nseg - 1) CHECK(ce == p.Lp, "inverse L=%d: last segment end\n", L);
            CHECK(ce > cs && cs % 2 == 0 && ce % 2 == 0, "inverse L=%d: segment [%d, %d)\n", L, cs, ce);
            CHECK(nseg >= 1 && nseg <= S, "inverse L=%d: segment count\n", L);
            steps[g * S + i] = ce - cs;
            CHECK(seen[std::make_tuple(n0, m0, seg)]++ == 0, "inverse L=%d: duplicate segment\n", L);
        }
        CHECK(!items || bar == anymulti, "inverse L=%d: barrier flag of workgroup %zu\n", L, g);
    }
    // the chains of every group are covered from lstart to the last degree
    for (int n0 = 0; n0 < L; n0 += 64)
        for (int m0 = 0; m0 < L && (!tri || m0 <= n0 + 63); m0 += 2) {
            int nseg = -1;
            for (int k = 0; k < S; ++k)
                if (seen.count(std::make_tuple(n0, m0, k))) nseg = k + 1;
            CHECK(nseg >= 1, "inverse L=%d s=%d: group (%d, %d) missing\n", L, as, n0, m0);
            for (int k = 0; k < nseg; ++k)
                CHECK(seen.count(std::make_tuple(n0, m0, k)) == 1, "inverse L=%d: segment gap\n", L);
        }
    check_balance(tri ? "inverse (triangle)" : "inverse", L, w, S, tri ? RESIDENT_TRI : RESIDENT_INV, steps);
}

static void check_forward(int L)
{
    Plan p;
    p.L = L;
    p.Lp = L + (L & 1);
    CHECK(segment_chains(L, SEG_MAX, p.segf, p.nsegf), "forward L=%d: segmentation\n", L);
    ck_grid(L, p.segf, p.ckfg, p.nckf);
    CHECK(p.nckf <= CKI_MAX && p.ckfg % 2 == 0, "forward L=%d: plane grid\n", L);
    auto plane = [&](int c) { return c > 0 && c < L && c % p.ckfg == 0 && c / p.ckfg < p.nckf; };
    const std::vector<int4> w = forward_work(p);
    CHECK(w.size() % SEG_MAX == 0, "forward L=%d: size\n", L);
    std::map<std::tuple<int, int, int>, int> seen;
    std::vector<long> steps(w.size(), 0);
    for (size_t g = 0; g < w.size() / SEG_MAX; ++g) {
        const int4* s = &w[g * SEG_MAX];
        const int bar = (s[0].z >> 24) & 1;
        int anymulti = 0, items = 0;
        for (int i = 0; i < SEG_MAX; ++i) {
            CHECK(((s[i].z >> 24) & 1) == bar, "forward L=%d: barrier flag differs\n", L);
            if (s[i].x < 0) continue;
            ++items;
            const int l0 = s[i].x, mb = s[i].y, seg = s[i].z & 0xff, nseg = (s[i].z >> 8) & 0xff;
            const int lead = (s[i].z >> 16) & 0xff;
            const int lo = s[i].w & 0xffff, hi = (int)((unsigned)s[i].w >> 16);
            const int nmax = std::min(l0 + 63, L - 1);
            anymulti |= nseg > 1;
            CHECK(l0 % 64 == 0 && mb % MT_FWD == 0 && mb <= nmax, "forward L=%d: group (%d, %d)\n", L, l0, mb);
            CHECK(nseg >= 1 && nseg <= SEG_MAX && seg < nseg, "forward L=%d: segment count\n", L);
            CHECK(lead + seg == i && lead + nseg <= SEG_MAX, "forward L=%d: slot layout\n", L);
            for (int k = 0; k < nseg && lead + k < SEG_MAX; ++k) {
                const int4 o = s[lead + k];
                CHECK(o.x == l0 && o.y == mb && (o.z & 0xff) == k, "forward L=%d: sibling segment\n", L);
                // segment k ends where segment k+1 starts
                if (k + 1 < nseg && lead + k + 1 < SEG_MAX)
                    CHECK(((unsigned)o.w >> 16) == (unsigned)(s[lead + k + 1].w & 0xffff),
                          "forward L=%d: segments not contiguous\n", L);
            }
            // the lowest segment ends at row 0, the top one starts at nmax and reaches
            // down past every lane start (l0); lower ones restart at checkpoint planes
            if (seg == 0) CHECK(lo == 0, "forward L=%d: lowest segment\n", L);
            if (seg == nseg - 1) CHECK(hi == nmax + 1 && lo <= l0, "forward L=%d: top segment [%d, %d)\n", L, lo, hi);
            else CHECK(plane(hi) && hi <= l0, "forward L=%d: restart row %d\n", L, hi);
            CHECK(hi > lo && lo % 2 == 0, "forward L=%d: segment [%d, %d)\n", L, lo, hi);
            steps[g * SEG_MAX + i] = hi - lo;
            CHECK(seen[std::make_tuple(l0, mb, seg)]++ == 0, "forward L=%d: duplicate segment\n", L);
        }
        CHECK(!items || bar == anymulti, "forward L=%d: barrier flag of workgroup %zu\n", L, g);
    }
    for (int l0 = 0; l0 < L; l0 += 64) {
        const int nmax = std::min(l0 + 63, L - 1);
        for (int mb = 0; mb <= nmax; mb += MT_FWD) {
            int nseg = 0;
            while (nseg < SEG_MAX && seen.count(std::make_tuple(l0, mb, nseg))) ++nseg;
            CHECK(nseg >= 1, "forward L=%d: group (%d, %d) missing\n", L, l0, mb);
            for (int k = nseg; k < SEG_MAX; ++k)
                CHECK(seen.count(std::make_tuple(l0, mb, k)) == 0, "forward L=%d: segment gap\n", L);
        }
    }
    check_balance("forward", L, w, SEG_MAX, RESIDENT_FWD, steps);
}

int main()
{
    std::vector<int> Ls;
    for (int L = 1; L <= 260; ++L) Ls.push_back(L);
    for (int L : {300, 383, 384, 511, 512, 513, 640, 901, 1000, 1024, 1500, 2047, 2048, 2049, 3001, 4095, 4096})
        Ls.push_back(L);
    long cases = 0;
    for (int L : Ls) {
        check_forward(L);
        ++cases;
        for (int as : {0, 1, 2, 3, 7, 63, 64, 65, 100, 200, L - 1}) {
            if (as < 0 || as >= L) continue;
            check_inverse(L, as, false);
            check_inverse(L, as, true);
            cases += 2;
        }
    }
    printf("%ld work lists checked, %ld problems\n", cases, bad);
    return bad != 0;
}
