// C ABI of libmw: argument validation, per-device plan/workspace cache and the
// launch sequence of each transform.  See include/mw.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <mutex>
#include <tuple>
#include <string>
#include <utility>
#include <vector>

#include "../../include/mw.h"
#include "../../include/mw_profile.h"
#include "mw_internal.h"

namespace {

using mw::Plan;
using mw::SpinTable;

thread_local std::string g_last_error;

// Workspace of mw_forward_noalloc: a file-scope device array, so that the entry
// point needs no allocation.  Each device holds its own copy (at its own
// address) from the library's load until the process ends.  In host code the
// name is only a stand-in for the symbol: the device address comes from
// hipGetSymbolAddress, once per device (DeviceState::scratch).
constexpr size_t NOALLOC_BYTES = MW_NOALLOC_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

struct DeviceState {
    std::map<int, Plan> plans;                    // by L
    std::map<std::pair<int, int>, SpinTable> spins;  // by (L, |s|)
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // Outgrown workspaces stay allocated until mw_release: a graph captured
    // earlier may still reference one.
    std::vector<void*> retired;
    // Two internal streams (default priority) on which the chunks of a call
    // alternate, each with its half of the workspace, so that one chunk's
    // Fourier stages (LDS-bound) overlap another's contractions (VALU-bound);
    // fork and join events tie them to the caller's stream.
    hipStream_t lane[2] = {nullptr, nullptr};
    hipEvent_t fork = nullptr, join[2] = {nullptr, nullptr};
    // Caller-owned workspaces bound to streams (mw_set_workspace): calls on such
    // a stream use the caller's buffer and never the library's.
    std::map<hipStream_t, std::pair<void*, size_t>> user_ws;
    // Device address of this device's copy of `scratch` (set on the first
    // mw_forward_noalloc call on the device).
    void* scratch = nullptr;
};

// Create the two chunk streams and their events on the current device.
bool make_lanes(DeviceState& d)
{
    if (d.lane[0]) return true;
    for (int k = 0; k < 2; ++k) {
        if (hipStreamCreateWithFlags(&d.lane[k], hipStreamNonBlocking) != hipSuccess) return false;
        if (hipEventCreateWithFlags(&d.join[k], hipEventDisableTiming) != hipSuccess) return false;
    }
    return hipEventCreateWithFlags(&d.fork, hipEventDisableTiming) == hipSuccess;
}

std::mutex g_mu;
std::map<int, DeviceState> g_dev;

// ---- opt-in per-stage event timing --------------------------------------
struct ProfRec { int stage; hipEvent_t a, b; };
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event()
{
    if (!g_event_pool.empty()) { hipEvent_t e = g_event_pool.back(); g_event_pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// Runs one launcher, bracketed by events when profiling is on.
template <class F>
hipError_t staged(int stage, hipStream_t st, bool prof, F&& launch)
{
    if (!g_prof_on || !prof) return launch();
    ProfRec r{stage, take_event(), take_event()};
    (void)hipEventRecord(r.a, st);
    hipError_t e = launch();
    (void)hipEventRecord(r.b, st);
    g_prof.push_back(r);
    return e;
}

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int validate(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
             void* const* ptrs, int32_t precision, bool need_ptrs)
{
    if (batch < 1) return fail(MW_EINVAL, "batch must be >= 1 (got %d)", batch);
    if (!L || !spin || !reality) return fail(MW_EINVAL, "L, spin and reality arrays must be non-NULL");
    if (precision != MW_FP64 && precision != MW_FP32C) return fail(MW_EINVAL, "unknown precision %d", precision);
    if (need_ptrs && !ptrs) return fail(MW_EINVAL, "ptrs must be non-NULL");
    for (int b = 0; b < batch; ++b) {
        if (L[b] < 1 || L[b] > MW_LMAX) return fail(MW_EINVAL, "map %d: L = %d outside [1, %d]", b, L[b], MW_LMAX);
        if (spin[b] <= -L[b] || spin[b] >= L[b])
            return fail(MW_EINVAL, "map %d: |spin| = %d must be < L = %d", b, spin[b], L[b]);
        if (reality[b] != 0 && reality[b] != 1) return fail(MW_EINVAL, "map %d: reality must be 0 or 1", b);
        if (reality[b] == 1 && spin[b] != 0) return fail(MW_EINVAL, "map %d: reality = 1 needs spin = 0", b);
        if (need_ptrs && (!ptrs[2 * b] || !ptrs[2 * b + 1])) return fail(MW_EINVAL, "map %d: NULL pointer", b);
    }
    return MW_OK;
}

// Three regions: W0 = N1 x L complex (G, or the inverse's F); W1 = max(N1 x L
// complex, forward Hp records of L x Lp x 4 doubles); W2 = the inverse's
// coefficient stream (L x Lp x 4 doubles).  Each starts 256-byte aligned.
size_t ws_region(int L, int which)
{
    const size_t n1 = 2 * (size_t)L - 1;
    const size_t lp = (size_t)L + (L & 1);
    const size_t a = n1 * (size_t)L * sizeof(double2);
    const size_t rec = (size_t)L * lp * 4 * sizeof(double);
    const size_t r = which == 0 ? a : which == 1 ? std::max(a, rec) : rec;
    return (r + 255) & ~(size_t)255;
}

size_t ws_need(int L) { return ws_region(L, 0) + ws_region(L, 1) + ws_region(L, 2) + 256; }

bool capturing(hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) return false;
    return cs != hipStreamCaptureStatusNone;
}

// Plan of band-limit L on this device (built on first use, outside capture).
int get_plan(DeviceState& d, int L, bool may_alloc, const Plan** plan)
{
    std::string err;
    auto it = d.plans.find(L);
    if (it == d.plans.end()) {
        if (!may_alloc) return fail(MW_ENOMEM, "plan for L=%d not prepared (call mw_prepare before capture)", L);
        Plan p;
        int rc = mw::build_plan(L, p, err);
        if (rc) { mw::free_plan(p); return fail(rc == -2 ? MW_ENOMEM : MW_EHIP, "plan L=%d: %s", L, err.c_str()); }
        it = d.plans.emplace(L, p).first;
    }
    *plan = &it->second;
    return MW_OK;
}

// Spin-row table Delta^l_{n,|s|} for l < L.
int get_spin(DeviceState& d, const Plan& p, int as, bool may_alloc, const SpinTable** spt)
{
    std::string err;
    const int L = p.L;
    auto key = std::make_pair(L, as);
    auto jt = d.spins.find(key);
    if (jt == d.spins.end()) {
        if (!may_alloc) return fail(MW_ENOMEM, "spin table L=%d |s|=%d not prepared", L, as);
        SpinTable t;
        int rc = mw::build_spin_table(p, as, t, err);
        if (rc) { mw::free_spin_table(t); return fail(rc == -2 ? MW_ENOMEM : MW_EHIP, "spin table: %s", err.c_str()); }
        jt = d.spins.emplace(key, t).first;
    }
    *spt = &jt->second;
    return MW_OK;
}

// The device's workspace, grown to ws_bytes when allowed.
int get_ws(DeviceState& d, size_t ws_bytes, bool may_alloc, void** ws)
{
    if (d.ws_bytes < ws_bytes) {
        if (!may_alloc) return fail(MW_ENOMEM, "workspace of %zu bytes not prepared", ws_bytes);
        if (d.ws) d.retired.push_back(d.ws);
        d.ws = nullptr;
        d.ws_bytes = 0;
        if (hipMalloc(&d.ws, ws_bytes) != hipSuccess) return fail(MW_ENOMEM, "workspace hipMalloc(%zu) failed", ws_bytes);
        d.ws_bytes = ws_bytes;
    }
    *ws = d.ws;
    return MW_OK;
}

enum class Op { Forward, Inverse, ForwardAdjoint, InverseAdjoint };

constexpr double TWO_PI = 6.283185307179586476925286766559;

struct Regions { double2* W0; double2* W1; double* W2; };

// Workspace slot k when the call's largest band-limit is Lws: three regions for
// a map of band-limit L, W0 (N1 x L complex), W1 (max of N1 x L complex and the
// H records), W2 (the inverse's coefficient stream), each 256-byte aligned.
Regions slot(void* ws, int Lws, int L, int k)
{
    char* base = (char*)(((uintptr_t)ws + 255) & ~(uintptr_t)255) + (size_t)k * ws_need(Lws);
    Regions r;
    r.W0 = (double2*)base;
    r.W1 = (double2*)(base + ws_region(L, 0));
    r.W2 = (double*)(base + ws_region(L, 0) + ws_region(L, 1));
    return r;
}

// Maps of one call run in chunks.  In FP64 a chunk holds maps of one band-limit,
// reality and spin (the FP64 contractions run one spin row).  In mixed precision
// a chunk holds maps of one reality, sorted by (-L, |s|, s), whose maps share
// the Wigner order chains in groups of up to G maps with at most two different
// |s| (the spin rows run beside the shared chains, Sec. V's remark on several
// spins); the maps of a band-limit with few maps in the call (`ride`) may join
// the last group of a larger band-limit, whose chains run to that band-limit
// (each map masks the degrees l >= L_b).  Every Fourier stage is one launch per
// band-limit of the chunk (blockIdx.y = map, each map with its own spin).
struct Chunk {
    int L = 0, s = 0, real = 0;   // L: the largest band-limit; s: the spin of an FP64 chunk
    std::vector<int> maps;    // batch indices
    std::vector<int> spins;   // their spins
    std::vector<int> Ls;      // their band-limits
    std::map<int, int> G;     // mixed precision: group size of the groups that start at each band-limit
    std::set<int> ride;       // band-limits whose maps may join a group that starts at a larger one
};

// End of the mixed group that starts at map i of a sequence of n maps sorted by
// (-L, |s|): up to G[L_i] maps, each of band-limit L_i or in `ride`, with at
// most two different |s|.  Lof(k), asof(k): band-limit and |s| of map k.
template <class LF, class AF>
size_t group_end(size_t n, size_t i, LF Lof, AF asof, const std::map<int, int>& G, const std::set<int>& ride)
{
    const int L0 = Lof(i), Gl = G.at(L0);
    int rows[mw::NSMAX] = {-1, -1}, nr = 0;
    size_t j = i;
    while (j < n && (int)(j - i) < Gl && (Lof(j) == L0 || ride.count(Lof(j)))) {
        const int as = asof(j);
        if (rows[0] != as && rows[1] != as) {
            if (nr == mw::NSMAX) break;
            rows[nr++] = as;
        }
        ++j;
    }
    return j;
}

// The distinct band-limits of a chunk, in chunk order (descending).
std::vector<int> chunk_ls(const Chunk& c)
{
    std::vector<int> a;
    for (int L : c.Ls)
        if (a.empty() || a.back() != L) a.push_back(L);
    return a;
}

// Autotuned group size per (band-limit, reality, maps of that band-limit and reality), from mw_prepare.
std::map<std::tuple<int, int, int>, int> g_tuned;

int pow2_ceil(int n) { return n <= 1 ? 1 : n <= 2 ? 2 : n <= 4 ? 4 : 8; }

// Chunk capacity: at most MAXB maps and 8 GiB of workspace.
int chunk_cap(int L)
{
    const size_t lim = (size_t)8 << 30;
    const size_t cap = std::min<size_t>(mw::MAXB, std::max<size_t>(1, lim / ws_need(L)));
    return (int)std::max<size_t>(cap, 1);
}

// Group size of a mixed-precision chunk: the autotuned one for this shape, else
// the largest the LDS allows, up to the map count.
int group_size(int L, int real, int n)
{
    auto it = g_tuned.find(std::make_tuple(L, real, n));
    if (it != g_tuned.end()) return it->second;
    return std::min(pow2_ceil(n), mw::mix_group_max());
}

// Chunks of a call (host only: no plan, no allocation), the same for the call
// itself, mw_prepare and mw_workspace_size.
std::vector<Chunk> make_chunks(const int32_t* L, const int32_t* spin, const int32_t* reality, int batch,
                               int precision)
{
    const bool mix = precision != MW_FP64;
    // class key: (-L, reality, spin) in FP64, (reality) in mixed precision;
    // members sorted by (-L, |s|, s, index)
    std::map<std::tuple<int, int, int>, std::vector<std::tuple<int, int, int, int>>> cls;
    for (int b = 0; b < batch; ++b) {
        const int as = spin[b] < 0 ? -spin[b] : spin[b];
        cls[std::make_tuple(mix ? 0 : -L[b], reality[b], mix ? 0 : spin[b])].push_back(
            std::make_tuple(-L[b], as, spin[b], b));
    }
    std::vector<Chunk> out;
    for (auto& kv : cls) {
        const int rc_ = std::get<1>(kv.first);
        auto v = kv.second;
        std::sort(v.begin(), v.end());
        // group size per band-limit L: the autotuned one for (L, reality, maps
        // of band-limit <= L and that reality: those a group starting at L can
        // take), else the largest the LDS allows
        std::map<int, int> G;
        for (const auto& t : v) G[-std::get<0>(t)] = 0;
        for (auto& kl : G) {
            int nle = 0;
            for (const auto& t : v) nle += (-std::get<0>(t) <= kl.first) ? 1 : 0;
            kl.second = mix ? group_size(kl.first, rc_, nle) : 1;
        }
        const int cap = chunk_cap(-std::get<0>(v[0]));
        // Maps of a band-limit fewer than the largest group ride along in the
        // last group of a larger band-limit (its chains reach their degrees
        // already); band-limits with that many maps or more keep to their own
        // groups, since a group of mixed band-limits costs an extra launch of
        // every Fourier stage and saves at most one small group.
        std::set<int> ride;
        if (mix) {
            std::map<int, int> nl;
            for (const auto& t : v) ++nl[-std::get<0>(t)];
            for (const auto& kl : nl)
                if (kl.first != -std::get<0>(v[0]) && kl.second < mw::mix_group_max()) ride.insert(kl.first);
        }
        auto Lof = [&](size_t k) { return -std::get<0>(v[k]); };
        auto asof = [&](size_t k) { return std::get<1>(v[k]); };
        // whole groups, formed as mix_of forms them, go into chunks of equal
        // group band-limit up to the capacity
        size_t i = 0;
        while (i < v.size()) {
            Chunk c;
            c.L = -std::get<0>(v[i]); c.real = rc_; c.G = G; c.ride = ride;
            while (i < v.size() && -std::get<0>(v[i]) == c.L) {
                const size_t j = mix ? group_end(v.size(), i, Lof, asof, G, ride) : i + 1;
                if (!c.maps.empty() && c.maps.size() + (j - i) > (size_t)cap) break;
                for (size_t k = i; k < j; ++k) {
                    c.maps.push_back(std::get<3>(v[k]));
                    c.spins.push_back(std::get<2>(v[k]));
                    c.Ls.push_back(-std::get<0>(v[k]));
                }
                i = j;
            }
            c.s = c.spins[0];
            out.push_back(c);
        }
    }
    // chunks of one band-limit run next to each other (the two chunk streams then
    // overlap stages of similar sizes)
    std::stable_sort(out.begin(), out.end(), [](const Chunk& a, const Chunk& b) { return a.L > b.L; });
    return out;
}

// Per-map descriptor of one stage: map k of the chunk reads in(k), writes out(k).
template <class In, class Out>
mw::Batch batch_of(const Chunk& c, In in, Out out)
{
    mw::Batch B{};
    B.n = (int)c.maps.size();
    for (int k = 0; k < B.n; ++k) {
        B.in[k] = in(k);
        B.out[k] = out(k);
        B.s[k] = c.spins[k];
    }
    return B;
}

// The same for the maps of band-limit L of the chunk (map k reads in(k) with k
// the chunk's index): one stage launch of that band-limit.
template <class In, class Out>
mw::Batch batch_sub(const Chunk& c, int L, In in, Out out)
{
    mw::Batch B{};
    for (int k = 0; k < (int)c.maps.size(); ++k) {
        if (c.Ls[k] != L) continue;
        B.in[B.n] = in(k);
        B.out[B.n] = out(k);
        B.s[B.n] = c.spins[k];
        ++B.n;
    }
    return B;
}

// The distinct |s| of a chunk (ascending).
std::vector<int> chunk_abs_spins(const Chunk& c)
{
    std::vector<int> a;
    for (int s : c.spins) a.push_back(s < 0 ? -s : s);
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
    return a;
}

// One launch of a mixed contraction: up to MIXG groups with the same spin rows
// and the same largest band-limit L (the plan the launch runs).
struct MixLaunch {
    mw::MixBatch M{};
    int L = 0;
    int G = 1;   // the group size limit of its groups (kernel instance)
    int asmax = 0;   // the largest |s| of the spin rows (its spin table's work list runs the inverse)
};

// Groups of the chunk's maps (in chunk order, sorted by (-L, |s|)): up to
// c.G[L] maps, L the band-limit of the group's first (largest) map, with at most
// two different |s|; groups with the same spin rows and the same largest
// band-limit share launches.  stab(L, as) gives the spin table of
// band-limit L and |s| = as (inverse) or nullptr (forward).
template <class Src, class Dst, class Tab>
std::vector<MixLaunch> mix_of(const Chunk& c, Src src, Dst dst, Tab stab)
{
    // groups by (largest L, spin rows (as0, as1 or -1))
    std::map<std::tuple<int, int, int>, std::vector<mw::MixMaps>> byrows;
    const int n = (int)c.maps.size();
    auto Lof = [&](size_t k) { return c.Ls[k]; };
    auto asof = [&](size_t k) { return c.spins[k] < 0 ? -c.spins[k] : c.spins[k]; };
    for (int i = 0; i < n;) {
        mw::MixMaps mm{};
        int rows[mw::NSMAX] = {0, 0}, nr = 0, nm = 0, Lg = 0;
        const int iend = (int)group_end((size_t)n, (size_t)i, Lof, asof, c.G, c.ride);
        while (i < iend) {
            const int s = c.spins[i], as = s < 0 ? -s : s;
            int j = 0;
            while (j < nr && rows[j] != as) ++j;
            if (j == nr) rows[nr++] = as;
            mm.src[nm] = (const float*)src(i);
            mm.dst[nm] = (double2*)dst(i);
            mm.L[nm] = c.Ls[i];
            Lg = std::max(Lg, c.Ls[i]);
            mm.meta |= (j << (4 + nm)) | ((s < 0 ? 1 : 0) << (12 + nm));
            ++nm;
            ++i;
        }
        mm.meta |= nm;
        byrows[std::make_tuple(-Lg, rows[0], nr > 1 ? rows[1] : -1)].push_back(mm);
    }
    std::vector<MixLaunch> out;
    for (auto& kv : byrows) {
        const auto& gs = kv.second;
        const int Lg = -std::get<0>(kv.first), as0 = std::get<1>(kv.first), as1 = std::get<2>(kv.first);
        for (size_t k = 0; k < gs.size(); k += mw::MIXG) {
            MixLaunch ml;
            ml.L = Lg;
            ml.G = c.G.at(Lg);
            ml.M.ng = (int)std::min<size_t>(mw::MIXG, gs.size() - k);
            for (int g = 0; g < ml.M.ng; ++g) ml.M.g[g] = gs[k + g];
            ml.M.ns = as1 >= 0 ? 2 : 1;
            ml.M.as[0] = as0;
            ml.M.as[1] = as1 >= 0 ? as1 : as0;
            for (int j = 0; j < mw::NSMAX; ++j) {
                const SpinTable* t = stab(Lg, ml.M.as[j]);
                ml.M.stab[j] = t ? t->val : nullptr;
                ml.M.stabk[j] = t ? t->k : nullptr;
                ml.M.ssv[j] = t ? t->sval : nullptr;
                ml.M.ssvf[j] = t ? t->svalf : nullptr;
            }
            ml.asmax = std::max(ml.M.as[0], ml.M.as[1]);
            out.push_back(ml);
        }
    }
    return out;
}

// Plans of one chunk by band-limit; spin tables by (band-limit, |s|).
using ChunkPlans = std::map<int, const Plan*>;
using ChunkSpins = std::map<std::pair<int, int>, const SpinTable*>;

// compact: maps in the compact storage of Sec. IV-C ((L-1)(2L-1)+1 samples, the
// south pole once), expanded or contracted by the phi stages.
// plans: the plan of every band-limit of the chunk; sps: the spin tables of its
// (band-limits, |s|).
hipError_t run_chunk(Op op, const Chunk& c, const ChunkPlans& plans, const ChunkSpins& sps, int precision,
                     void* const* ptrs, void* ws, int Lws, hipStream_t st, bool prof = true, bool compact = false)
{
    const int pole_in = compact ? 1 : 0;    // a map read as the forward's input: expand the pole sample
    const int pole_out = compact ? 1 : 0;   // a map written by the inverse: keep the pole sample
    const int pole_adj = compact ? 2 : 0;   // the adjoints of those two
    const bool mix = precision != MW_FP64;
    const int s = c.s, real = c.real;
    const std::vector<int> Ls = chunk_ls(c);
    auto user_in = [&](int k) { return (void*)ptrs[2 * c.maps[k]]; };
    auto user_out = [&](int k) { return (void*)ptrs[2 * c.maps[k] + 1]; };
    auto w0 = [&](int k) { return (void*)slot(ws, Lws, c.Ls[k], k).W0; };
    auto w1 = [&](int k) { return (void*)slot(ws, Lws, c.Ls[k], k).W1; };
    auto w2 = [&](int k) { return (void*)slot(ws, Lws, c.Ls[k], k).W2; };
    hipError_t e = hipSuccess;
    auto go = [&](int stage, auto launch) {
        if (e == hipSuccess) e = staged(stage, st, prof, launch);
    };
    // one launch of a stage per band-limit of the chunk: launch(plan, maps of that L)
    auto per_l = [&](int stage, auto in, auto out, auto launch) {
        for (int L : Ls) {
            const Plan& p = *plans.at(L);
            const mw::Batch B = batch_sub(c, L, in, out);
            go(stage, [&] { return launch(p, B); });
        }
    };
    auto tab = [&](int L, int as) -> const SpinTable* {
        auto it = sps.find(std::make_pair(L, as));
        return it == sps.end() ? nullptr : it->second;
    };
    // the mixed contractions of the chunk: one launch per (largest L, spin rows)
    auto mix_forward = [&](int stage, auto src, auto dst) {
        for (const MixLaunch& ml : mix_of(c, src, dst, tab))
            go(stage, [&] { return mw::launch_contract_forward_mix(*plans.at(ml.L), ml.M, ml.G, ml.M.ns, st); });
    };
    // FP64 chunks hold one band-limit
    const Plan& p0 = *plans.at(c.L);
    switch (op) {
    case Op::Forward: {
        per_l(0, user_in, w0, [&](const Plan& p, const mw::Batch& B) {
            return mw::launch_phi_forward(p, B, real, TWO_PI / (double)p.N1, pole_in, st);
        });
        per_l(1, w0, w1, [&](const Plan& p, const mw::Batch& B) { return mw::launch_theta_forward(p, B, mix, real, st); });
        if (mix) {
            mix_forward(2, w1, user_out);
        } else {
            const SpinTable* sp = tab(c.L, s < 0 ? -s : s);
            if (!sp) return hipErrorInvalidValue;
            const mw::Batch B3 = batch_of(c, w1, user_out);
            go(2, [&] {
                return mw::launch_contract_forward(p0, *sp, s, real, (const double*)w1(0), ws_need(Lws) / 8, B3, st);
            });
        }
        break;
    }
    case Op::Inverse:
    case Op::ForwardAdjoint: {
        // The adjoint of the forward starts with the inverse's contraction (the
        // conjugate transpose of the forward's contraction and fold) on the
        // coefficients as given (no real-map expansion), then the theta and phi
        // adjoints; with real = 1 it stores Re(A^H y).
        const bool inv = op == Op::Inverse;
        // A lone real map runs the FP64 inverse contraction in either precision:
        // its triangle kernel (one chain per pair (m, n), (n, m), orders m >= 0
        // only) has no mixed form, and a group of one shares no chain.
        const bool mixc = mix && !(inv && real && c.maps.size() == 1);
        per_l(8, user_in, w2, [&](const Plan& p, const mw::Batch& B) {
            return mw::launch_inverse_stream(p, inv ? real : 0, B, mixc, st);
        });
        if (mixc) {
            for (const MixLaunch& ml : mix_of(c, w2, w0, tab)) {
                const SpinTable* wsp = tab(ml.L, ml.asmax);
                if (!wsp) { e = hipErrorInvalidValue; break; }
                go(inv ? 3 : 6, [&] {
                    return mw::launch_contract_inverse_mix(*plans.at(ml.L), *wsp, ml.M, ml.G, ml.M.ns, st);
                });
            }
        } else {
            const SpinTable* sp = tab(c.L, s < 0 ? -s : s);
            if (!sp) return hipErrorInvalidValue;
            // the FP64 kernels read the stream from the workspace and f_lm itself
            const mw::Batch B2 = batch_of(c, user_in, w0);
            go(inv ? 3 : 6, [&] {
                return mw::launch_contract_inverse(p0, *sp, s, inv ? real : 0, (const double*)w2(0), ws_need(Lws) / 8,
                                                   B2, st);
            });
        }
        if (inv) {
            // real maps: orders m >= 0 only, negative orders by conjugate symmetry
            per_l(4, w0, w1, [&](const Plan& p, const mw::Batch& B) { return mw::launch_theta_inverse(p, B, real, st); });
            per_l(5, w1, user_out, [&](const Plan& p, const mw::Batch& B) {
                return mw::launch_phi_inverse(p, B, real ? 2 : 0, 1.0, pole_out, st);
            });
        } else {
            per_l(8, w0, w1, [&](const Plan& p, const mw::Batch& B) { return mw::launch_theta_forward_adjoint(p, B, st); });
            per_l(8, w1, user_out, [&](const Plan& p, const mw::Batch& B) {
                return mw::launch_phi_inverse(p, B, real, TWO_PI / (double)p.N1, pole_adj, st);
            });
        }
        break;
    }
    case Op::InverseAdjoint: {
        // grid -> coefficients: phi and theta adjoints, then the forward's
        // contraction (the conjugate transpose of the inverse's); with real = 1
        // the real-map coefficient expansion is adjoined last.
        per_l(8, user_in, w0, [&](const Plan& p, const mw::Batch& B) {
            return mw::launch_phi_forward(p, B, real, 1.0, pole_adj, st);
        });
        per_l(8, w0, w1, [&](const Plan& p, const mw::Batch& B) {
            return mw::launch_theta_inverse_adjoint(p, B, mix, st);
        });
        if (mix) {
            mix_forward(7, w1, user_out);
        } else {
            const SpinTable* sp = tab(c.L, s < 0 ? -s : s);
            if (!sp) return hipErrorInvalidValue;
            const mw::Batch B3 = batch_of(c, w1, user_out);
            go(7, [&] {
                return mw::launch_contract_forward(p0, *sp, s, 0, (const double*)w1(0), ws_need(Lws) / 8, B3, st);
            });
        }
        if (real)
            per_l(8, w1, user_out, [&](const Plan& p, const mw::Batch& B) { return mw::launch_real_fold(p.L, B, st); });
        break;
    }
    }
    return e;
}

int batch_lmax(const int32_t* L, int batch)
{
    int m = 0;
    for (int b = 0; b < batch; ++b) m = std::max(m, (int)L[b]);
    return m;
}

size_t chunks_ws(const std::vector<Chunk>& ch, int Lws)
{
    size_t slots = 1;
    for (const Chunk& c : ch) slots = std::max(slots, c.maps.size());
    return slots * ws_need(Lws) + 256;
}

// Workspace of a call: one half per chunk stream when it has several chunks.
size_t call_ws(const std::vector<Chunk>& ch, int Lws) { return (ch.size() > 1 ? 2 : 1) * chunks_ws(ch, Lws); }

// The plans of a chunk's band-limits and the spin tables of every (band-limit,
// |s|) of the chunk (a mixed group's chains run to its largest band-limit with
// the rows of all its spins).
int resolve_chunk(DeviceState& d, const Chunk& c, bool may_alloc, ChunkPlans& plans, ChunkSpins& tabs)
{
    int rc;
    for (int Lc : chunk_ls(c)) {
        const Plan* p = nullptr;
        if ((rc = get_plan(d, Lc, may_alloc, &p))) return rc;
        plans[Lc] = p;
        for (int as : chunk_abs_spins(c)) {
            if (as >= Lc) continue;   // no map of band-limit Lc has this spin (|s| < L)
            const SpinTable* t = nullptr;
            if ((rc = get_spin(d, *p, as, may_alloc, &t))) return rc;
            tabs[std::make_pair(Lc, as)] = t;
        }
    }
    return MW_OK;
}

int run(Op op, const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
        void* const* ptrs, int32_t precision, void* stream, bool compact = false)
{
    int rc = validate(L, spin, reality, batch, ptrs, precision, true);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MW_EHIP, "hipGetDevice failed");
    const bool may_alloc = !capturing(st);
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState& d = g_dev[dev];
    const std::vector<Chunk> chunks = make_chunks(L, spin, reality, batch, precision);
    // every plan, spin table and the workspace are resolved before anything is
    // enqueued, so that a failure leaves the stream (and a capture) untouched
    std::vector<ChunkPlans> plans(chunks.size());
    std::vector<ChunkSpins> spins(chunks.size());
    for (size_t i = 0; i < chunks.size(); ++i)
        if ((rc = resolve_chunk(d, chunks[i], may_alloc, plans[i], spins[i]))) return rc;
    const int Lws = batch_lmax(L, batch);
    const size_t need = call_ws(chunks, Lws);
    void* ws = nullptr;
    auto uw = d.user_ws.find(st);
    if (uw != d.user_ws.end()) {
        if (uw->second.second < need)
            return fail(MW_ENOMEM, "the workspace set for this stream has %zu bytes, this call needs %zu",
                        uw->second.second, need);
        ws = uw->second.first;
    } else if ((rc = get_ws(d, need, may_alloc, &ws))) {
        return rc;
    }
    // several chunks alternate over the two chunk streams (per-stage profiling
    // keeps the caller's stream, so that its events time one launch each)
    const bool lanes = chunks.size() > 1 && !g_prof_on && (d.lane[0] || (may_alloc && make_lanes(d)));
    const size_t half = chunks_ws(chunks, Lws);
    if (lanes) {
        if (hipEventRecord(d.fork, st) != hipSuccess || hipStreamWaitEvent(d.lane[0], d.fork, 0) != hipSuccess ||
            hipStreamWaitEvent(d.lane[1], d.fork, 0) != hipSuccess)
            return fail(MW_EHIP, "stream fork failed");
    }
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < chunks.size() && e == hipSuccess; ++i) {
        hipStream_t cs = lanes ? d.lane[i & 1] : st;
        void* cws = lanes ? (void*)((char*)ws + (i & 1) * half) : ws;
        e = run_chunk(op, chunks[i], plans[i], spins[i], precision, ptrs, cws, Lws, cs, true, compact);
    }
    if (lanes) {
        // join both chunk streams back into the caller's stream, also after a failed launch
        bool joined = true;
        for (int k = 0; k < 2; ++k)
            joined = (hipEventRecord(d.join[k], d.lane[k]) == hipSuccess &&
                      hipStreamWaitEvent(st, d.join[k], 0) == hipSuccess) && joined;
        if (!joined) return fail(MW_EHIP, "stream join failed");
    }
    if (e != hipSuccess) return fail(MW_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    g_last_error.clear();
    return MW_OK;
}

// ---- the group-size autotuner and its cache --------------------------------
// Entries "gfx950 L real n G" (one per line; anything else is skipped), read
// from and appended to the file named by MW_TUNE_CACHE when that is set.
const char* tune_cache_path()
{
    const char* p = getenv("MW_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

int tune_cache_load(const char* path)
{
    FILE* f = fopen(path, "r");
    if (!f) return 0;
    char line[256];
    int got = 0;
    while (fgets(line, sizeof(line), f)) {
        char arch[32];
        int Lc, rc_, n, G;
        char tail[8];
        if (sscanf(line, "%31s %d %d %d %d %7s", arch, &Lc, &rc_, &n, &G, tail) != 5) continue;
        if (strcmp(arch, "gfx950") != 0 || Lc < 1 || Lc > MW_LMAX || (rc_ != 0 && rc_ != 1) || n < 1 ||
            (G != 1 && G != 2 && G != 4 && G != 8) || G > mw::mix_group_max())
            continue;
        g_tuned[std::make_tuple(Lc, rc_, n)] = G;
        ++got;
    }
    fclose(f);
    return got;
}

void tune_cache_append(const char* path, int Lc, int rc_, int n, int G)
{
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "gfx950 %d %d %d %d\n", Lc, rc_, n, G);
    fclose(f);
}

// Times the mixed forward contraction of the maps of each (L, reality) of a call
// (up to one chunk's worth, with their own spins), per candidate group size, on
// zeroed workspace, and keeps the fastest per map for the key (L, reality, maps
// of band-limit <= L and that reality), the group size of the groups that start
// at L in make_chunks; results do not depend on the choice (each map keeps its
// own accumulators over the shared chains).
int autotune(DeviceState& d, const int32_t* L, const int32_t* spin, const int32_t* reality, int batch)
{
    const char* cache = tune_cache_path();
    if (cache) tune_cache_load(cache);
    // the maps of each (L, reality), sorted by (|s|, s) as in a chunk
    std::map<std::pair<int, int>, std::vector<std::tuple<int, int, int>>> cls;
    for (int b = 0; b < batch; ++b) {
        const int as = spin[b] < 0 ? -spin[b] : spin[b];
        cls[std::make_pair(L[b], reality[b])].push_back(std::make_tuple(as, spin[b], b));
    }
    const int Lws = batch_lmax(L, batch);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(MW_EHIP, "hipEventCreate failed");
    int rc = MW_OK;
    for (auto& kv : cls) {
        const int Lc = kv.first.first, rc_ = kv.first.second;
        int n = 0;   // maps of band-limit <= Lc and this reality
        for (int b = 0; b < batch; ++b) n += (reality[b] == rc_ && L[b] <= Lc) ? 1 : 0;
        const auto key = std::make_tuple(Lc, rc_, n);
        if (g_tuned.count(key)) continue;
        auto v = kv.second;
        std::sort(v.begin(), v.end());
        Chunk c0;
        c0.L = Lc; c0.real = rc_;
        for (int k = 0; k < std::min(n, chunk_cap(Lc)); ++k) {
            c0.maps.push_back(std::get<2>(v[k]));
            c0.spins.push_back(std::get<1>(v[k]));
            c0.Ls.push_back(Lc);
        }
        c0.s = c0.spins[0];
        ChunkPlans plans;
        ChunkSpins tabs;   // the timed launches read the same spin tables as a call
        if ((rc = resolve_chunk(d, c0, true, plans, tabs))) break;
        const int gmax = std::min(pow2_ceil(n), mw::mix_group_max());
        const int nt = (int)c0.maps.size();
        void* ws = nullptr;
        if ((rc = get_ws(d, (size_t)nt * ws_need(Lws) + 256, true, &ws))) break;
        for (int k = 0; k < nt; ++k) (void)hipMemset(slot(ws, Lws, Lc, k).W1, 0, ws_region(Lc, 1));
        // from the largest size down: a smaller group must be 3% faster per map
        // in the forward contraction to be chosen (the inverse, not timed here,
        // gains from larger groups as well)
        int best = gmax;
        double best_t = 1e30;
        for (int G = gmax; G >= 1; G >>= 1) {
            Chunk c = c0;
            c.G[Lc] = G;
            const std::vector<MixLaunch> ls =
                mix_of(c, [&](int k) { return (void*)slot(ws, Lws, Lc, k).W1; },
                       [&](int k) { return (void*)slot(ws, Lws, Lc, k).W0; },
                       [&](int Lt, int as) -> const SpinTable* {
                           auto it = tabs.find(std::make_pair(Lt, as));
                           return it == tabs.end() ? nullptr : it->second;
                       });
            double t = 1e30;   // the fastest of four timed repetitions (after one warm-up)
            for (int rep = 0; rep < 5 && !rc; ++rep) {
                (void)hipEventRecord(e0, nullptr);
                hipError_t e = hipSuccess;
                for (const MixLaunch& ml : ls)
                    if (e == hipSuccess) e = mw::launch_contract_forward_mix(*plans.at(Lc), ml.M, G, ml.M.ns, nullptr);
                (void)hipEventRecord(e1, nullptr);
                if (e != hipSuccess) { rc = fail(MW_EHIP, "autotune launch failed"); break; }
                (void)hipEventSynchronize(e1);
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0) t = std::min(t, (double)ms);
            }
            if (rc) break;
            const double per_map = t / nt;
            if (per_map < best_t * 0.97) { best_t = per_map; best = G; }
        }
        if (rc) break;
        g_tuned[key] = best;
        if (cache) tune_cache_append(cache, Lc, rc_, n, best);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // namespace

extern "C" {

int mw_forward(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
               void* const* ptrs, int32_t precision, void* stream)
{
    return run(Op::Forward, L, spin, reality, batch, ptrs, precision, stream);
}

int mw_forward_noalloc(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                       void* const* ptrs, int32_t precision, void* stream)
{
    int rc = validate(L, spin, reality, batch, ptrs, precision, true);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MW_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState& d = g_dev[dev];
    const std::vector<Chunk> chunks = make_chunks(L, spin, reality, batch, precision);
    std::vector<ChunkPlans> plans(chunks.size());
    std::vector<ChunkSpins> tabs(chunks.size());
    for (size_t i = 0; i < chunks.size(); ++i)
        if ((rc = resolve_chunk(d, chunks[i], false, plans[i], tabs[i])))
            return fail(MW_ENOMEM, "mw_forward_noalloc: a plan or spin table of this call is not prepared (call "
                                   "mw_prepare first)");
    // the chunks run one after another on the caller's stream, all in the one
    // set of workspace slots
    const int Lws = batch_lmax(L, batch);
    const size_t need = chunks_ws(chunks, Lws);
    if (need > NOALLOC_BYTES)
        return fail(MW_ENOMEM, "mw_forward_noalloc: this call needs %zu bytes of workspace, the static scratch holds %zu",
                    need, NOALLOC_BYTES);
    if (!d.scratch) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MW_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        d.scratch = ptr;
    }
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < chunks.size() && e == hipSuccess; ++i)
        e = run_chunk(Op::Forward, chunks[i], plans[i], tabs[i], precision, ptrs, d.scratch, Lws, st, false);
    if (e != hipSuccess) return fail(MW_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    g_last_error.clear();
    return MW_OK;
}

int mw_inverse(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
               void* const* ptrs, int32_t precision, void* stream)
{
    return run(Op::Inverse, L, spin, reality, batch, ptrs, precision, stream);
}

int mw_forward_adjoint(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                       void* const* ptrs, int32_t precision, void* stream)
{
    return run(Op::ForwardAdjoint, L, spin, reality, batch, ptrs, precision, stream);
}

int mw_inverse_adjoint(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                       void* const* ptrs, int32_t precision, void* stream)
{
    return run(Op::InverseAdjoint, L, spin, reality, batch, ptrs, precision, stream);
}

int mw_quadrature_weights(int32_t L, int32_t spin, double* q, void* stream)
{
    if (L < 1 || L > MW_LMAX) return fail(MW_EINVAL, "L = %d outside [1, %d]", L, MW_LMAX);
    if (spin <= -L || spin >= L) return fail(MW_EINVAL, "|spin| = %d must be < L = %d", spin, L);
    if (!q) return fail(MW_EINVAL, "q must be non-NULL");
    const hipError_t e = mw::launch_quad_weights(L, spin, q, (hipStream_t)stream);
    if (e != hipSuccess) return fail(MW_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    g_last_error.clear();
    return MW_OK;
}

int mw_integrate(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch, void* const* ptrs,
                 int32_t grid, void* stream)
{
    int rc = validate(L, spin, reality, batch, ptrs, MW_FP64, true);
    if (rc) return rc;
    if (grid != MW_GRID_QUADRATURE && grid != MW_GRID_TRANSFORM)
        return fail(MW_EINVAL, "grid must be MW_GRID_QUADRATURE or MW_GRID_TRANSFORM (got %d)", grid);
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MW_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState& d = g_dev[dev];
    // maps of equal (L, spin, reality) share a launch; the ring partials of a
    // chunk (maps x L complex) live in the workspace
    const std::vector<Chunk> chunks = make_chunks(L, spin, reality, batch, MW_FP64);
    size_t need = 256;
    for (const Chunk& c : chunks) need = std::max(need, c.maps.size() * (size_t)c.L * sizeof(double2) + 256);
    void* ws = nullptr;
    auto uw = d.user_ws.find(st);
    if (uw != d.user_ws.end()) {
        if (uw->second.second < need)
            return fail(MW_ENOMEM, "the workspace set for this stream has %zu bytes, this call needs %zu",
                        uw->second.second, need);
        ws = uw->second.first;
    } else if ((rc = get_ws(d, need, !capturing(st), &ws))) {
        return rc;
    }
    double2* partial = (double2*)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    hipError_t e = hipSuccess;
    for (size_t i = 0; i < chunks.size() && e == hipSuccess; ++i) {
        const Chunk& c = chunks[i];
        const int nphi = grid == MW_GRID_QUADRATURE ? c.L : 2 * c.L - 1;
        const mw::Batch B = batch_of(c, [&](int k) { return (void*)ptrs[2 * c.maps[k]]; },
                                     [&](int k) { return (void*)ptrs[2 * c.maps[k] + 1]; });
        e = mw::launch_integrate(c.L, nphi, c.real, B, partial, st);
    }
    if (e != hipSuccess) return fail(MW_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    g_last_error.clear();
    return MW_OK;
}

int mw_forward_compact(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                       void* const* ptrs, int32_t precision, void* stream)
{
    return run(Op::Forward, L, spin, reality, batch, ptrs, precision, stream, true);
}

int mw_inverse_compact(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                       void* const* ptrs, int32_t precision, void* stream)
{
    return run(Op::Inverse, L, spin, reality, batch, ptrs, precision, stream, true);
}

int mw_forward_adjoint_compact(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                               void* const* ptrs, int32_t precision, void* stream)
{
    return run(Op::ForwardAdjoint, L, spin, reality, batch, ptrs, precision, stream, true);
}

int mw_inverse_adjoint_compact(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                               void* const* ptrs, int32_t precision, void* stream)
{
    return run(Op::InverseAdjoint, L, spin, reality, batch, ptrs, precision, stream, true);
}

int mw_spin_flip(const int32_t* L, const int32_t* spin, int32_t batch, void* const* ptrs, void* stream)
{
    if (batch < 1 || !L || !spin || !ptrs) return fail(MW_EINVAL, "batch >= 1 and non-NULL L, spin and ptrs required");
    for (int b = 0; b < batch; ++b) {
        if (L[b] < 1 || L[b] > MW_LMAX) return fail(MW_EINVAL, "map %d: L = %d outside [1, %d]", b, L[b], MW_LMAX);
        if (spin[b] <= -L[b] || spin[b] >= L[b])
            return fail(MW_EINVAL, "map %d: |spin| = %d must be < L = %d", b, spin[b], L[b]);
        if (!ptrs[2 * b] || !ptrs[2 * b + 1]) return fail(MW_EINVAL, "map %d: NULL pointer", b);
    }
    hipStream_t st = (hipStream_t)stream;
    // maps of equal band-limit share a launch (at most MAXB per launch)
    std::map<int, std::vector<int>> byL;
    for (int b = 0; b < batch; ++b) byL[L[b]].push_back(b);
    hipError_t e = hipSuccess;
    for (auto& kv : byL) {
        for (size_t i = 0; i < kv.second.size() && e == hipSuccess; i += mw::MAXB) {
            mw::Batch B{};
            B.n = (int)std::min<size_t>(mw::MAXB, kv.second.size() - i);
            for (int k = 0; k < B.n; ++k) {
                const int b = kv.second[i + k];
                B.in[k] = ptrs[2 * b];
                B.out[k] = ptrs[2 * b + 1];
                B.s[k] = spin[b];
            }
            e = mw::launch_spin_flip(kv.first, B, st);
        }
    }
    if (e != hipSuccess) return fail(MW_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    g_last_error.clear();
    return MW_OK;
}

int mw_workspace_size(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                      int32_t precision, size_t* bytes)
{
    int rc = validate(L, spin, reality, batch, nullptr, precision, false);
    if (rc) return rc;
    if (!bytes) return fail(MW_EINVAL, "bytes must be non-NULL");
    // the chunks the call itself would form (group sizes as tuned so far)
    std::lock_guard<std::mutex> lock(g_mu);
    *bytes = call_ws(make_chunks(L, spin, reality, batch, precision), batch_lmax(L, batch));
    return MW_OK;
}

int mw_prepare(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch, int32_t precision)
{
    int rc = validate(L, spin, reality, batch, nullptr, precision, false);
    if (rc) return rc;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MW_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lock(g_mu);
    // work already in flight (on any stream) may use the workspace that the
    // autotuner below overwrites
    if (hipDeviceSynchronize() != hipSuccess) return fail(MW_EHIP, "hipDeviceSynchronize failed");
    DeviceState& d = g_dev[dev];
    for (int b = 0; b < batch; ++b) {
        const Plan* p;
        const SpinTable* sp;
        const int as = spin[b] < 0 ? -spin[b] : spin[b];
        if ((rc = get_plan(d, L[b], true, &p))) return rc;
        if ((rc = get_spin(d, *p, as, true, &sp))) return rc;
    }
    const std::vector<Chunk> chunks = make_chunks(L, spin, reality, batch, precision);
    for (const Chunk& c : chunks) {
        ChunkPlans plans;
        ChunkSpins tabs;
        if ((rc = resolve_chunk(d, c, true, plans, tabs))) return rc;
    }
    if (precision != MW_FP64 && (rc = autotune(d, L, spin, reality, batch))) return rc;
    void* ws = nullptr;
    if ((rc = get_ws(d, call_ws(chunks, batch_lmax(L, batch)), true, &ws))) return rc;
    if (chunks.size() > 1 && !make_lanes(d)) return fail(MW_EHIP, "chunk stream creation failed");
    if (hipDeviceSynchronize() != hipSuccess) return fail(MW_EHIP, "hipDeviceSynchronize failed");
    return MW_OK;
}

int mw_set_workspace(void* dptr, size_t bytes, void* stream)
{
    if (dptr && bytes == 0) return fail(MW_EINVAL, "a workspace needs bytes > 0");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MW_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState& d = g_dev[dev];
    hipStream_t st = (hipStream_t)stream;
    if (dptr) d.user_ws[st] = std::make_pair(dptr, bytes);
    else d.user_ws.erase(st);
    g_last_error.clear();
    return MW_OK;
}

int mw_release(void)
{
    std::lock_guard<std::mutex> lock(g_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_dev) {
        (void)hipSetDevice(kv.first);
        (void)hipDeviceSynchronize();
        for (auto& pp : kv.second.plans) mw::free_plan(pp.second);
        for (auto& ss : kv.second.spins) mw::free_spin_table(ss.second);
        if (kv.second.ws) (void)hipFree(kv.second.ws);
        for (void* q : kv.second.retired) (void)hipFree(q);
        for (int k = 0; k < 2; ++k) {
            if (kv.second.lane[k]) (void)hipStreamDestroy(kv.second.lane[k]);
            if (kv.second.join[k]) (void)hipEventDestroy(kv.second.join[k]);
        }
        if (kv.second.fork) (void)hipEventDestroy(kv.second.fork);
    }
    g_dev.clear();
    (void)hipSetDevice(cur);
    return MW_OK;
}

const char* mw_status_string(int status)
{
    switch (status) {
        case MW_OK: return "success";
        case MW_EINVAL: return "invalid argument";
        case MW_ENOMEM: return "allocation failed or resources not prepared";
        case MW_EHIP: return "HIP runtime error";
        case MW_ENOTSUP: return "not supported";
        default: return "unknown status";
    }
}

const char* mw_last_error(void) { return g_last_error.c_str(); }

const char* mw_version(void) { return "mw-hip 0.1 (gfx950)"; }

int mw_profile_enable(int on)
{
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto& r : g_prof) { g_event_pool.push_back(r.a); g_event_pool.push_back(r.b); }
    g_prof.clear();
    g_prof_on = on != 0;
    return MW_OK;
}

int mw_profile_read(double* ms, int* count)
{
    if (!ms || !count) return fail(MW_EINVAL, "ms and count must be non-NULL");
    std::lock_guard<std::mutex> lock(g_mu);
    for (int i = 0; i < MW_PROFILE_NSTAGE; ++i) { ms[i] = 0.0; count[i] = 0; }
    int rc = MW_OK;
    for (auto& r : g_prof) {
        float t = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) {
            rc = fail(MW_EHIP, "event timing failed");
        } else if (r.stage >= 0 && r.stage < MW_PROFILE_NSTAGE) {
            ms[r.stage] += t;
            count[r.stage] += 1;
        }
        g_event_pool.push_back(r.a);
        g_event_pool.push_back(r.b);
    }
    g_prof.clear();
    return rc;
}

int mw_profile_split_fft(int mode)
{
    if (mode != 0 && mode != 1) return fail(MW_EINVAL, "split mode must be 0 or 1");
    std::lock_guard<std::mutex> lock(g_mu);
    mw::g_split_min_n2 = mode ? 2048 : 16384;
    return MW_OK;
}

int mw_profile_inverse_triangle(int mode)
{
    if (mode != 0 && mode != 1) return fail(MW_EINVAL, "triangle mode must be 0 or 1");
    std::lock_guard<std::mutex> lock(g_mu);
    mw::g_inv_tri_all = mode;
    return MW_OK;
}

int mw_profile_tuned_group(int L, int reality, int nmaps, int* G)
{
    if (!G) return fail(MW_EINVAL, "G must be non-NULL");
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_tuned.find(std::make_tuple(L, reality, nmaps));
    *G = (it == g_tuned.end()) ? 0 : it->second;
    return MW_OK;
}

int mw_profile_tune_cache_load(const char* path, int* entries)
{
    if (!path || !entries) return fail(MW_EINVAL, "path and entries must be non-NULL");
    std::lock_guard<std::mutex> lock(g_mu);
    *entries = tune_cache_load(path);
    return MW_OK;
}

const char* mw_profile_stage_name(int stage)
{
    static const char* names[MW_PROFILE_NSTAGE] = {
        "phi_forward", "theta_forward", "contract_forward", "contract_inverse", "theta_inverse",
        "phi_inverse", "contract_forward_adjoint", "contract_inverse_adjoint", "other"};
    return (stage >= 0 && stage < MW_PROFILE_NSTAGE) ? names[stage] : "";
}

}  // extern "C"
