// C ABI of libmw: argument validation, per-device plan/workspace cache and the
// launch sequence of each transform.  See include/mw.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <map>
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

struct DeviceState {
    std::map<int, Plan> plans;                    // by L
    std::map<std::pair<int, int>, SpinTable> spins;  // by (L, |s|)
    void* ws = nullptr;
    size_t ws_bytes = 0;
};

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
hipError_t staged(int stage, hipStream_t st, F&& launch)
{
    if (!g_prof_on) return launch();
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
        if (L[b] < 1 || L[b] > 2048) return fail(MW_EINVAL, "map %d: L = %d outside [1, 2048]", b, L[b]);
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
int get_spin(DeviceState& d, int L, int as, bool may_alloc, const SpinTable** spt)
{
    std::string err;
    auto key = std::make_pair(L, as);
    auto jt = d.spins.find(key);
    if (jt == d.spins.end()) {
        if (!may_alloc) return fail(MW_ENOMEM, "spin table L=%d |s|=%d not prepared", L, as);
        SpinTable t;
        int rc = mw::build_spin_table(L, as, t, err);
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
        if (d.ws) (void)hipFree(d.ws);
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

// Workspace slot k of a call whose largest band-limit is Lmax: three regions,
// W0 (N1 x L complex), W1 (max of N1 x L complex and the H records), W2 (the
// inverse's coefficient stream), each 256-byte aligned.
Regions slot(void* ws, int Lmax, int L, int k)
{
    char* base = (char*)(((uintptr_t)ws + 255) & ~(uintptr_t)255) + (size_t)k * ws_need(Lmax);
    Regions r;
    r.W0 = (double2*)base;
    r.W1 = (double2*)(base + ws_region(L, 0));
    r.W2 = (double*)(base + ws_region(L, 0) + ws_region(L, 1));
    return r;
}

// FP64 launch sequence of one map.
hipError_t run_map(Op op, const Plan& p, const SpinTable* sp, int s, int real, const void* in, void* out,
                   const Regions& w, hipStream_t st)
{
    hipError_t e = hipSuccess;
    const double phi_sc = TWO_PI / (double)p.N1;
    double2* W0 = w.W0;
    double2* W1 = w.W1;
    double* W2 = w.W2;
    switch (op) {
    case Op::Forward:
        e = staged(0, st, [&] { return mw::launch_phi_forward(p, in, real, W0, phi_sc, st); });
        if (e == hipSuccess) e = staged(1, st, [&] { return mw::launch_theta_forward(p, s, W0, W1, 0, st); });
        if (e == hipSuccess)
            e = staged(2, st, [&] { return mw::launch_contract_forward(p, s, real, (const double*)W1, (double2*)out, st); });
        break;
    case Op::Inverse:
        e = staged(8, st, [&] { return mw::launch_inverse_stream(p, s, real, (const double2*)in, W2, 0, st); });
        if (e == hipSuccess) e = staged(3, st, [&] { return mw::launch_contract_inverse(p, *sp, s, W2, W0, st); });
        if (e == hipSuccess) e = staged(4, st, [&] { return mw::launch_theta_inverse(p, s, W0, W1, st); });
        if (e == hipSuccess) e = staged(5, st, [&] { return mw::launch_phi_inverse(p, W1, out, real, 1.0, st); });
        break;
    case Op::ForwardAdjoint:
        // coefficients -> grid: the inverse's contraction is the conjugate transpose
        // of the forward's contraction and fold; then the theta and phi adjoints.
        // The coefficients are used as given (no real-map expansion): with real = 1
        // the result is Re(A^H y), the adjoint of the forward restricted to real maps.
        e = staged(8, st, [&] { return mw::launch_inverse_stream(p, s, 0, (const double2*)in, W2, 0, st); });
        if (e == hipSuccess) e = staged(6, st, [&] { return mw::launch_contract_inverse(p, *sp, s, W2, W0, st); });
        if (e == hipSuccess) e = staged(8, st, [&] { return mw::launch_theta_forward_adjoint(p, s, W0, W1, st); });
        if (e == hipSuccess) e = staged(8, st, [&] { return mw::launch_phi_inverse(p, W1, out, real, phi_sc, st); });
        break;
    case Op::InverseAdjoint:
        // grid -> coefficients: phi and theta adjoints, then the forward's
        // contraction (the conjugate transpose of the inverse's).  With real = 1
        // the real-map coefficient expansion is adjoined last.
        e = staged(8, st, [&] { return mw::launch_phi_forward(p, in, real, W0, 1.0, st); });
        if (e == hipSuccess) e = staged(8, st, [&] { return mw::launch_theta_inverse_adjoint(p, s, W0, W1, 0, st); });
        if (e == hipSuccess)
            e = staged(7, st, [&] { return mw::launch_contract_forward(p, s, 0, (const double*)W1, (double2*)out, st); });
        if (e == hipSuccess && real) e = staged(8, st, [&] { return mw::launch_real_fold(p.L, (double2*)out, st); });
        break;
    }
    return e;
}

// ---- mixed precision: groups of maps of one spin share the Wigner chains ---
struct Group {
    int s = 0, Lmax = 0, G = 1;
    std::vector<int> maps;   // batch indices, band-limits descending
};

// Autotuned group size per (largest band-limit, spin, maps of that spin in the
// call); filled by mw_prepare.
std::map<std::tuple<int, int, int>, int> g_tuned;

int pow2_ceil(int n) { return n <= 1 ? 1 : n <= 2 ? 2 : 4; }

int default_group(const Plan& p, int nmaps) { return std::min(pow2_ceil(nmaps), mw::mix_group_max(p)); }

// Maps of each spin, sorted by band-limit (largest first) and cut into groups
// of the tuned (else default) size.
std::vector<Group> make_groups(DeviceState& d, const int32_t* L, const int32_t* spin, int batch, bool may_alloc,
                               int& rc)
{
    std::map<int, std::vector<int>> by_spin;
    for (int b = 0; b < batch; ++b) by_spin[spin[b]].push_back(b);
    std::vector<Group> out;
    rc = MW_OK;
    for (auto& kv : by_spin) {
        auto& v = kv.second;
        std::stable_sort(v.begin(), v.end(), [L](int a, int b) { return L[a] > L[b]; });
        const int Lmax = L[v.front()];
        const Plan* p = nullptr;
        if ((rc = get_plan(d, Lmax, may_alloc, &p))) return out;
        auto it = g_tuned.find(std::make_tuple(Lmax, kv.first, (int)v.size()));
        const int gsz = (it != g_tuned.end()) ? it->second : default_group(*p, (int)v.size());
        for (size_t i = 0; i < v.size(); i += gsz) {
            Group g;
            g.s = kv.first;
            g.maps.assign(v.begin() + i, v.begin() + std::min(v.size(), i + (size_t)gsz));
            g.Lmax = L[g.maps.front()];
            g.G = pow2_ceil((int)g.maps.size());
            out.push_back(g);
        }
    }
    return out;
}

// One group in mixed precision: per-map Fourier stages in FP64 around one
// shared contraction launch.  Map k of the group uses workspace slot k.
hipError_t run_group(Op op, DeviceState& d, const Group& g, const int32_t* L, const int32_t* reality,
                     void* const* ptrs, void* ws, int Lws, hipStream_t st, int& rc)
{
    hipError_t e = hipSuccess;
    const Plan* pg = nullptr;
    const SpinTable* spg = nullptr;
    const int as = g.s < 0 ? -g.s : g.s;
    if ((rc = get_plan(d, g.Lmax, false, &pg))) return hipSuccess;
    const bool inv = (op == Op::Inverse || op == Op::ForwardAdjoint);
    if (inv && (rc = get_spin(d, g.Lmax, as, false, &spg))) return hipSuccess;
    mw::MixMaps mm{};
    mm.n = (int)g.maps.size();
    std::vector<const Plan*> pl(mm.n);
    for (int k = 0; k < mm.n; ++k) {
        const int b = g.maps[k];
        if ((rc = get_plan(d, L[b], false, &pl[k]))) return hipSuccess;
        const Regions w = slot(ws, Lws, L[b], k);
        mm.L[k] = L[b];
        if (op == Op::Forward || op == Op::InverseAdjoint) {
            mm.src[k] = (const float*)w.W1;
            mm.dst[k] = (double2*)ptrs[2 * b + 1];
        } else {
            mm.src[k] = (const float*)w.W2;
            mm.dst[k] = w.W0;
        }
    }
    // Fourier stages before the contraction
    for (int k = 0; k < mm.n && e == hipSuccess; ++k) {
        const int b = g.maps[k];
        const Plan& p = *pl[k];
        const Regions w = slot(ws, Lws, L[b], k);
        const int real = reality[b];
        const void* in = ptrs[2 * b];
        switch (op) {
        case Op::Forward:
            e = staged(0, st, [&] { return mw::launch_phi_forward(p, in, real, w.W0, TWO_PI / (double)p.N1, st); });
            if (e == hipSuccess) e = staged(1, st, [&] { return mw::launch_theta_forward(p, g.s, w.W0, w.W1, 1, st); });
            break;
        case Op::InverseAdjoint:
            e = staged(8, st, [&] { return mw::launch_phi_forward(p, in, real, w.W0, 1.0, st); });
            if (e == hipSuccess)
                e = staged(8, st, [&] { return mw::launch_theta_inverse_adjoint(p, g.s, w.W0, w.W1, 1, st); });
            break;
        case Op::Inverse:
            e = staged(8, st, [&] { return mw::launch_inverse_stream(p, g.s, real, (const double2*)in, w.W2, 1, st); });
            break;
        case Op::ForwardAdjoint:
            e = staged(8, st, [&] { return mw::launch_inverse_stream(p, g.s, 0, (const double2*)in, w.W2, 1, st); });
            break;
        }
    }
    if (e != hipSuccess) return e;
    // the shared contraction
    if (op == Op::Forward || op == Op::InverseAdjoint)
        e = staged(op == Op::Forward ? 2 : 7, st, [&] { return mw::launch_contract_forward_mix(*pg, g.s, mm, g.G, st); });
    else
        e = staged(op == Op::Inverse ? 3 : 6, st,
                   [&] { return mw::launch_contract_inverse_mix(*pg, *spg, g.s, mm, g.G, st); });
    // Fourier stages after the contraction
    for (int k = 0; k < mm.n && e == hipSuccess; ++k) {
        const int b = g.maps[k];
        const Plan& p = *pl[k];
        const Regions w = slot(ws, Lws, L[b], k);
        const int real = reality[b];
        void* out = ptrs[2 * b + 1];
        switch (op) {
        case Op::Forward:
            break;
        case Op::InverseAdjoint:
            if (real) e = staged(8, st, [&] { return mw::launch_real_fold(p.L, (double2*)out, st); });
            break;
        case Op::Inverse:
            e = staged(4, st, [&] { return mw::launch_theta_inverse(p, g.s, w.W0, w.W1, st); });
            if (e == hipSuccess) e = staged(5, st, [&] { return mw::launch_phi_inverse(p, w.W1, out, real, 1.0, st); });
            break;
        case Op::ForwardAdjoint:
            e = staged(8, st, [&] { return mw::launch_theta_forward_adjoint(p, g.s, w.W0, w.W1, st); });
            if (e == hipSuccess)
                e = staged(8, st, [&] {
                    return mw::launch_phi_inverse(p, w.W1, out, real, TWO_PI / (double)p.N1, st);
                });
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

// Workspace slots a call needs: one for FP64 (maps run in turn), one per map of
// the largest group in mixed precision.
int ws_slots(DeviceState& d, const int32_t* L, const int32_t* spin, int batch, int precision, bool may_alloc,
             int& rc)
{
    rc = MW_OK;
    if (precision == MW_FP64) return 1;
    int slots = 1;
    for (const Group& g : make_groups(d, L, spin, batch, may_alloc, rc)) slots = std::max(slots, (int)g.maps.size());
    return slots;
}

int run(Op op, const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
        void* const* ptrs, int32_t precision, void* stream)
{
    int rc = validate(L, spin, reality, batch, ptrs, precision, true);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MW_EHIP, "hipGetDevice failed");
    const bool may_alloc = !capturing(st);
    const bool need_spin = (op == Op::Inverse || op == Op::ForwardAdjoint);
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState& d = g_dev[dev];
    const int Lws = batch_lmax(L, batch);
    const int slots = ws_slots(d, L, spin, batch, precision, may_alloc, rc);
    if (rc) return rc;
    void* ws = nullptr;
    if ((rc = get_ws(d, (size_t)slots * ws_need(Lws) + 256, may_alloc, &ws))) return rc;
    for (int b = 0; b < batch; ++b) {   // every plan and spin table the call touches
        const Plan* p = nullptr;
        const SpinTable* sp = nullptr;
        if ((rc = get_plan(d, L[b], may_alloc, &p))) return rc;
        if (need_spin && (rc = get_spin(d, L[b], spin[b] < 0 ? -spin[b] : spin[b], may_alloc, &sp))) return rc;
    }
    if (precision == MW_FP64) {
        for (int b = 0; b < batch; ++b) {
            const Plan* p = nullptr;
            const SpinTable* sp = nullptr;
            const int s = spin[b], as = s < 0 ? -s : s;
            get_plan(d, L[b], false, &p);
            if (need_spin) get_spin(d, L[b], as, false, &sp);
            hipError_t e = run_map(op, *p, sp, s, reality[b], ptrs[2 * b], ptrs[2 * b + 1], slot(ws, Lws, L[b], 0), st);
            if (e != hipSuccess) return fail(MW_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
        }
    } else {
        const std::vector<Group> groups = make_groups(d, L, spin, batch, may_alloc, rc);
        if (rc) return rc;
        for (const Group& g : groups) {
            if (need_spin) {
                const SpinTable* sp = nullptr;
                if ((rc = get_spin(d, g.Lmax, g.s < 0 ? -g.s : g.s, may_alloc, &sp))) return rc;
            }
            hipError_t e = run_group(op, d, g, L, reality, ptrs, ws, Lws, st, rc);
            if (rc) return rc;
            if (e != hipSuccess) return fail(MW_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
        }
    }
    g_last_error.clear();
    return MW_OK;
}

// Times the mixed forward contraction of one group per candidate size on the
// workspace (whatever it holds) and keeps the fastest per map.
int autotune(DeviceState& d, const int32_t* L, const int32_t* spin, int batch, hipStream_t st)
{
    std::map<int, std::vector<int>> by_spin;
    for (int b = 0; b < batch; ++b) by_spin[spin[b]].push_back(b);
    const int Lws = batch_lmax(L, batch);
    for (auto& kv : by_spin) {
        auto& v = kv.second;
        int Lmax = 0;
        for (int b : v) Lmax = std::max(Lmax, (int)L[b]);
        const auto key = std::make_tuple(Lmax, kv.first, (int)v.size());
        if (g_tuned.count(key)) continue;
        const Plan* p = nullptr;
        int rc = get_plan(d, Lmax, true, &p);
        if (rc) return rc;
        void* ws = nullptr;
        const int gmax = std::min(pow2_ceil((int)v.size()), mw::mix_group_max(*p));
        if ((rc = get_ws(d, (size_t)std::max(gmax, 1) * ws_need(Lws) + 256, true, &ws))) return rc;
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            return fail(MW_EHIP, "hipEventCreate failed");
        int best = 1;
        double best_t = 1e30;
        for (int G = 1; G <= gmax; G <<= 1) {
            mw::MixMaps mm{};
            mm.n = G;
            for (int k = 0; k < G; ++k) {
                const Regions w = slot(ws, Lws, Lmax, k);
                // zero staging input: the timing does not depend on the values
                (void)hipMemsetAsync(w.W1, 0, ws_region(Lmax, 1), st);
                mm.src[k] = (const float*)w.W1;
                mm.dst[k] = w.W0;   // f_lm (L^2 entries) fits in W0
                mm.L[k] = Lmax;
            }
            double t = 0;
            for (int rep = 0; rep < 3; ++rep) {
                (void)hipEventRecord(e0, st);
                hipError_t e = mw::launch_contract_forward_mix(*p, kv.first, mm, G, st);
                (void)hipEventRecord(e1, st);
                if (e != hipSuccess) { hipEventDestroy(e0); hipEventDestroy(e1); return fail(MW_EHIP, "autotune launch failed"); }
                (void)hipEventSynchronize(e1);
                float ms = 0;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (rep > 0) t += ms;
            }
            const double per_map = t / G;
            if (per_map < best_t * 0.97) { best_t = per_map; best = G; }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        g_tuned[key] = best;
    }
    return MW_OK;
}

}  // namespace

extern "C" {

int mw_forward(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
               void* const* ptrs, int32_t precision, void* stream)
{
    return run(Op::Forward, L, spin, reality, batch, ptrs, precision, stream);
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

int mw_workspace_size(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch,
                      int32_t precision, size_t* bytes)
{
    int rc = validate(L, spin, reality, batch, nullptr, precision, false);
    if (rc) return rc;
    if (!bytes) return fail(MW_EINVAL, "bytes must be non-NULL");
    int slots = 1;
    if (precision != MW_FP64) {   // one slot per map of the largest group, at most GMAX
        std::map<int, int> cnt;
        for (int b = 0; b < batch; ++b) slots = std::max(slots, std::min(++cnt[spin[b]], mw::GMAX));
    }
    *bytes = (size_t)slots * ws_need(batch_lmax(L, batch)) + 256;
    return MW_OK;
}

int mw_prepare(const int32_t* L, const int32_t* spin, const int32_t* reality, int32_t batch, int32_t precision)
{
    int rc = validate(L, spin, reality, batch, nullptr, precision, false);
    if (rc) return rc;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(MW_EHIP, "hipGetDevice failed");
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState& d = g_dev[dev];
    if (precision != MW_FP64 && (rc = autotune(d, L, spin, batch, nullptr))) return rc;
    const int Lws = batch_lmax(L, batch);
    const int slots = ws_slots(d, L, spin, batch, precision, true, rc);
    if (rc) return rc;
    void* ws = nullptr;
    if ((rc = get_ws(d, (size_t)slots * ws_need(Lws) + 256, true, &ws))) return rc;
    for (int b = 0; b < batch; ++b) {
        const Plan* p;
        const SpinTable* sp;
        const int as = spin[b] < 0 ? -spin[b] : spin[b];
        if ((rc = get_plan(d, L[b], true, &p))) return rc;
        if ((rc = get_spin(d, L[b], as, true, &sp))) return rc;
    }
    if (precision != MW_FP64) {   // the groups' spin tables at their largest band-limit
        for (const Group& g : make_groups(d, L, spin, batch, true, rc)) {
            const SpinTable* sp;
            if ((rc = get_spin(d, g.Lmax, g.s < 0 ? -g.s : g.s, true, &sp))) return rc;
        }
        if (rc) return rc;
    }
    if (hipDeviceSynchronize() != hipSuccess) return fail(MW_EHIP, "hipDeviceSynchronize failed");
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

const char* mw_profile_stage_name(int stage)
{
    static const char* names[MW_PROFILE_NSTAGE] = {
        "phi_forward", "theta_forward", "contract_forward", "contract_inverse", "theta_inverse",
        "phi_inverse", "contract_forward_adjoint", "contract_inverse_adjoint", "other"};
    return (stage >= 0 && stage < MW_PROFILE_NSTAGE) ? names[stage] : "";
}

}  // extern "C"
