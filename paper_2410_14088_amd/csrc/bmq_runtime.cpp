// Host runtime of the compressed stage loop: the C ABI of include/bmq.h,
// the planner (Algorithm 1, tile passes, gate fusion) and the device-arena
// layout.  All codec and simulation arithmetic runs in bmq_kernels.hip; this
// file only plans, lays out memory and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/bmq.h"
#include "bmq_internal.h"

using bmq::OpDesc;
using cd = std::complex<double>;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(SV_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

constexpr int kDefaultTile = 12;
constexpr int kMaxDiagQubits = bmq::kMaxDiagQubits;
constexpr size_t kMaxLaunchesPerBatch = 512;    // counter blocks of one batch of pass launches
constexpr size_t kStageCounters = (size_t)bmq::kSegments * bmq::C_NUM;   // words per launch
constexpr int kPartials = 1024;
constexpr uint64_t kOpsArenaBytes = 8ull << 20;    // fused matrices and diagonal tables of one plan
constexpr uint64_t kStageBytes = 4ull << 20;       // host-reference slices, sampling tables
constexpr int kMaxSampleGroups = 1 << 16;          // sampling: |psi|^2 per group, at most this many groups
constexpr uint64_t kSampleBatch = 1ull << 16;      // samples per sampling kernel
static_assert(kMaxSampleGroups * 8ull + kSampleBatch * 20ull <= kStageBytes, "sampling tables fit the staging area");

// ------------------------------------------------------------------ gates

struct GateRec {
    int kind, nq, q[2];
    double p[3];
    bool diag;
};

bool gate_is_diagonal(int kind)
{
    switch (kind) {
    case SV_GATE_Z: case SV_GATE_S: case SV_GATE_T: case SV_GATE_RZ:
    case SV_GATE_CZ: case SV_GATE_CP: case SV_GATE_RZZ: return true;
    default: return false;
    }
}

int gate_nq(int kind) { return kind >= SV_GATE_CX ? 2 : 1; }

// Gate matrix, row major, dimension 2^nq (1-qubit: 2x2 in u[0..3]).
void gate_unitary(const GateRec &g, cd *u)
{
    const double c = std::cos(g.p[0] / 2), s = std::sin(g.p[0] / 2);
    const cd I(0, 1);
    auto ph = [](double a) { return std::polar(1.0, a); };
    for (int i = 0; i < 16; ++i) u[i] = 0;
    const double r2 = 1.0 / std::sqrt(2.0);
    switch (g.kind) {
    case SV_GATE_H: u[0] = r2; u[1] = r2; u[2] = r2; u[3] = -r2; break;
    case SV_GATE_X: u[1] = 1; u[2] = 1; break;
    case SV_GATE_Y: u[1] = -I; u[2] = I; break;
    case SV_GATE_Z: u[0] = 1; u[3] = -1; break;
    case SV_GATE_S: u[0] = 1; u[3] = I; break;
    case SV_GATE_T: u[0] = 1; u[3] = ph(M_PI / 4); break;
    case SV_GATE_RX: u[0] = c; u[1] = -I * s; u[2] = -I * s; u[3] = c; break;
    case SV_GATE_RY: u[0] = c; u[1] = -s; u[2] = s; u[3] = c; break;
    case SV_GATE_RZ: u[0] = ph(-g.p[0] / 2); u[3] = ph(g.p[0] / 2); break;
    case SV_GATE_U3:
        u[0] = c; u[1] = -ph(g.p[2]) * s; u[2] = ph(g.p[1]) * s; u[3] = ph(g.p[1] + g.p[2]) * c; break;
    case SV_GATE_CX: u[0] = 1; u[5] = 1; u[11] = 1; u[14] = 1; break;
    case SV_GATE_CZ: u[0] = 1; u[5] = 1; u[10] = 1; u[15] = -1; break;
    case SV_GATE_CP: u[0] = 1; u[5] = 1; u[10] = 1; u[15] = ph(g.p[0]); break;
    case SV_GATE_RZZ:
        u[0] = ph(-g.p[0] / 2); u[5] = ph(g.p[0] / 2); u[10] = ph(g.p[0] / 2); u[15] = ph(-g.p[0] / 2); break;
    default: break;
    }
}

// index of the gate's own matrix for an operation index x over qubits Q
int gate_sub_index(const GateRec &g, const std::vector<int> &Q, uint32_t x)
{
    auto bit = [&](int qubit) {
        const int j = (int)(std::find(Q.begin(), Q.end(), qubit) - Q.begin());
        return (int)((x >> j) & 1u);
    };
    if (g.nq == 1) return bit(g.q[0]);
    return 2 * bit(g.q[0]) + bit(g.q[1]);
}

uint32_t gate_mask(const GateRec &g, const std::vector<int> &Q)
{
    uint32_t m = 0;
    for (int i = 0; i < g.nq; ++i)
        m |= 1u << (int)(std::find(Q.begin(), Q.end(), g.q[i]) - Q.begin());
    return m;
}

// ------------------------------------------------------------------ plan

struct FusedOp {
    int type;                    // bmq::OP_DENSE / OP_DIAG
    std::vector<int> qubits;     // ascending
    std::vector<size_t> gates;   // circuit gate indices, in order
};

struct PassPlan {
    std::vector<int> tileq;      // t qubits: 0..5, then the rest ascending
    int op_begin = 0, op_end = 0;
};

struct StagePlan {
    size_t g0 = 0, g1 = 0;
    std::vector<int> inner;
    std::vector<PassPlan> passes;
};

}  // namespace

struct sv_plan {
    sv_config_t cfg{};
    int t = kDefaultTile;
    std::vector<GateRec> gates;          // in plan order (input order unless SV_FLAG_COMMUTE)
    std::vector<uint32_t> order;         // plan position -> input gate index (kNoInput: a remapping swap)
    std::vector<int32_t> layout;         // logical qubit -> bit position at the end (identity unless SV_FLAG_REMAP)
    std::vector<StagePlan> stages;
    std::vector<OpDesc> ops;
    std::vector<float2> data;
    uint64_t uid = 0;
};

struct sv_state {
    sv_config_t cfg{};
    int n = 0, b = 0;
    hipStream_t stream = nullptr;
    uint8_t *arena = nullptr;
    uint64_t arena_bytes = 0;
    uint64_t *dir[2] = {nullptr, nullptr};
    uint8_t *pool[2] = {nullptr, nullptr};
    uint64_t pool_cap = 0;
    float *scr_re = nullptr, *scr_im = nullptr;   // NULL with SV_FLAG_NO_SCRATCH
    uint64_t scr_elems = 0;                       // amplitudes per scratch plane
    bool group_scratch = false;                   // planes hold one group (SV_FLAG_GROUP_SCRATCH)
    uint8_t *host[2] = {nullptr, nullptr};        // host pool halves (second memory level), device view
    uint8_t *host_h[2] = {nullptr, nullptr};      // the same halves, host view
    uint64_t host_cap = 0;                        // usable bytes per half
    uint64_t live_host = 0;                       // of live_bytes, those in the host pool
    unsigned long long *counters = nullptr;
    double *partials = nullptr;
    double *out5 = nullptr;
    uint8_t *ops_arena = nullptr;
    int cur = 0;
    uint64_t live_bytes = 0;
    uint64_t uploaded_uid = 0;
    float *dump_re = nullptr, *dump_im = nullptr;     // test hook (sv_debug_dump)
    float *dumpd_re = nullptr, *dumpd_im = nullptr;
    uint64_t dump_lo = 0, dump_n = 0;
    uint8_t *stage = nullptr;                         // kStageBytes of device staging
    bool poisoned = false;
    bool reset_pending = false;                 // live_bytes is in the init counters
    sv_graph *pending_graph = nullptr;          // replayed graph whose counters are unread
    std::vector<hipEvent_t> events;             // per-stage timing, created on demand
};

struct sv_graph {
    sv_state *sv = nullptr;
    const sv_plan *plan = nullptr;
    uint64_t plan_uid = 0;
    size_t first = 0, count = 0, launches = 0;
    int cur_begin = 0, cur_end = 0;
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    // a captured whole-circuit queue launch: its workspace (launch arguments,
    // queue and done-counters, caller-owned) and the abort flags in it
    bool persistent = false;
    uint8_t *ws = nullptr;
    std::vector<uint64_t> flag_offs;
    uint64_t limit_us = 0;
};

namespace {

int resolve_graph(sv_t *sv);
std::atomic<uint64_t> g_plan_uid{1};

int step_shift(float ebf);
bool step_ok(int domain, int s);

int validate_cfg(const sv_config_t *c)
{
    if (!c) return fail(SV_ERR_INVALID, "config is NULL");
    if (c->n_qubits < 10 || c->n_qubits > 40)
        return fail(SV_ERR_INVALID, "n_qubits %d outside [10, 40]", c->n_qubits);
    if (c->block_qubits < 6 || c->block_qubits > c->n_qubits)
        return fail(SV_ERR_INVALID, "block_qubits %d outside [6, n]", c->block_qubits);
    if (c->fuse_qubits < 1 || c->fuse_qubits > 5)
        return fail(SV_ERR_INVALID, "fuse_qubits %d outside [1, 5]", c->fuse_qubits);
    if (c->domain != SV_DOMAIN_LIN && c->domain != SV_DOMAIN_LOG && c->domain != SV_DOMAIN_RAW)
        return fail(SV_ERR_INVALID, "domain %d", c->domain);
    const int t = c->tile_qubits ? c->tile_qubits : kDefaultTile;
    if (t < 10 || t > bmq::kMaxTile || t > c->n_qubits)
        return fail(SV_ERR_INVALID, "tile_qubits %d outside [10, min(13, n)]", t);
    if (!(c->eb > 0) || !std::isfinite(c->eb) || !std::isfinite((float)c->eb) || (float)c->eb <= 0)
        return fail(SV_ERR_INVALID, "eb must be a positive finite float32");
    if (c->flags & ~(SV_FLAG_NO_SCRATCH | SV_FLAG_NO_MFMA | SV_FLAG_GATE_PER_STAGE | SV_FLAG_DIAGONAL_FREE |
                     SV_FLAG_COMMUTE | SV_FLAG_GROUP_SCRATCH | SV_FLAG_REMAP))
        return fail(SV_ERR_INVALID, "unknown flags 0x%x", c->flags);
    if (c->reserved) return fail(SV_ERR_INVALID, "reserved must be 0");
    if (c->domain != SV_DOMAIN_RAW && !step_ok(c->domain, step_shift((float)c->eb)))
        return fail(SV_ERR_INVALID, "eb %g outside the codec's range for this domain (LOG: 2^-23 <= eb < 1/2)", c->eb);
    return SV_OK;
}

int tile_of(const sv_config_t *c) { return c->tile_qubits ? c->tile_qubits : kDefaultTile; }

// Quantization step delta = 2^-s: the largest power of two <= 2 eb (eb
// rounded to float32), so that scaling by 2^s is exact.
int step_shift(float ebf)
{
    int ex;
    (void)std::frexp(2.0f * ebf, &ex);   // 2 eb = m 2^ex, m in [1/2, 1)
    return 1 - ex;
}

bool step_ok(int domain, int s)
{
    return domain == SV_DOMAIN_LOG ? (s >= 1 && s <= 22) : (s >= -100 && s <= 100);
}

bmq::CodecParams codec_params(const sv_config_t &c)
{
    bmq::CodecParams cp;
    cp.domain = c.domain;
    cp.ebf = (float)c.eb;
    cp.s = step_shift(cp.ebf);
    cp.code_ok = c.domain != SV_DOMAIN_RAW && step_ok(c.domain, cp.s) ? 1 : 0;   // RAW: every chunk verbatim
    const int s = cp.code_ok ? cp.s : 0;
    cp.s = s;
    cp.delta = std::ldexp(1.0f, -s);
    cp.scale = std::ldexp(1.0f, s);
    return cp;
}

// Algorithm 1: greedy in gate order, close the stage when its global indices
// would exceed threshold = max(inner, 2).  Never emits an empty stage.  With
// per_gate every gate closes its own stage (the per-gate workflow of Section
// 3, for comparison); with diag_free a diagonal gate adds no global index
// (it pairs no blocks, so it runs inside any group).
int partition(const std::vector<GateRec> &gates, int b, int inner, bool per_gate, bool diag_free,
              std::vector<StagePlan> &out)
{
    const int threshold = std::max(inner, 2);
    size_t start = 0;
    std::vector<int> cur;
    for (size_t i = 0; i < gates.size(); ++i) {
        std::vector<int> gq;
        for (int j = 0; j < gates[i].nq; ++j)
            if (gates[i].q[j] >= b && !(diag_free && gates[i].diag)) gq.push_back(gates[i].q[j]);
        if ((int)gq.size() > threshold)
            return fail(SV_ERR_INVALID, "gate %zu touches %zu global qubits > threshold %d", i, gq.size(), threshold);
        std::vector<int> uni = cur;
        for (int q : gq)
            if (std::find(uni.begin(), uni.end(), q) == uni.end()) uni.push_back(q);
        if ((int)uni.size() > threshold || per_gate) {
            if (i > start) {
                StagePlan s;
                s.g0 = start;
                s.g1 = i;
                s.inner = cur;
                std::sort(s.inner.begin(), s.inner.end());
                out.push_back(s);
            }
            start = i;
            uni = gq;
        }
        cur = uni;
    }
    if (gates.size() > start) {
        StagePlan s;
        s.g0 = start;
        s.g1 = gates.size();
        s.inner = cur;
        std::sort(s.inner.begin(), s.inner.end());
        out.push_back(s);
    }
    return SV_OK;
}

// Algorithm 1 with commutation: each stage takes, in input order, every
// remaining gate that fits the threshold and commutes with every remaining
// gate it would overtake (the ones deferred before it in this sweep); the
// deferred gates form the next sweep.  Two gates commute here when their
// qubits are disjoint or both are diagonal, so the reordered circuit has the
// same unitary.  Commutation is tracked per qubit: a diagonal gate is blocked
// by a deferred non-diagonal gate on one of its qubits, any other gate by any
// deferred gate on one of its qubits.  gates is permuted into plan order,
// order receives plan position -> input index.
int partition_commute(std::vector<GateRec> &gates, int b, int inner, bool diag_free, std::vector<StagePlan> &out,
                      std::vector<uint32_t> &order)
{
    const int threshold = std::max(inner, 2);
    auto globals_of = [&](const GateRec &g) {
        std::vector<int> gq;
        for (int j = 0; j < g.nq; ++j)
            if (g.q[j] >= b && !(diag_free && g.diag)) gq.push_back(g.q[j]);
        return gq;
    };
    for (size_t i = 0; i < gates.size(); ++i)
        if ((int)globals_of(gates[i]).size() > threshold)
            return fail(SV_ERR_INVALID, "gate %zu touches more than threshold %d global qubits", i, threshold);
    std::vector<uint32_t> remaining(gates.size());
    for (size_t i = 0; i < gates.size(); ++i) remaining[i] = (uint32_t)i;
    std::vector<GateRec> planned;
    order.clear();
    std::vector<uint8_t> blocked_any(64), blocked_nondiag(64);
    while (!remaining.empty()) {
        std::fill(blocked_any.begin(), blocked_any.end(), 0);
        std::fill(blocked_nondiag.begin(), blocked_nondiag.end(), 0);
        std::vector<uint32_t> deferred;
        std::vector<int> cur;
        StagePlan s;
        s.g0 = planned.size();
        for (uint32_t i : remaining) {
            const GateRec &g = gates[i];
            bool ok = true;
            for (int j = 0; j < g.nq && ok; ++j)
                ok = g.diag ? !blocked_nondiag[g.q[j]] : !blocked_any[g.q[j]];
            std::vector<int> uni = cur;
            if (ok) {
                for (int q : globals_of(g))
                    if (std::find(uni.begin(), uni.end(), q) == uni.end()) uni.push_back(q);
                ok = (int)uni.size() <= threshold;
            }
            if (ok) {
                planned.push_back(g);
                order.push_back(i);
                cur = uni;
            } else {
                deferred.push_back(i);
                for (int j = 0; j < g.nq; ++j) {
                    blocked_any[g.q[j]] = 1;
                    if (!g.diag) blocked_nondiag[g.q[j]] = 1;
                }
            }
        }
        s.g1 = planned.size();
        s.inner = cur;
        std::sort(s.inner.begin(), s.inner.end());
        out.push_back(s);
        remaining.swap(deferred);
    }
    gates.swap(planned);
    return SV_OK;
}

constexpr uint32_t kNoInput = 0xFFFFFFFFu;

// Algorithm 1 with qubit remapping.  Logical qubit L sits at bit position
// phys[L] (identity at the start); a gate acts on its qubits' positions and
// Algorithm 1 counts the global positions (>= b).  When the next gate would
// exceed the threshold, before the stage is closed, each inner position pg
// of the stage, ascending, whose logical qubit is used again is offered a
// swap: the local position whose logical qubit is next used last (ties: the
// lowest) is taken when that use comes strictly later, and the stage ends
// with SWAP(l, pg) = CX(l, pg) CX(pg, l) CX(l, pg) -- both positions are in
// the stage already, so no global index is added.  Later gates map through
// the new positions.  gates becomes the physical circuit; order receives its
// input indices (kNoInput for swap gates), layout the final positions.
int partition_remap(std::vector<GateRec> &gates, int n, int b, int inner, bool diag_free, std::vector<StagePlan> &out,
                    std::vector<uint32_t> &order, std::vector<int32_t> &layout)
{
    const int threshold = std::max(inner, 2);
    const uint64_t never = 1ull << 62;
    std::vector<int> log_at(n), phys(n);
    for (int q = 0; q < n; ++q) log_at[q] = phys[q] = q;
    std::vector<std::vector<uint32_t>> uses(n);
    for (size_t i = 0; i < gates.size(); ++i)
        for (int j = 0; j < gates[i].nq; ++j) uses[gates[i].q[j]].push_back((uint32_t)i);
    std::vector<size_t> ptr(n, 0);
    auto next_use = [&](int L, size_t i) -> uint64_t {
        while (ptr[L] < uses[L].size() && uses[L][ptr[L]] < i) ++ptr[L];
        return ptr[L] < uses[L].size() ? uses[L][ptr[L]] : never;
    };
    auto globals_of = [&](const GateRec &g) {
        std::vector<int> gq;
        for (int j = 0; j < g.nq; ++j)
            if (phys[g.q[j]] >= b && !(diag_free && g.diag)) gq.push_back(phys[g.q[j]]);
        return gq;
    };
    std::vector<GateRec> res;
    order.clear();
    size_t start = 0;
    std::vector<int> cur;
    auto close = [&](size_t end) {
        StagePlan s;
        s.g0 = start;
        s.g1 = end;
        s.inner = cur;
        std::sort(s.inner.begin(), s.inner.end());
        out.push_back(s);
        start = end;
        cur.clear();
    };
    for (size_t i = 0; i < gates.size(); ++i) {
        std::vector<int> gq = globals_of(gates[i]);
        if ((int)gq.size() > threshold)
            return fail(SV_ERR_INVALID, "gate %zu touches %zu global qubits > threshold %d", i, gq.size(), threshold);
        std::vector<int> uni = cur;
        for (int q : gq)
            if (std::find(uni.begin(), uni.end(), q) == uni.end()) uni.push_back(q);
        if ((int)uni.size() > threshold && res.size() > start) {
            std::vector<int> inner_now = cur;
            std::sort(inner_now.begin(), inner_now.end());
            for (int pg : inner_now) {
                uint64_t best_nu = next_use(log_at[pg], i);
                if (best_nu == never) continue;
                int best = -1;
                for (int l = 0; l < b; ++l) {
                    const uint64_t v = next_use(log_at[l], i);
                    if (v > best_nu) {
                        best = l;
                        best_nu = v;
                    }
                }
                if (best < 0) continue;
                const int pairs[3][2] = {{best, pg}, {pg, best}, {best, pg}};
                for (const auto &pr : pairs) {
                    GateRec cx;
                    cx.kind = SV_GATE_CX;
                    cx.nq = 2;
                    cx.q[0] = pr[0];
                    cx.q[1] = pr[1];
                    cx.p[0] = cx.p[1] = cx.p[2] = 0.0;
                    cx.diag = false;
                    res.push_back(cx);
                    order.push_back(kNoInput);
                }
                const int la = log_at[best], lg = log_at[pg];
                log_at[best] = lg;
                log_at[pg] = la;
                phys[lg] = best;
                phys[la] = pg;
            }
            close(res.size());
            gq = globals_of(gates[i]);
            uni = gq;
        }
        cur = uni;
        GateRec r = gates[i];
        for (int j = 0; j < r.nq; ++j) r.q[j] = phys[gates[i].q[j]];
        res.push_back(r);
        order.push_back((uint32_t)i);
    }
    if (res.size() > start) close(res.size());
    gates.swap(res);
    layout.assign(phys.begin(), phys.end());
    return SV_OK;
}

// Cut a stage into on-chip passes: every qubit >= 6 that a non-diagonal gate
// acts on must be one of the pass's t-6 free tile qubits.  Greedy, in order.
bool plan_passes(sv_plan &P, StagePlan &st)
{
    const int n = P.cfg.n_qubits, b = P.cfg.block_qubits, t = P.t;
    const int free_slots = t - 6;
    std::vector<std::vector<size_t>> pass_gates;
    std::vector<std::vector<int>> pass_need;
    std::vector<size_t> cur;
    std::vector<int> need;
    for (size_t g = st.g0; g < st.g1; ++g) {
        const GateRec &gr = P.gates[g];
        std::vector<int> add = need;
        if (!gr.diag)
            for (int j = 0; j < gr.nq; ++j)
                if (gr.q[j] >= 6 && std::find(add.begin(), add.end(), gr.q[j]) == add.end()) add.push_back(gr.q[j]);
        if ((int)add.size() > free_slots && !cur.empty()) {
            pass_gates.push_back(cur);
            pass_need.push_back(need);
            cur.clear();
            add.clear();
            if (!gr.diag)
                for (int j = 0; j < gr.nq; ++j)
                    if (gr.q[j] >= 6 && std::find(add.begin(), add.end(), gr.q[j]) == add.end()) add.push_back(gr.q[j]);
        }
        need = add;
        cur.push_back(g);
    }
    pass_gates.push_back(cur);
    pass_need.push_back(need);

    for (size_t pi = 0; pi < pass_gates.size(); ++pi) {
        // tile qubits: 0..5, the needed ones, then fill with local qubits,
        // the stage's inner qubits and finally any other qubit, ascending
        std::vector<int> tq = pass_need[pi];
        auto has = [&](int q) { return q < 6 || std::find(tq.begin(), tq.end(), q) != tq.end(); };
        for (int q = 6; q < b && (int)tq.size() < free_slots; ++q)
            if (!has(q)) tq.push_back(q);
        for (int q : st.inner)
            if ((int)tq.size() < free_slots && !has(q)) tq.push_back(q);
        for (int q = 6; q < n && (int)tq.size() < free_slots; ++q)
            if (!has(q)) tq.push_back(q);
        std::sort(tq.begin(), tq.end());
        PassPlan pp;
        for (int q = 0; q < 6; ++q) pp.tileq.push_back(q);
        for (int q : tq) pp.tileq.push_back(q);
        auto in_tile = [&](int q) { return std::find(pp.tileq.begin(), pp.tileq.end(), q) != pp.tileq.end(); };

        // fusion with deferred diagonals.  Diagonal gates commute with each
        // other and with any gate on other qubits, so a diagonal gate that does
        // not fit the dense operation being built waits in a pending set that
        // is applied after that operation.  A later non-diagonal gate takes the
        // pending gates that share a qubit with it (they must act before it)
        // into its own dense operation when they fit there, else they go out
        // first as one diagonal operation; the other pending gates keep
        // waiting.  Every gate thus moves only past gates it commutes with,
        // and the ladders of several controlled phases share one diagonal
        // operation instead of one each.
        const int K = P.cfg.fuse_qubits;
        std::vector<FusedOp> fused;
        FusedOp cur{-1, {}, {}};                       // dense operation being built
        std::vector<size_t> pend;                      // deferred diagonal gates, in order
        auto add_qubits = [&](std::vector<int> &qs, size_t g) {
            const GateRec &r = P.gates[g];
            for (int j = 0; j < r.nq; ++j)
                if (std::find(qs.begin(), qs.end(), r.q[j]) == qs.end()) qs.push_back(r.q[j]);
        };
        auto qubits_of = [&](const std::vector<size_t> &gs) {
            std::vector<int> qs;
            for (size_t g : gs) add_qubits(qs, g);
            std::sort(qs.begin(), qs.end());
            return qs;
        };
        auto emit_cur = [&]() {
            if (cur.type >= 0) fused.push_back(cur);
            cur = FusedOp{-1, {}, {}};
        };
        auto emit_diag = [&](const std::vector<size_t> &gs) {
            if (!gs.empty()) fused.push_back(FusedOp{bmq::OP_DIAG, qubits_of(gs), gs});
        };
        for (size_t g : pass_gates[pi]) {
            const GateRec &gr = P.gates[g];
            if (gr.diag) {
                bool subset = cur.type >= 0;
                for (int j = 0; j < gr.nq && subset; ++j)
                    subset = std::find(cur.qubits.begin(), cur.qubits.end(), gr.q[j]) != cur.qubits.end();
                if (subset) { cur.gates.push_back(g); continue; }
                std::vector<size_t> trial = pend;
                trial.push_back(g);
                if ((int)qubits_of(trial).size() <= kMaxDiagQubits) { pend.swap(trial); continue; }
                emit_cur();
                emit_diag(pend);
                pend.assign(1, g);
                continue;
            }
            std::vector<size_t> before, rest;
            for (size_t d : pend) {
                const GateRec &dr = P.gates[d];
                bool shares = false;
                for (int a = 0; a < dr.nq; ++a)
                    for (int c = 0; c < gr.nq; ++c) shares = shares || dr.q[a] == gr.q[c];
                (shares ? before : rest).push_back(d);
            }
            const std::vector<int> bq = qubits_of(before);
            bool before_in_tile = true;
            for (int q : bq) before_in_tile = before_in_tile && in_tile(q);
            std::vector<int> need = bq;
            add_qubits(need, g);
            if (cur.type >= 0) {
                std::vector<int> grown = need;
                for (int q : cur.qubits)
                    if (std::find(grown.begin(), grown.end(), q) == grown.end()) grown.push_back(q);
                if (before_in_tile && (int)grown.size() <= K) {
                    std::sort(grown.begin(), grown.end());
                    cur.qubits = grown;
                    cur.gates.insert(cur.gates.end(), before.begin(), before.end());
                    cur.gates.push_back(g);
                    pend.swap(rest);
                    continue;
                }
            }
            emit_cur();
            std::sort(need.begin(), need.end());
            if (before_in_tile && (int)need.size() <= K) {
                cur = FusedOp{bmq::OP_DENSE, need, before};
                cur.gates.push_back(g);
            } else {
                emit_diag(before);
                cur = FusedOp{bmq::OP_DENSE, {}, {g}};
                add_qubits(cur.qubits, g);
                std::sort(cur.qubits.begin(), cur.qubits.end());
            }
            pend.swap(rest);
        }
        emit_cur();
        emit_diag(pend);

        pp.op_begin = (int)P.ops.size();
        for (const FusedOp &f : fused) {
            OpDesc d;
            std::memset(&d, 0, sizeof(d));
            d.type = f.type;
            d.k = (int)f.qubits.size();
            for (int j = 0; j < d.k; ++j) {
                d.gq[j] = f.qubits[j];
                const auto it = std::find(pp.tileq.begin(), pp.tileq.end(), f.qubits[j]);
                d.pos[j] = it == pp.tileq.end() ? -1 : (int)(it - pp.tileq.begin());
            }
            d.data = (uint32_t)P.data.size();
            const uint32_t D = 1u << d.k;
            if (f.type == bmq::OP_DENSE)
                for (int j = 0; j < d.k; ++j)
                    if (d.pos[j] < 0) return false;   // a dense operation must lie inside the tile
            if (f.type == bmq::OP_DIAG) {
                std::vector<cd> tab(D, cd(1, 0));
                for (size_t g : f.gates) {
                    cd u[16];
                    gate_unitary(P.gates[g], u);
                    const int dim = 1 << P.gates[g].nq;
                    for (uint32_t x = 0; x < D; ++x) {
                        const int s = gate_sub_index(P.gates[g], f.qubits, x);
                        tab[x] *= u[s * dim + s];
                    }
                }
                for (uint32_t x = 0; x < D; ++x) P.data.push_back(make_float2((float)tab[x].real(), (float)tab[x].imag()));
            } else {
                std::vector<cd> M(D * D, cd(0, 0));
                for (uint32_t x = 0; x < D; ++x) M[x * D + x] = 1;
                for (size_t g : f.gates) {
                    cd u[16];
                    gate_unitary(P.gates[g], u);
                    const int dim = 1 << P.gates[g].nq;
                    const uint32_t gm = gate_mask(P.gates[g], f.qubits);
                    std::vector<cd> E(D * D, cd(0, 0));
                    for (uint32_t r = 0; r < D; ++r)
                        for (uint32_t c = 0; c < D; ++c)
                            if ((r & ~gm) == (c & ~gm))
                                E[r * D + c] = u[gate_sub_index(P.gates[g], f.qubits, r) * dim +
                                                 gate_sub_index(P.gates[g], f.qubits, c)];
                    std::vector<cd> R(D * D, cd(0, 0));
                    for (uint32_t r = 0; r < D; ++r)
                        for (uint32_t k = 0; k < D; ++k) {
                            const cd e = E[r * D + k];
                            if (e == cd(0, 0)) continue;
                            for (uint32_t c = 0; c < D; ++c) R[r * D + c] += e * M[k * D + c];
                        }
                    M.swap(R);
                }
                for (uint32_t x = 0; x < D * D; ++x) P.data.push_back(make_float2((float)M[x].real(), (float)M[x].imag()));
            }
            P.ops.push_back(d);
        }
        pp.op_end = (int)P.ops.size();
        st.passes.push_back(pp);
    }
    return true;
}

// log2 of the amplitudes one scratch plane holds: the whole state, or with
// SV_FLAG_GROUP_SCRATCH one SV group of the largest multi-pass stage the
// configuration plans (block qubits + threshold, at least a tile)
int scratch_qubits(const sv_config_t &c)
{
    if (!(c.flags & SV_FLAG_GROUP_SCRATCH)) return c.n_qubits;
    const int t = c.tile_qubits ? c.tile_qubits : kDefaultTile;
    return std::min(c.n_qubits, std::max(c.block_qubits + std::max(c.inner_size, 2), t));
}

struct ArenaLayout {
    uint64_t dir_bytes, pool_cap, scr_elems, scr_bytes, counters_bytes, partials_bytes, ops_bytes, total;
    uint64_t off_dir0, off_dir1, off_pool0, off_pool1, off_scr_re, off_scr_im, off_counters,
        off_partials, off_out5, off_ops, off_stage;
};

uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

ArenaLayout layout_for(const sv_config_t &c)
{
    ArenaLayout L{};
    const uint64_t nch = 1ull << (c.n_qubits - 6);
    L.dir_bytes = align256(nch * 8);
    const uint64_t worst = nch * bmq::kMaxBodyBytes + bmq::kSegments * 256ull;
    L.pool_cap = c.pool_bytes ? c.pool_bytes : worst;
    const uint64_t pool_alloc = align256(L.pool_cap + 1024);    // decoders read a little past a body
    L.scr_elems = (c.flags & SV_FLAG_NO_SCRATCH) ? 0 : 1ull << scratch_qubits(c);
    L.scr_bytes = align256(L.scr_elems * 4ull);
    L.counters_bytes = align256((kMaxLaunchesPerBatch + 1) * kStageCounters * 8ull);
    L.partials_bytes = align256(kPartials * 5 * 8ull);
    L.ops_bytes = kOpsArenaBytes;
    uint64_t o = 0;
    L.off_dir0 = o; o += L.dir_bytes;
    L.off_dir1 = o; o += L.dir_bytes;
    L.off_pool0 = o; o += pool_alloc;
    L.off_pool1 = o; o += pool_alloc;
    L.off_scr_re = o; o += L.scr_bytes;
    L.off_scr_im = o; o += L.scr_bytes;
    L.off_counters = o; o += L.counters_bytes;
    L.off_partials = o; o += L.partials_bytes;
    L.off_out5 = o; o += 256;
    L.off_ops = o; o += L.ops_bytes;
    L.off_stage = o; o += kStageBytes;
    L.total = o;
    return L;
}

// body bytes of one plane from its 12-bit header (stream format parse)
uint32_t body_bytes_host(uint32_t hdr)
{
    const uint32_t mode = hdr & 3u, w = (hdr >> 2) & 63u, sc = (hdr >> 8) & 3u, zc = (hdr >> 10) & 3u;
    if (mode == 0) return 0;
    if (mode == 3) return 256;
    return (mode == 1 ? 4u : 0u) + 8u * ((sc == 2u) + (zc == 2u)) + 8u * w;
}

bmq::PoolView pool_view(const sv_t *sv, int which)
{
    return bmq::PoolView{sv->pool[which], sv->host[which], sv->pool_cap};
}

int check_state(const sv_t *sv)
{
    if (!sv) return fail(SV_ERR_INVALID, "state is NULL");
    if (sv->poisoned) return fail(SV_ERR_CAPACITY, "state is poisoned by an earlier overflow, aborted launch or bad directory");
    return SV_OK;
}

}  // namespace

namespace {
// the 7 stage features of the block predictor (features 25..31): gate
// counts of the stage, distinct local qubits, fused operations, position in
// the plan, log2 of the error bound
bmq::StageFeats stage_feats(const sv_plan_t *p, size_t stage)
{
    const StagePlan &st = p->stages[stage];
    const int b = p->cfg.block_qubits;
    int nondiag = 0, diag = 0, global = 0;
    uint64_t local_mask = 0;
    for (size_t g = st.g0; g < st.g1; ++g) {
        const GateRec &gr = p->gates[g];
        (gr.diag ? diag : nondiag)++;
        bool touches_global = false;
        for (int i = 0; i < gr.nq; ++i) {
            if (gr.q[i] >= b) touches_global = true;
            else local_mask |= 1ull << gr.q[i];
        }
        global += touches_global;
    }
    int nops = 0;
    for (const auto &pp : st.passes) nops += pp.op_end - pp.op_begin;
    bmq::StageFeats sf;
    sf.v[0] = (float)(nondiag / 64.0);
    sf.v[1] = (float)(diag / 64.0);
    sf.v[2] = (float)(global / 64.0);
    sf.v[3] = (float)((double)__builtin_popcountll(local_mask) / b);
    sf.v[4] = (float)(nops / 16.0);
    sf.v[5] = (float)((double)stage / (double)p->stages.size());
    sf.v[6] = (float)(std::log2(p->cfg.eb) / 32.0);
    return sf;
}

// work space of mlp_predict_bytes: a two-block directory, one record, init
// counters, the block features, the outputs and the per-stage totals
struct PredictWork {
    uint64_t off_dir, off_pool, off_cnt, off_x, off_out, off_tot, total;
};
PredictWork predict_work(const sv_config_t &c, size_t n_stages)
{
    const uint64_t cpb = 1ull << (c.block_qubits - 6), nb = 1ull << (c.n_qubits - c.block_qubits);
    PredictWork w{};
    uint64_t o = 0;
    w.off_dir = o; o += align256(2 * cpb * 8);
    w.off_pool = o; o += 1024;
    w.off_cnt = o; o += align256(bmq::C_NUM * 8);
    w.off_x = o; o += align256(nb * SV_MLP_IN * 4);
    w.off_out = o; o += align256(nb * SV_MLP_OUT * 4);
    w.off_tot = o; o += align256((n_stages + 1) * 8);
    w.total = o;
    return w;
}
}  // namespace

// ====================================================================== ABI

extern "C" {

const char *sv_last_error(void) { return g_err.c_str(); }

int stage_plan(const sv_gate_t *gates, size_t n_gates, const sv_config_t *cfg, sv_plan_t **out)
{
    if (!out) return fail(SV_ERR_INVALID, "out is NULL");
    if (int rc = validate_cfg(cfg)) return rc;
    if (n_gates && !gates) return fail(SV_ERR_INVALID, "gates is NULL");
    sv_plan *P = new (std::nothrow) sv_plan;
    if (!P) return fail(SV_ERR_OOM, "host allocation failed");
    P->cfg = *cfg;
    P->t = tile_of(cfg);
    const int n = cfg->n_qubits;
    for (size_t i = 0; i < n_gates; ++i) {
        const sv_gate_t &g = gates[i];
        if (g.kind < 0 || g.kind >= SV_GATE_COUNT) { delete P; return fail(SV_ERR_INVALID, "gate %zu: bad kind %d", i, g.kind); }
        GateRec r;
        r.kind = g.kind;
        r.nq = gate_nq(g.kind);
        r.q[0] = g.q[0];
        r.q[1] = r.nq == 2 ? g.q[1] : -1;
        for (int j = 0; j < 3; ++j) r.p[j] = g.p[j];
        r.diag = gate_is_diagonal(g.kind);
        for (int j = 0; j < r.nq; ++j)
            if (r.q[j] < 0 || r.q[j] >= n) { delete P; return fail(SV_ERR_INVALID, "gate %zu: qubit %d out of range", i, r.q[j]); }
        if (r.nq == 2 && r.q[0] == r.q[1]) { delete P; return fail(SV_ERR_INVALID, "gate %zu: repeated qubit", i); }
        P->gates.push_back(r);
    }
    const bool per_gate = (cfg->flags & SV_FLAG_GATE_PER_STAGE) != 0;
    const bool diag_free = (cfg->flags & SV_FLAG_DIAGONAL_FREE) != 0;
    int prc;
    const bool remap = (cfg->flags & SV_FLAG_REMAP) != 0;
    if (remap && (per_gate || (cfg->flags & SV_FLAG_COMMUTE))) {
        delete P;
        return fail(SV_ERR_INVALID, "SV_FLAG_REMAP combines with neither SV_FLAG_GATE_PER_STAGE nor SV_FLAG_COMMUTE");
    }
    if (remap) {
        prc = partition_remap(P->gates, n, cfg->block_qubits, cfg->inner_size, diag_free, P->stages, P->order,
                              P->layout);
    } else if ((cfg->flags & SV_FLAG_COMMUTE) && !per_gate) {
        prc = partition_commute(P->gates, cfg->block_qubits, cfg->inner_size, diag_free, P->stages, P->order);
    } else {
        prc = partition(P->gates, cfg->block_qubits, cfg->inner_size, per_gate, diag_free, P->stages);
        P->order.resize(P->gates.size());
        for (size_t i = 0; i < P->order.size(); ++i) P->order[i] = (uint32_t)i;
    }
    if (prc) { delete P; return prc; }
    if (P->layout.empty())
        for (int q = 0; q < n; ++q) P->layout.push_back(q);
    for (StagePlan &st : P->stages)
        if (!plan_passes(*P, st)) { delete P; return fail(SV_ERR_INVALID, "internal: dense operation outside its tile"); }
    if ((uint64_t)P->ops.size() * sizeof(OpDesc) + P->data.size() * sizeof(float2) + 256 > kOpsArenaBytes) {
        delete P;
        return fail(SV_ERR_UNSUPPORTED, "plan too large for the operation arena");
    }
    P->uid = g_plan_uid.fetch_add(1);
    *out = P;
    return SV_OK;
}

int plan_info(const sv_plan_t *p, size_t *n_stages, size_t *n_ops, size_t *n_passes)
{
    if (!p) return fail(SV_ERR_INVALID, "plan is NULL");
    if (n_stages) *n_stages = p->stages.size();
    if (n_ops) *n_ops = p->ops.size();
    if (n_passes) {
        size_t np = 0;
        for (const auto &s : p->stages) np += s.passes.size();
        *n_passes = np;
    }
    return SV_OK;
}

int plan_stage_ops(const sv_plan_t *p, size_t s, size_t *op_begin, size_t *op_end)
{
    if (!p) return fail(SV_ERR_INVALID, "plan is NULL");
    if (s >= p->stages.size()) return fail(SV_ERR_INVALID, "stage %zu out of range", s);
    const StagePlan &st = p->stages[s];
    if (op_begin) *op_begin = st.passes.empty() ? 0 : (size_t)st.passes.front().op_begin;
    if (op_end) *op_end = st.passes.empty() ? 0 : (size_t)st.passes.back().op_end;
    return SV_OK;
}

int plan_op(const sv_plan_t *p, size_t i, int32_t *type, int32_t *k, int32_t *qubits, void *data_host,
            size_t cap_elems)
{
    if (!p) return fail(SV_ERR_INVALID, "plan is NULL");
    if (i >= p->ops.size()) return fail(SV_ERR_INVALID, "operation %zu out of range", i);
    const OpDesc &d = p->ops[i];
    const size_t D = (size_t)1 << d.k, n = d.type == bmq::OP_DENSE ? D * D : D;
    if (type) *type = d.type;
    if (k) *k = d.k;
    if (qubits)
        for (int j = 0; j < d.k; ++j) qubits[j] = d.gq[j];
    if (data_host) {
        if (cap_elems < n) return fail(SV_ERR_INVALID, "operation %zu has %zu complex64 values", i, n);
        std::memcpy(data_host, p->data.data() + d.data, n * sizeof(float2));
    }
    return SV_OK;
}

int plan_gate_order(const sv_plan_t *p, uint32_t *order_out, size_t n)
{
    if (!p) return fail(SV_ERR_INVALID, "plan is NULL");
    if (n != p->order.size()) return fail(SV_ERR_INVALID, "order array of %zu entries for %zu gates", n, p->order.size());
    if (n && !order_out) return fail(SV_ERR_INVALID, "order_out is NULL");
    std::copy(p->order.begin(), p->order.end(), order_out);
    return SV_OK;
}

int plan_layout(const sv_plan_t *p, int32_t *phys_of_logical, size_t n)
{
    if (!p || !phys_of_logical) return fail(SV_ERR_INVALID, "plan or output is NULL");
    if (n != p->layout.size()) return fail(SV_ERR_INVALID, "layout array of %zu entries for %zu qubits", n, p->layout.size());
    std::copy(p->layout.begin(), p->layout.end(), phys_of_logical);
    return SV_OK;
}

int plan_gate(const sv_plan_t *p, size_t k, int32_t *kind, int32_t *qubits, double *params)
{
    if (!p) return fail(SV_ERR_INVALID, "plan is NULL");
    if (k >= p->gates.size()) return fail(SV_ERR_INVALID, "gate %zu outside the plan's %zu gates", k, p->gates.size());
    const GateRec &g = p->gates[k];
    if (kind) *kind = g.kind;
    if (qubits) {
        qubits[0] = g.q[0];
        qubits[1] = g.nq == 2 ? g.q[1] : -1;
    }
    if (params)
        for (int j = 0; j < 3; ++j) params[j] = g.p[j];
    return SV_OK;
}

int plan_stage(const sv_plan_t *p, size_t s, size_t *gate_begin, size_t *gate_end,
               int32_t *inner_out, int32_t *n_inner, int32_t *n_passes)
{
    if (!p) return fail(SV_ERR_INVALID, "plan is NULL");
    if (s >= p->stages.size()) return fail(SV_ERR_INVALID, "stage %zu out of range", s);
    const StagePlan &st = p->stages[s];
    if (gate_begin) *gate_begin = st.g0;
    if (gate_end) *gate_end = st.g1;
    if (n_inner) *n_inner = (int32_t)st.inner.size();
    if (inner_out)
        for (size_t i = 0; i < st.inner.size() && i < 8; ++i) inner_out[i] = st.inner[i];
    if (n_passes) *n_passes = (int32_t)st.passes.size();
    return SV_OK;
}

void plan_destroy(sv_plan_t *p) { delete p; }

int sv_mem_required(const sv_config_t *cfg, uint64_t *bytes)
{
    if (int rc = validate_cfg(cfg)) return rc;
    if (!bytes) return fail(SV_ERR_INVALID, "bytes is NULL");
    *bytes = layout_for(*cfg).total;
    return SV_OK;
}

int sv_create(const sv_config_t *cfg, void *dev_arena, uint64_t dev_bytes, void *hip_stream, sv_t **out)
{
    if (int rc = validate_cfg(cfg)) return rc;
    if (!out) return fail(SV_ERR_INVALID, "out is NULL");
    if (!dev_arena || ((uintptr_t)dev_arena & 255u)) return fail(SV_ERR_INVALID, "arena must be non-NULL and 256-byte aligned");
    const ArenaLayout L = layout_for(*cfg);
    if (dev_bytes < L.total)
        return fail(SV_ERR_OOM, "arena of %llu bytes < %llu required", (unsigned long long)dev_bytes,
                    (unsigned long long)L.total);
    sv_state *S = new (std::nothrow) sv_state;
    if (!S) return fail(SV_ERR_OOM, "host allocation failed");
    S->cfg = *cfg;
    S->n = cfg->n_qubits;
    S->b = cfg->block_qubits;
    S->stream = (hipStream_t)hip_stream;
    S->arena = (uint8_t *)dev_arena;
    S->arena_bytes = dev_bytes;
    S->dir[0] = (uint64_t *)(S->arena + L.off_dir0);
    S->dir[1] = (uint64_t *)(S->arena + L.off_dir1);
    S->pool[0] = S->arena + L.off_pool0;
    S->pool[1] = S->arena + L.off_pool1;
    S->pool_cap = L.pool_cap;
    if (L.scr_elems) {
        S->scr_re = (float *)(S->arena + L.off_scr_re);
        S->scr_im = (float *)(S->arena + L.off_scr_im);
        S->scr_elems = L.scr_elems;
        S->group_scratch = L.scr_elems < (1ull << S->n);
    }
    S->counters = (unsigned long long *)(S->arena + L.off_counters);
    S->partials = (double *)(S->arena + L.off_partials);
    S->out5 = (double *)(S->arena + L.off_out5);
    S->ops_arena = S->arena + L.off_ops;
    S->stage = S->arena + L.off_stage;
    S->cur = 0;
    const uint64_t nch = 1ull << (S->n - 6);
    unsigned long long *ic = S->counters + kMaxLaunchesPerBatch * kStageCounters;
    hipError_t e = bmq::launch_fill_u64((uint64_t *)ic, kStageCounters, 0, S->stream);
    if (e == hipSuccess) e = bmq::launch_init_state(S->dir[0], nch, S->pool[0], ic, codec_params(*cfg), S->stream);
    unsigned long long cursor = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&cursor, ic + bmq::C_CURSOR, 8, hipMemcpyDeviceToHost, S->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) {
        delete S;
        return fail(SV_ERR_HIP, "sv_create: %s", hipGetErrorString(e));
    }
    S->live_bytes = cursor;
    *out = S;
    return SV_OK;
}

void sv_destroy(sv_t *sv)
{
    if (!sv) return;
    (void)hipStreamSynchronize(sv->stream);
    for (hipEvent_t e : sv->events) (void)hipEventDestroy(e);
    delete sv;
}

int sv_attach_host_pool(sv_t *sv, void *host_pinned, uint64_t host_bytes)
{
    if (int rc = check_state(sv)) return rc;
    if (int rc = resolve_graph(sv)) return rc;
    if (!sv->reset_pending && sv->live_host)
        return fail(SV_ERR_INVALID, "the live state still has %llu bytes in the attached host pool",
                    (unsigned long long)sv->live_host);
    HIP_TRY(hipStreamSynchronize(sv->stream));     // no kernel may still use the old pool
    if (!host_pinned || !host_bytes) {
        sv->host[0] = sv->host[1] = sv->host_h[0] = sv->host_h[1] = nullptr;
        sv->host_cap = 0;
        return SV_OK;
    }
    void *dptr = nullptr;
    const hipError_t e = hipHostGetDevicePointer(&dptr, host_pinned, 0);
    if (e != hipSuccess || !dptr)
        return fail(SV_ERR_INVALID, "host pool is not pinned device-addressable memory (%s)", hipGetErrorString(e));
    const uint64_t half = (host_bytes / 2) & ~255ull;
    if (half < 4096) return fail(SV_ERR_INVALID, "host pool of %llu bytes is too small", (unsigned long long)host_bytes);
    const uint64_t cap = half - 1024;              // decoders read a little past a body
    if (sv->pool_cap + cap > bmq::kDirOffsetMask)
        return fail(SV_ERR_INVALID, "device + host pool exceed the directory's 40-bit offsets");
    sv->host[0] = (uint8_t *)dptr;
    sv->host[1] = (uint8_t *)dptr + half;
    sv->host_h[0] = (uint8_t *)host_pinned;
    sv->host_h[1] = (uint8_t *)host_pinned + half;
    sv->host_cap = cap;
    return SV_OK;
}

int sv_host_alloc(uint64_t bytes, void **ptr)
{
    if (!ptr) return fail(SV_ERR_INVALID, "ptr is NULL");
    if (!bytes) return fail(SV_ERR_INVALID, "zero bytes");
    *ptr = nullptr;
    void *p = nullptr;
    HIP_TRY(hipHostMalloc(&p, bytes, hipHostMallocDefault));
    *ptr = p;
    return SV_OK;
}

int sv_host_free(void *ptr)
{
    if (!ptr) return SV_OK;
    HIP_TRY(hipHostFree(ptr));
    return SV_OK;
}

int sv_reset(sv_t *sv)
{
    if (!sv) return fail(SV_ERR_INVALID, "state is NULL");
    sv->pending_graph = nullptr;          // the replay's result is discarded
    const uint64_t nch = 1ull << (sv->n - 6);
    unsigned long long *ic = sv->counters + kMaxLaunchesPerBatch * kStageCounters;
    HIP_TRY(bmq::launch_fill_u64((uint64_t *)ic, kStageCounters, 0, sv->stream));
    HIP_TRY(bmq::launch_init_state(sv->dir[0], nch, sv->pool[0], ic, codec_params(sv->cfg), sv->stream));
    sv->cur = 0;
    sv->poisoned = false;
    sv->reset_pending = true;
    return SV_OK;
}

}  // extern "C"

namespace {

int check_plan(const sv_t *sv, const sv_plan_t *p, size_t first, size_t count)
{
    if (!p) return fail(SV_ERR_INVALID, "plan is NULL");
    if (p->cfg.n_qubits != sv->cfg.n_qubits || p->cfg.block_qubits != sv->cfg.block_qubits ||
        p->cfg.domain != sv->cfg.domain || p->cfg.eb != sv->cfg.eb)
        return fail(SV_ERR_INVALID, "plan and state configurations differ");
    if (first > p->stages.size() || count > p->stages.size() - first)
        return fail(SV_ERR_INVALID, "stage range [%zu, %zu) outside the plan's %zu stages", first, first + count,
                    p->stages.size());
    return SV_OK;
}

int upload_plan(sv_t *sv, const sv_plan_t *p)
{
    if (sv->uploaded_uid == p->uid) return SV_OK;
    const uint64_t ob = p->ops.size() * sizeof(OpDesc);
    if (align256(ob) + p->data.size() * sizeof(float2) > kOpsArenaBytes)
        return fail(SV_ERR_UNSUPPORTED, "plan's fused operations exceed the %llu-byte operation arena",
                    (unsigned long long)kOpsArenaBytes);
    if (ob) HIP_TRY(hipMemcpyAsync(sv->ops_arena, p->ops.data(), ob, hipMemcpyHostToDevice, sv->stream));
    if (!p->data.empty())
        HIP_TRY(hipMemcpyAsync(sv->ops_arena + align256(ob), p->data.data(), p->data.size() * sizeof(float2),
                               hipMemcpyHostToDevice, sv->stream));
    HIP_TRY(hipStreamSynchronize(sv->stream));   // host vectors are pageable
    sv->uploaded_uid = p->uid;
    return SV_OK;
}

// One SV group of a multi-pass stage run with group-sized scratch planes:
// the group's qubits (ascending: the block qubits, the stage's inner
// indices and any other qubit a pass's tile holds), the other (outer) qubits,
// and the group's index, whose bits are deposited at the outer qubits.
struct GroupRun {
    std::vector<int> qubits, outer;
    uint64_t g = 0;
};

// The group qubits of stage st (see GroupRun) of an n-qubit state with b
// block qubits.
void group_qubits(int n, int b, const StagePlan &st, GroupRun &gr)
{
    std::vector<bool> in(n, false);
    for (int q = 0; q < b; ++q) in[q] = true;
    for (int q : st.inner) in[q] = true;
    for (const PassPlan &pp : st.passes)
        for (int q : pp.tileq) in[q] = true;
    gr.qubits.clear();
    gr.outer.clear();
    for (int q = 0; q < n; ++q) (in[q] ? gr.qubits : gr.outer).push_back(q);
}

// Tile geometry of pass pp in a: tile and non-tile qubits (of the whole
// state, or of group grp with its outer bits fixed), their packed positions
// in the group (scratch and packed directories), and the segment rotation
// of the group's waves.
void fill_geometry(bmq::PassArgs &a, int n, int t, const PassPlan &pp, const GroupRun *grp)
{
    for (int j = 0; j < t; ++j) a.tileq[j] = a.stileq[j] = pp.tileq[j];
    int nn = 0;
    if (!grp) {
        for (int q = 0; q < n; ++q)
            if (std::find(pp.tileq.begin(), pp.tileq.end(), q) == pp.tileq.end()) {
                a.snontile[nn] = q;
                a.nontile[nn++] = q;
            }
    } else {
        // packed position of a group qubit: its rank among the group qubits
        auto rank = [&](int q) { return (int)(std::find(grp->qubits.begin(), grp->qubits.end(), q) - grp->qubits.begin()); };
        for (int j = 0; j < t; ++j) a.stileq[j] = rank(pp.tileq[j]);
        for (int q : grp->qubits)
            if (std::find(pp.tileq.begin(), pp.tileq.end(), q) == pp.tileq.end()) {
                a.snontile[nn] = rank(q);
                a.nontile[nn++] = q;
            }
        for (size_t k = 0; k < grp->outer.size(); ++k)
            a.fixed |= ((grp->g >> k) & 1ull) << grp->outer[k];
        // the group's waves continue the segment rotation of the earlier groups
        a.seg_base = (uint32_t)((grp->g << nn) * (t == 13 ? 8u : 4u));
    }
    a.n_nontile = nn;
}

// Arguments of pass pi of stage st with counter block li; flips the state's
// current copy when the pass writes compressed output.  With a group, the
// launch covers that group's tiles only and addresses the group-sized
// scratch planes by the group qubits' packed positions.
void build_pass_args(sv_t *sv, const sv_plan_t *p, const StagePlan &st, int pi, size_t li, bmq::PassArgs &a,
                     const GroupRun *grp = nullptr)
{
    const int n = sv->n;
    const bool scratch = sv->scr_re != nullptr;
    const int np = (int)st.passes.size();
    // output pool segments: as many as waves, at most kSegments; each holds
    // the worst case of its tiles when the pool has its default size
    const uint64_t waves = (1ull << (n - p->t)) * (p->t == 13 ? 8u : 4u);
    const int n_seg = (int)std::min<uint64_t>((uint64_t)bmq::kSegments, waves);
    const PassPlan &pp = st.passes[pi];
    std::memset(&a, 0, sizeof(a));
    a.n = n;
    a.t = p->t;
    fill_geometry(a, n, p->t, pp, grp);
    a.op_begin = pp.op_begin;
    a.op_end = pp.op_end;
    // with scratch planes, passes between the first and the last stay
    // uncompressed; without, every pass is a compressed round
    a.in_mode = (!scratch || pi == 0) ? bmq::IO_COMPRESSED : bmq::IO_SCRATCH;
    a.out_mode = (!scratch || pi == np - 1) ? bmq::IO_COMPRESSED : bmq::IO_SCRATCH;
    a.cp = codec_params(sv->cfg);
    a.dir_in = sv->dir[sv->cur];
    a.pool_in = sv->pool[sv->cur];
    a.host_in = sv->host[sv->cur];
    a.dir_out = sv->dir[sv->cur ^ 1];
    a.pool_out = sv->pool[sv->cur ^ 1];
    a.host_out = sv->host[sv->cur ^ 1];
    a.pool_cap = sv->pool_cap;
    a.host_cap = sv->host_cap;
    a.n_seg = n_seg;
    a.seg_cap = (sv->pool_cap / (uint64_t)n_seg) & ~3ull;
    a.counters = sv->counters + li * kStageCounters;
    a.scr_re = sv->scr_re;
    a.scr_im = sv->scr_im;
    a.ops = (const OpDesc *)sv->ops_arena;
    a.opdata = (const float2 *)(sv->ops_arena + align256(p->ops.size() * sizeof(OpDesc)));
    a.dump_re = sv->dump_re;
    a.dump_im = sv->dump_im;
    a.dumpd_re = sv->dumpd_re;
    a.dumpd_im = sv->dumpd_im;
    a.dump_lo = sv->dump_lo;
    a.dump_n = sv->dump_n;
    a.mfma = (sv->cfg.flags & SV_FLAG_NO_MFMA) ? 0 : 1;
    if (a.out_mode == bmq::IO_COMPRESSED) sv->cur ^= 1;
}

// Enqueue pass pi of stage st on stream s with counter block li.
int enqueue_pass(sv_t *sv, const sv_plan_t *p, const StagePlan &st, int pi, size_t li, hipStream_t s)
{
    bmq::PassArgs a;
    build_pass_args(sv, p, st, pi, li, a);
    HIP_TRY(bmq::launch_pass(a, s));
    return SV_OK;
}

// Enqueue every launch of stage st on stream s, pass pi with counter block
// li0 + pi.  A multi-pass stage on group-sized scratch planes runs all its
// passes for one group, then the next group (groups are independent within a
// stage); the launches of a pass share its counter block, so its segments'
// cursors and statistics continue from group to group.
int enqueue_stage(sv_t *sv, const sv_plan_t *p, const StagePlan &st, size_t li0, hipStream_t s)
{
    const int np = (int)st.passes.size();
    if (!(sv->group_scratch && sv->scr_re && np > 1)) {
        for (int pi = 0; pi < np; ++pi)
            if (int rc = enqueue_pass(sv, p, st, pi, li0 + pi, s)) return rc;
        return SV_OK;
    }
    GroupRun gr;
    group_qubits(sv->n, sv->b, st, gr);
    if (gr.qubits.size() >= 64 || (1ull << gr.qubits.size()) > sv->scr_elems)
        return fail(SV_ERR_INVALID, "a multi-pass stage spans %zu qubits; the state's group scratch holds %llu "
                                    "amplitudes (create the state with this inner size and tile)",
                    gr.qubits.size(), (unsigned long long)sv->scr_elems);
    const int cur0 = sv->cur;
    for (gr.g = 0; gr.g < (1ull << gr.outer.size()); ++gr.g)
        for (int pi = 0; pi < np; ++pi) {
            sv->cur = cur0;
            bmq::PassArgs a;
            build_pass_args(sv, p, st, pi, li0 + pi, a, &gr);
            HIP_TRY(bmq::launch_pass(a, s));
        }
    sv->cur = cur0 ^ 1;
    return SV_OK;
}

// Whether the states' plans can run in one batched or queue launch: with
// group-sized scratch planes, a multi-pass stage runs group by group.
int check_full_scratch(const sv_t *sv, const sv_plan_t *p, size_t i)
{
    if (!sv->group_scratch || !sv->scr_re) return SV_OK;
    for (const StagePlan &st : p->stages)
        if (st.passes.size() > 1)
            return fail(SV_ERR_UNSUPPORTED, "state %zu has group-sized scratch planes and a multi-pass stage: run it "
                                            "with stage_apply_compressed", i);
    return SV_OK;
}

// Launches and counter blocks of the stage run [first, first + batch).
size_t launches_of(const sv_plan_t *p, size_t first, size_t batch)
{
    size_t l = 0;
    for (size_t i = 0; i < batch; ++i) l += p->stages[first + i].passes.size();
    return l;
}

// The batched launches of several states: launch k runs the k-th pass of
// every state that has one, grouped by tile size.
struct BatchGroup {
    size_t k;
    int t, dom;
    std::vector<size_t> members;     // state indices
    uint64_t args_off, fb_off;       // workspace offsets
    uint32_t blocks;
};

int plan_batch(sv_t *const *states, const sv_plan_t *const *plans, size_t count, std::vector<BatchGroup> &groups,
               uint64_t &bytes)
{
    if (!states || !plans || count == 0) return fail(SV_ERR_INVALID, "empty batch");
    size_t kmax = 0;
    for (size_t i = 0; i < count; ++i) {
        if (int rc = check_state(states[i])) return rc;
        if (int rc = check_plan(states[i], plans[i], 0, plans[i] ? plans[i]->stages.size() : 0)) return rc;
        if (int rc = check_full_scratch(states[i], plans[i], i)) return rc;
        for (size_t j = 0; j < i; ++j)
            if (states[j] == states[i]) return fail(SV_ERR_INVALID, "state %zu appears twice in the batch", i);
        if (states[i]->dump_re || states[i]->dumpd_re)
            return fail(SV_ERR_UNSUPPORTED, "the debug dump cannot run in a batch");
        const size_t l = launches_of(plans[i], 0, plans[i]->stages.size());
        if (l > kMaxLaunchesPerBatch)
            return fail(SV_ERR_UNSUPPORTED, "circuit %zu needs %zu pass launches (at most %zu in a batch)", i, l,
                        kMaxLaunchesPerBatch);
        kmax = std::max(kmax, l);
    }
    groups.clear();
    bytes = 0;
    for (size_t k = 0; k < kmax; ++k)
        for (int key = 30; key < 3 * (bmq::kMaxTile + 1); ++key) {      // tile sizes 10.. x domains
            const int t = key / 3, dom = key % 3;
            BatchGroup g{k, t, dom, {}, 0, 0, 0};
            uint64_t blocks = 0;
            for (size_t i = 0; i < count; ++i)
                if (plans[i]->t == t && states[i]->cfg.domain == dom &&
                    launches_of(plans[i], 0, plans[i]->stages.size()) > k) {
                    g.members.push_back(i);
                    blocks += 1ull << (states[i]->n - t);
                }
            if (g.members.empty()) continue;
            if (blocks > 0x7FFFFFFFull) return fail(SV_ERR_UNSUPPORTED, "a batched launch exceeds 2^31 workgroups");
            g.blocks = (uint32_t)blocks;
            g.args_off = bytes;
            bytes += align256(g.members.size() * sizeof(bmq::PassArgs));
            g.fb_off = bytes;
            bytes += align256((g.members.size() + 1) * sizeof(uint32_t));
            groups.push_back(std::move(g));
        }
    return SV_OK;
}

// Read the counter blocks of stages [first, first + batch) (host copy hc),
// check for overflow, fill stats (without ms) and advance the footprint.
int collect_stages(sv_t *sv, const sv_plan_t *p, size_t first, size_t batch,
                   const std::vector<unsigned long long> &hc, sv_stage_stats_t *stats)
{
    const bool scratch = sv->scr_re != nullptr;
    const int n = sv->n;
    const uint64_t nch = 1ull << (n - 6);
    size_t li = 0;
    for (size_t i = 0; i < batch; ++i) {
        const StagePlan &st = p->stages[first + i];
        const size_t np = st.passes.size();
        uint64_t inter = 0, out_dev = 0, out_host = 0, zero = 0, mh[4] = {0, 0, 0, 0};
        bool overflow = false;
        for (size_t pi = 0; pi < np; ++pi, ++li) {
            if (scratch && pi + 1 < np) continue;          // uncompressed intermediate pass
            // per segment: cursor, overflow flag, zero chunks, spilled and host
            // bytes, the ZERO count and the Q0|VERBATIM counts packed two
            // 32-bit counts per word; device bytes are the cursor less the
            // spilled bytes, LZ planes the rest of the pass's 2 nch planes
            uint64_t dev = 0, host = 0, z = 0, m4[4] = {0, 0, 0, 0};
            for (int g = 0; g < bmq::kSegments; ++g) {
                const unsigned long long *sg = &hc[li * kStageCounters + (size_t)g * bmq::C_NUM];
                overflow |= sg[bmq::C_OVERFLOW] != 0;
                dev += sg[bmq::C_CURSOR] - sg[bmq::C_SPILLED];
                host += sg[bmq::C_HOST_BYTES];
                z += sg[bmq::C_ZERO_CHUNKS];
                m4[0] += sg[bmq::C_MODE0];
                m4[2] += sg[bmq::C_MODE0 + 2] & 0xFFFFFFFFull;
                m4[3] += sg[bmq::C_MODE0 + 2] >> 32;
            }
            m4[1] = 2 * nch - m4[0] - m4[2] - m4[3];
            if (pi + 1 < np) inter += 2 * (dev + host);
            out_dev = dev;
            out_host = host;
            zero = z;
            for (int q = 0; q < 4; ++q) mh[q] = m4[q];
        }
        if (overflow) {
            sv->poisoned = true;
            return fail(SV_ERR_CAPACITY,
                        "stage %zu overflowed the compressed pools (device pool %llu bytes, host pool %llu bytes)",
                        first + i, (unsigned long long)sv->pool_cap, (unsigned long long)sv->host_cap);
        }
        if (stats) {
            sv_stage_stats_t &s = stats[i];
            const float ms = s.ms;
            std::memset(&s, 0, sizeof(s));
            s.ms = ms;
            s.bytes_in = sv->live_bytes;
            s.bytes_out = out_dev + out_host;
            s.bytes_out_host = out_host;
            s.inter_bytes = inter;
            s.dir_bytes = (scratch ? 1 : np) * 2ull * nch * 8ull;
            s.scratch_bytes = scratch ? (uint64_t)(np - 1) * 2ull * (1ull << n) * 8ull : 0;
            s.zero_chunks_out = zero;
            s.mode_hist[0] = mh[0]; s.mode_hist[1] = mh[1]; s.mode_hist[2] = mh[2]; s.mode_hist[3] = mh[3];
            s.passes = (uint32_t)np;
            s.launches = (uint32_t)np;
            if (sv->group_scratch && scratch && np > 1) {
                GroupRun gr;
                group_qubits(sv->n, sv->b, st, gr);
                s.launches = (uint32_t)(np << gr.outer.size());
            }
            uint32_t nops = 0;
            for (const auto &pp : st.passes) nops += (uint32_t)(pp.op_end - pp.op_begin);
            s.n_ops = nops;
            s.n_gates = (uint32_t)(st.g1 - st.g0);
            s.n_inner = (uint32_t)st.inner.size();
        }
        sv->live_bytes = out_dev + out_host;
        sv->live_host = out_host;
    }
    return SV_OK;
}

// Copy a batch's counters (and, after a reset, the initial footprint) to the
// host, synchronising the stream.
int read_counters(sv_t *sv, size_t launches, std::vector<unsigned long long> &hc)
{
    hc.resize(launches * kStageCounters);
    HIP_TRY(hipMemcpyAsync(hc.data(), sv->counters, hc.size() * 8, hipMemcpyDeviceToHost, sv->stream));
    unsigned long long init_cursor = 0;
    if (sv->reset_pending)
        HIP_TRY(hipMemcpyAsync(&init_cursor, sv->counters + kMaxLaunchesPerBatch * kStageCounters + bmq::C_CURSOR, 8,
                               hipMemcpyDeviceToHost, sv->stream));
    HIP_TRY(hipStreamSynchronize(sv->stream));
    if (sv->reset_pending) {
        sv->live_bytes = init_cursor;
        sv->live_host = 0;
        sv->reset_pending = false;
    }
    return SV_OK;
}

// A replayed graph leaves its counters on the device; read them before
// anything else uses the counter blocks or the footprint.
int resolve_graph(sv_t *sv)
{
    if (!sv->pending_graph) return SV_OK;
    const sv_graph *g = sv->pending_graph;
    sv->pending_graph = nullptr;
    if (g->persistent) {
        // abort flags first: an aborted launch leaves the state half-written
        std::vector<uint32_t> flags(g->flag_offs.size(), 0);
        for (size_t k = 0; k < flags.size(); ++k)
            HIP_TRY(hipMemcpyAsync(&flags[k], g->ws + g->flag_offs[k], 4, hipMemcpyDeviceToHost, sv->stream));
        HIP_TRY(hipStreamSynchronize(sv->stream));
        for (uint32_t f : flags)
            if (f) {
                sv->poisoned = true;
                return fail(SV_ERR_TIMEOUT, "a replayed persistent launch waited longer than %llu us for a "
                                            "dependency and was aborted; the state is poisoned",
                            (unsigned long long)g->limit_us);
            }
    }
    std::vector<unsigned long long> hc;
    if (int rc = read_counters(sv, g->launches, hc)) return rc;
    return collect_stages(sv, g->plan, g->first, g->count, hc, nullptr);
}

}  // namespace

extern "C" {

int stage_apply_compressed(sv_t *sv, const sv_plan_t *p, size_t first, size_t count, sv_stage_stats_t *stats)
{
    if (int rc = check_state(sv)) return rc;
    if (int rc = check_plan(sv, p, first, count)) return rc;
    if (count == 0) return SV_OK;
    if (int rc = resolve_graph(sv)) return rc;
    if (int rc = upload_plan(sv, p)) return rc;
    size_t done = 0;
    std::vector<unsigned long long> hc;
    while (done < count) {
        // a batch: whole stages whose passes fit the counter blocks
        size_t batch = 0, launches = 0;
        while (done + batch < count) {
            const size_t np = p->stages[first + done + batch].passes.size();
            if (batch && launches + np > kMaxLaunchesPerBatch) break;
            launches += np;
            ++batch;
        }
        HIP_TRY(bmq::launch_fill_u64((uint64_t *)sv->counters, launches * kStageCounters, 0, sv->stream));
        if (stats)
            while (sv->events.size() < 2 * batch) {
                hipEvent_t e;
                HIP_TRY(hipEventCreate(&e));
                sv->events.push_back(e);
            }
        size_t li = 0;
        for (size_t i = 0; i < batch; ++i) {
            const StagePlan &st = p->stages[first + done + i];
            if (stats) HIP_TRY(hipEventRecord(sv->events[2 * i], sv->stream));
            if (int rc = enqueue_stage(sv, p, st, li, sv->stream)) return rc;
            li += st.passes.size();
            if (stats) HIP_TRY(hipEventRecord(sv->events[2 * i + 1], sv->stream));
        }
        if (int rc = read_counters(sv, launches, hc)) return rc;
        if (stats)
            for (size_t i = 0; i < batch; ++i)
                HIP_TRY(hipEventElapsedTime(&stats[done + i].ms, sv->events[2 * i], sv->events[2 * i + 1]));
        if (int rc = collect_stages(sv, p, first + done, batch, hc, stats ? stats + done : nullptr)) return rc;
        done += batch;
    }
    return SV_OK;
}

int sv_autotune_space(const sv_gate_t *gates, size_t n_gates, const sv_config_t *cfg, void *dev_arena,
                      uint64_t dev_bytes, void *hip_stream, const sv_tune_space_t *space, sv_config_t *best,
                      float *ms_out)
{
    if (int rc = validate_cfg(cfg)) return rc;
    if (!best) return fail(SV_ERR_INVALID, "best is NULL");
    if (!space) return fail(SV_ERR_INVALID, "space is NULL");
    const sv_tune_space_t &S = *space;
    if (S.n_tiles < 1 || S.n_tiles > 4 || S.n_fuse < 1 || S.n_fuse > 5 || S.n_inner < 1 || S.n_inner > 6)
        return fail(SV_ERR_INVALID, "search space sizes (%d tiles, %d fusion widths, %d inner sizes) outside "
                                    "[1, 4] x [1, 5] x [1, 6]", S.n_tiles, S.n_fuse, S.n_inner);
    for (int i = 0; i < S.n_tiles; ++i)
        if (S.tiles[i] < 10 || S.tiles[i] > bmq::kMaxTile || S.tiles[i] > cfg->n_qubits)
            return fail(SV_ERR_INVALID, "tile candidate %d outside [10, min(13, n)]", S.tiles[i]);
    for (int i = 0; i < S.n_fuse; ++i)
        if (S.fuse[i] < 1 || S.fuse[i] > 5) return fail(SV_ERR_INVALID, "fusion candidate %d outside [1, 5]", S.fuse[i]);
    for (int i = 0; i < S.n_inner; ++i)
        if (S.inner[i] < 1 || S.inner[i] > 8) return fail(SV_ERR_INVALID, "inner-size candidate %d outside [1, 8]", S.inner[i]);
    const size_t ng = S.probe_gates && S.probe_gates < n_gates ? (size_t)S.probe_gates : n_gates;
    const int total = S.n_tiles * S.n_fuse * S.n_inner;
    if (ms_out)
        for (int i = 0; i < total; ++i) ms_out[i] = NAN;
    float best_ms = INFINITY;
    sv_config_t winner = *cfg;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int rc = SV_OK;
    for (int it = 0; it < S.n_tiles && rc == SV_OK; ++it)
        for (int ifu = 0; ifu < S.n_fuse && rc == SV_OK; ++ifu)
            for (int ii = 0; ii < S.n_inner && rc == SV_OK; ++ii) {
                sv_config_t c = *cfg;
                c.tile_qubits = S.tiles[it];
                c.fuse_qubits = S.fuse[ifu];
                c.inner_size = S.inner[ii];
                sv_plan_t *p = nullptr;
                sv_t *sv = nullptr;
                rc = stage_plan(gates, ng, &c, &p);
                if (rc == SV_ERR_INVALID) {          // a gate this inner size cannot hold: not a candidate
                    rc = SV_OK;
                    continue;
                }
                if (rc == SV_OK) rc = sv_create(&c, dev_arena, dev_bytes, hip_stream, &sv);
                float ms = 0.0f;
                // one warm-up run (first launches load code), then the timed run
                for (int rep = 0; rc == SV_OK && rep < 2; ++rep) {
                    rc = sv_reset(sv);
                    if (rc == SV_OK && hipEventRecord(e0, sv->stream) != hipSuccess) rc = fail(SV_ERR_HIP, "event");
                    if (rc == SV_OK) rc = stage_apply_compressed(sv, p, 0, p->stages.size(), nullptr);
                    if (rc == SV_OK && hipEventRecord(e1, sv->stream) != hipSuccess) rc = fail(SV_ERR_HIP, "event");
                    if (rc == SV_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(SV_ERR_HIP, "event");
                    if (rc == SV_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(SV_ERR_HIP, "event");
                }
                if (sv) sv_destroy(sv);
                if (p) plan_destroy(p);
                if (rc == SV_ERR_CAPACITY) rc = SV_OK;     // this candidate does not fit the pools: skip it
                else if (rc == SV_OK) {
                    if (ms_out) ms_out[(it * S.n_fuse + ifu) * S.n_inner + ii] = ms;
                    if (ms < best_ms) {
                        best_ms = ms;
                        winner = c;
                    }
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SV_OK) return rc;
    if (!(best_ms < INFINITY)) return fail(SV_ERR_CAPACITY, "no candidate fits the pools");
    *best = winner;
    return SV_OK;
}

int sv_autotune(const sv_gate_t *gates, size_t n_gates, const sv_config_t *cfg, void *dev_arena,
                uint64_t dev_bytes, void *hip_stream, size_t probe_stages, sv_config_t *best, float *ms_all)
{
    if (int rc = validate_cfg(cfg)) return rc;
    // the probe is a prefix of the circuit: the gates of its first probe_stages stages
    size_t probe_gates = 0;
    if (probe_stages) {
        sv_plan_t *p = nullptr;
        if (int rc = stage_plan(gates, n_gates, cfg, &p)) return rc;
        if (probe_stages < p->stages.size() && !(cfg->flags & SV_FLAG_COMMUTE))
            probe_gates = p->stages[probe_stages - 1].g1;
        plan_destroy(p);
    }
    sv_tune_space_t S{};
    S.n_tiles = 0;
    for (int t = 10; t <= bmq::kMaxTile && t <= cfg->n_qubits; ++t) S.tiles[S.n_tiles++] = t;
    S.n_fuse = 5;
    for (int k = 1; k <= 5; ++k) S.fuse[k - 1] = k;
    S.n_inner = 1;
    S.inner[0] = cfg->inner_size;
    S.probe_gates = probe_gates;
    float ms[20];
    const int rc = sv_autotune_space(gates, n_gates, cfg, dev_arena, dev_bytes, hip_stream, &S, best, ms);
    if (ms_all) {
        for (int i = 0; i < 20; ++i) ms_all[i] = NAN;
        if (rc == SV_OK)
            for (int it = 0; it < S.n_tiles; ++it)
                for (int k = 0; k < 5; ++k) ms_all[(S.tiles[it] - 10) * 5 + k] = ms[it * 5 + k];
    }
    return rc;
}

int sv_graph_capture(sv_t *sv, const sv_plan_t *p, size_t first, size_t count, sv_graph_t **out)
{
    if (int rc = check_state(sv)) return rc;
    if (int rc = check_plan(sv, p, first, count)) return rc;
    if (!out) return fail(SV_ERR_INVALID, "out is NULL");
    if (count == 0) return fail(SV_ERR_INVALID, "empty stage range");
    if (sv->dump_re || sv->dumpd_re) return fail(SV_ERR_UNSUPPORTED, "the debug dump cannot be captured");
    const size_t launches = launches_of(p, first, count);
    if (launches > kMaxLaunchesPerBatch)
        return fail(SV_ERR_UNSUPPORTED, "%zu pass launches exceed the %zu counter blocks of one graph", launches,
                    kMaxLaunchesPerBatch);
    if (int rc = resolve_graph(sv)) return rc;
    if (int rc = upload_plan(sv, p)) return rc;
    sv_graph *g = new (std::nothrow) sv_graph;
    if (!g) return fail(SV_ERR_OOM, "host allocation failed");
    g->sv = sv;
    g->plan = p;
    g->plan_uid = p->uid;
    g->first = first;
    g->count = count;
    g->launches = launches;
    g->cur_begin = sv->cur;
    // capture on a private stream (the legacy default stream cannot capture)
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    int rc = SV_OK;
    if (e == hipSuccess) {
        // counters are cleared by a kernel, not a memset node
        e = bmq::launch_fill_u64((uint64_t *)sv->counters, launches * kStageCounters, 0, cs);
        size_t li = 0;
        for (size_t i = 0; e == hipSuccess && rc == SV_OK && i < count; ++i) {
            const StagePlan &st = p->stages[first + i];
            rc = enqueue_stage(sv, p, st, li, cs);
            li += st.passes.size();
        }
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (e == hipSuccess) e = e2;
        g->g = graph;
        if (e == hipSuccess && rc == SV_OK) e = hipGraphInstantiate(&g->x, g->g, nullptr, nullptr, 0);
    }
    g->cur_end = sv->cur;
    sv->cur = g->cur_begin;                       // capture ran nothing
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess || rc != SV_OK) {
        sv_graph_destroy(g);
        return rc != SV_OK ? rc : fail(SV_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    }
    *out = g;
    return SV_OK;
}

int sv_graph_launch(sv_t *sv, sv_graph_t *g)
{
    if (int rc = check_state(sv)) return rc;
    if (!g || g->sv != sv) return fail(SV_ERR_INVALID, "graph was not captured on this state");
    if (g->plan_uid != sv->uploaded_uid)
        return fail(SV_ERR_INVALID, "another plan's operations were uploaded since the capture");
    if (sv->cur != g->cur_begin)
        return fail(SV_ERR_INVALID, "the state is in its other pool copy; replay needs the copy it was captured on");
    if (int rc = resolve_graph(sv)) return rc;
    HIP_TRY(hipGraphLaunch(g->x, sv->stream));
    sv->cur = g->cur_end;
    sv->pending_graph = g;
    return SV_OK;
}

int sv_graph_sync(sv_t *sv)
{
    if (int rc = check_state(sv)) return rc;
    return resolve_graph(sv);
}

void sv_graph_destroy(sv_graph_t *g)
{
    if (!g) return;
    if (g->sv && g->sv->pending_graph == g) (void)resolve_graph(g->sv);
    if (g->x) (void)hipGraphExecDestroy(g->x);
    if (g->g) (void)hipGraphDestroy(g->g);
    delete g;
}

int sv_batch_workspace(sv_t *const *states, const sv_plan_t *const *plans, size_t count, uint64_t *bytes)
{
    if (!bytes) return fail(SV_ERR_INVALID, "bytes is NULL");
    std::vector<BatchGroup> groups;
    return plan_batch(states, plans, count, groups, *bytes);
}

int sv_batch_apply(sv_t *const *states, const sv_plan_t *const *plans, size_t count, void *workspace_dev,
                   uint64_t workspace_bytes, void *hip_stream)
{
    std::vector<BatchGroup> groups;
    uint64_t need = 0;
    if (int rc = plan_batch(states, plans, count, groups, need)) return rc;
    if (!workspace_dev || ((uintptr_t)workspace_dev & 255u) || workspace_bytes < need)
        return fail(SV_ERR_INVALID, "workspace must be 256-byte aligned and hold %llu bytes", (unsigned long long)need);
    hipStream_t stream = (hipStream_t)hip_stream;
    for (size_t i = 0; i < count; ++i)
        if (states[i]->stream != stream)
            return fail(SV_ERR_INVALID, "state %zu was created on another stream", i);
    for (size_t i = 0; i < count; ++i) {
        if (int rc = resolve_graph(states[i])) return rc;
        if (int rc = upload_plan(states[i], plans[i])) return rc;
    }
    // every state's pass arguments in launch order (the current pool copy
    // advances as stage_apply_compressed would advance it)
    std::vector<std::vector<bmq::PassArgs>> args(count);
    for (size_t i = 0; i < count; ++i) {
        sv_t *sv = states[i];
        const sv_plan_t *p = plans[i];
        size_t li = 0;
        for (const StagePlan &st : p->stages)
            for (int pi = 0; pi < (int)st.passes.size(); ++pi, ++li) {
                bmq::PassArgs a;
                build_pass_args(sv, p, st, pi, li, a);
                args[i].push_back(a);
            }
    }
    std::vector<uint8_t> host(need, 0);
    for (const BatchGroup &g : groups) {
        bmq::PassArgs *ga = (bmq::PassArgs *)(host.data() + g.args_off);
        uint32_t *fb = (uint32_t *)(host.data() + g.fb_off);
        uint32_t acc = 0;
        for (size_t m = 0; m < g.members.size(); ++m) {
            const size_t i = g.members[m];
            ga[m] = args[i][g.k];
            fb[m] = acc;
            acc += (uint32_t)(1ull << (states[i]->n - g.t));
        }
        fb[g.members.size()] = acc;
    }
    uint8_t *ws = (uint8_t *)workspace_dev;
    HIP_TRY(hipMemcpyAsync(ws, host.data(), need, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));          // the host image is pageable
    for (size_t i = 0; i < count; ++i)
        HIP_TRY(bmq::launch_fill_u64((uint64_t *)states[i]->counters, args[i].size() * kStageCounters, 0, stream));
    for (const BatchGroup &g : groups)
        HIP_TRY(bmq::launch_pass_batch(g.t, g.dom, (const bmq::PassArgs *)(ws + g.args_off), (const uint32_t *)(ws + g.fb_off),
                                       (int)g.members.size(), g.blocks, stream));
    std::vector<unsigned long long> hc;
    int first_err = SV_OK;
    std::string err;
    for (size_t i = 0; i < count; ++i) {
        int rc = read_counters(states[i], args[i].size(), hc);
        if (rc == SV_OK) rc = collect_stages(states[i], plans[i], 0, plans[i]->stages.size(), hc, nullptr);
        if (rc != SV_OK && first_err == SV_OK) {
            first_err = rc;
            err = g_err;
        }
    }
    if (first_err != SV_OK) g_err = err;
    return first_err;
}

}  // extern "C"

namespace {

// One persistent launch per tile size and domain: the pass list of its
// circuits in queue order (pass k of every circuit that has one, then pass
// k + 1, ...), each pass depending on the previous pass of its circuit.
struct PersistClass {
    int t, dom;
    std::vector<size_t> members;                  // state indices
    std::vector<std::pair<size_t, size_t>> pass;  // (state index, pass index)
    std::vector<uint32_t> first_item;             // n_pass + 1
    std::vector<uint32_t> tpi;
    std::vector<int32_t> dep;
    uint64_t args_off, first_off, tpi_off, dep_off, sync_off, sync_words;
};

int plan_persistent(sv_t *const *states, const sv_plan_t *const *plans, size_t count,
                    std::vector<PersistClass> &classes, uint64_t &bytes, int cus)
{
    std::vector<BatchGroup> groups;              // validation shared with the batched launches
    uint64_t unused = 0;
    if (int rc = plan_batch(states, plans, count, groups, unused)) return rc;
    classes.clear();
    bytes = 0;
    for (int key = 30; key < 3 * (bmq::kMaxTile + 1); ++key) {          // tile sizes 10.. x domains
        PersistClass c;
        c.t = key / 3;
        c.dom = key % 3;
        size_t kmax = 0;
        for (size_t i = 0; i < count; ++i)
            if (plans[i]->t == c.t && states[i]->cfg.domain == c.dom) {
                c.members.push_back(i);
                kmax = std::max(kmax, launches_of(plans[i], 0, plans[i]->stages.size()));
            }
        if (c.members.empty()) continue;
        // An item is a run of consecutive tiles of one pass, so that the
        // device-wide claim of an item is paid once per run: as long as
        // every pass step still has about eight items per resident
        // workgroup (resident: four per compute unit), up to 32 tiles per
        // item.  Finished items are counted once per workgroup and pass.
        uint64_t widest = 0;
        for (size_t k = 0; k < kmax; ++k) {
            uint64_t w = 0;
            for (size_t i : c.members)
                if (launches_of(plans[i], 0, plans[i]->stages.size()) > k) w += 1ull << (states[i]->n - c.t);
            widest = std::max(widest, w);
        }
        uint64_t per_max = 1;
        while (per_max < 32 && widest / (2 * per_max) >= 8ull * 4ull * cus) per_max *= 2;
        std::vector<int32_t> last(count, -1);
        uint64_t items = 0;
        for (size_t k = 0; k < kmax; ++k)
            for (size_t i : c.members) {
                if (launches_of(plans[i], 0, plans[i]->stages.size()) <= k) continue;
                const uint64_t tiles = 1ull << (states[i]->n - c.t);
                const uint64_t per = std::min(per_max, tiles);
                c.first_item.push_back((uint32_t)items);
                c.tpi.push_back((uint32_t)per);
                c.dep.push_back(last[i]);
                last[i] = (int32_t)c.pass.size();
                c.pass.push_back({i, k});
                items += tiles / per;
                if (items > 0x7FFFFFFFull) return fail(SV_ERR_UNSUPPORTED, "a persistent launch exceeds 2^31 tiles");
            }
        if (c.pass.empty()) continue;
        c.first_item.push_back((uint32_t)items);
        c.args_off = bytes;
        bytes += align256(c.pass.size() * sizeof(bmq::PassArgs));
        c.first_off = bytes;
        bytes += align256(c.first_item.size() * sizeof(uint32_t));
        c.tpi_off = bytes;
        bytes += align256(c.tpi.size() * sizeof(uint32_t));
        c.dep_off = bytes;
        bytes += align256(c.dep.size() * sizeof(int32_t));
        c.sync_off = bytes;
        c.sync_words = (bmq::kSyncHead + c.pass.size() + 1) / 2;        // u64 words
        bytes += align256(c.sync_words * 8);
        classes.push_back(std::move(c));
    }
    return SV_OK;
}

}  // namespace

extern "C" {

int sv_persistent_workspace(sv_t *const *states, const sv_plan_t *const *plans, size_t count, uint64_t *bytes)
{
    if (!bytes) return fail(SV_ERR_INVALID, "bytes is NULL");
    std::vector<PersistClass> classes;
    return plan_persistent(states, plans, count, classes, *bytes, 256);   // sizes do not depend on the CU count
}

}  // extern "C"

namespace {

// The three steps of a whole-circuit queue launch.  prepare: checks, plan
// uploads and the workspace image (launch arguments, item table,
// dependencies), uploaded once (synchronises: the host image is pageable);
// it advances each state's current pool copy to where the launch leaves it.
// enqueue: the counter and queue-word clears (fill kernels) and the queue
// kernels -- kernels only, so that it can be captured in a graph.  collect:
// abort flags, then every stage's counters (synchronises).
struct PersistPrep {
    std::vector<PersistClass> classes;
    std::vector<std::vector<bmq::PassArgs>> args;
    std::vector<bmq::PersistArgs> pa;
    uint64_t limit_us = 0;
};

int persist_prepare(sv_t *const *states, const sv_plan_t *const *plans, size_t count, void *workspace_dev,
                    uint64_t workspace_bytes, uint32_t wait_limit_us, hipStream_t stream, PersistPrep &P)
{
    int dev = 0, khz = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    uint64_t need = 0;
    if (int rc = plan_persistent(states, plans, count, P.classes, need, std::max(cus, 1))) return rc;
    if (!workspace_dev || ((uintptr_t)workspace_dev & 255u) || workspace_bytes < need)
        return fail(SV_ERR_INVALID, "workspace must be 256-byte aligned and hold %llu bytes", (unsigned long long)need);
    for (size_t i = 0; i < count; ++i)
        if (states[i]->stream != stream)
            return fail(SV_ERR_INVALID, "state %zu was created on another stream", i);
    if (khz <= 0) return fail(SV_ERR_UNSUPPORTED, "the device reports no constant-rate clock");
    P.limit_us = wait_limit_us ? wait_limit_us : 10000000u;
    for (size_t i = 0; i < count; ++i) {
        if (int rc = resolve_graph(states[i])) return rc;
        if (int rc = upload_plan(states[i], plans[i])) return rc;
    }
    P.args.assign(count, {});
    for (size_t i = 0; i < count; ++i) {
        size_t li = 0;
        for (const StagePlan &st : plans[i]->stages)
            for (int pi = 0; pi < (int)st.passes.size(); ++pi, ++li) {
                bmq::PassArgs a;
                build_pass_args(states[i], plans[i], st, pi, li, a);
                P.args[i].push_back(a);
            }
    }
    std::vector<uint8_t> host(need, 0);
    for (const PersistClass &c : P.classes) {
        bmq::PassArgs *ga = (bmq::PassArgs *)(host.data() + c.args_off);
        for (size_t L = 0; L < c.pass.size(); ++L) ga[L] = P.args[c.pass[L].first][c.pass[L].second];
        std::memcpy(host.data() + c.first_off, c.first_item.data(), c.first_item.size() * sizeof(uint32_t));
        std::memcpy(host.data() + c.dep_off, c.dep.data(), c.dep.size() * sizeof(int32_t));
        std::memcpy(host.data() + c.tpi_off, c.tpi.data(), c.tpi.size() * sizeof(uint32_t));
    }
    uint8_t *ws = (uint8_t *)workspace_dev;
    HIP_TRY(hipMemcpyAsync(ws, host.data(), need, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));          // the host image is pageable
    P.pa.clear();
    for (const PersistClass &c : P.classes) {
        bmq::PersistArgs pa;
        std::memset(&pa, 0, sizeof(pa));
        pa.args = (const bmq::PassArgs *)(ws + c.args_off);
        pa.first_item = (const uint32_t *)(ws + c.first_off);
        pa.tiles_per_item = (const uint32_t *)(ws + c.tpi_off);
        pa.max_grid = (uint32_t)std::max(cus, 1) * 4u;       // resident workgroups
        pa.dep = (const int32_t *)(ws + c.dep_off);
        pa.sync = (uint32_t *)(ws + c.sync_off);
        pa.limit_ticks = P.limit_us * (uint64_t)khz / 1000u;
        pa.n_pass = (uint32_t)c.pass.size();
        pa.total = c.first_item.back();
        for (size_t i : c.members) pa.system_scope |= states[i]->host_cap ? 1 : 0;
        P.pa.push_back(pa);
    }
    return SV_OK;
}

hipError_t persist_enqueue(sv_t *const *states, size_t count, const PersistPrep &P, hipStream_t stream)
{
    hipError_t e = hipSuccess;
    for (size_t i = 0; e == hipSuccess && i < count; ++i)
        e = bmq::launch_fill_u64((uint64_t *)states[i]->counters, P.args[i].size() * kStageCounters, 0, stream);
    for (size_t k = 0; e == hipSuccess && k < P.classes.size(); ++k) {
        e = bmq::launch_fill_u64((uint64_t *)P.pa[k].sync, P.classes[k].sync_words, 0, stream);
        if (e == hipSuccess) e = bmq::launch_pass_queue(P.classes[k].t, P.classes[k].dom, P.pa[k], stream);
    }
    return e;
}

int persist_collect(sv_t *const *states, const sv_plan_t *const *plans, size_t count, const PersistPrep &P,
                    hipStream_t stream)
{
    // abort flags first: an aborted class leaves its states half-written
    std::vector<uint32_t> flags(P.classes.size(), 0);
    for (size_t k = 0; k < P.classes.size(); ++k)
        HIP_TRY(hipMemcpyAsync(&flags[k], P.pa[k].sync + 1, 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    bool aborted = false;
    for (size_t k = 0; k < P.classes.size(); ++k)
        if (flags[k]) {
            aborted = true;
            for (size_t i : P.classes[k].members) states[i]->poisoned = true;
        }
    if (aborted)
        return fail(SV_ERR_TIMEOUT, "a persistent launch waited longer than %llu us for a dependency and was "
                                    "aborted; its states are poisoned",
                    (unsigned long long)P.limit_us);
    std::vector<unsigned long long> hc;
    int first_err = SV_OK;
    std::string err;
    for (size_t i = 0; i < count; ++i) {
        int rc = read_counters(states[i], P.args[i].size(), hc);
        if (rc == SV_OK) rc = collect_stages(states[i], plans[i], 0, plans[i]->stages.size(), hc, nullptr);
        if (rc != SV_OK && first_err == SV_OK) {
            first_err = rc;
            err = g_err;
        }
    }
    if (first_err != SV_OK) g_err = err;
    return first_err;
}

}  // namespace

extern "C" {

int sv_persistent_apply(sv_t *const *states, const sv_plan_t *const *plans, size_t count, void *workspace_dev,
                        uint64_t workspace_bytes, uint32_t wait_limit_us, void *hip_stream)
{
    const hipStream_t stream = (hipStream_t)hip_stream;
    PersistPrep P;
    if (int rc = persist_prepare(states, plans, count, workspace_dev, workspace_bytes, wait_limit_us, stream, P))
        return rc;
    HIP_TRY(persist_enqueue(states, count, P, stream));
    return persist_collect(states, plans, count, P, stream);
}

int sv_graph_capture_persistent(sv_t *sv, const sv_plan_t *p, void *workspace_dev, uint64_t workspace_bytes,
                                uint32_t wait_limit_us, sv_graph_t **out)
{
    if (int rc = check_state(sv)) return rc;
    if (!p || !out) return fail(SV_ERR_INVALID, "NULL argument");
    if (p->stages.empty()) return fail(SV_ERR_INVALID, "empty plan");
    if (sv->dump_re || sv->dumpd_re) return fail(SV_ERR_UNSUPPORTED, "the debug dump cannot be captured");
    sv_t *const states[1] = {sv};
    const sv_plan_t *const plans[1] = {p};
    const int cur_begin = sv->cur;
    PersistPrep P;
    if (int rc = persist_prepare(states, plans, 1, workspace_dev, workspace_bytes, wait_limit_us, sv->stream, P)) {
        sv->cur = cur_begin;
        return rc;
    }
    sv_graph *g = new (std::nothrow) sv_graph;
    if (!g) {
        sv->cur = cur_begin;
        return fail(SV_ERR_OOM, "host allocation failed");
    }
    g->sv = sv;
    g->plan = p;
    g->plan_uid = p->uid;
    g->first = 0;
    g->count = p->stages.size();
    g->launches = P.args[0].size();
    g->cur_begin = cur_begin;
    g->cur_end = sv->cur;
    g->persistent = true;
    g->ws = (uint8_t *)workspace_dev;
    g->limit_us = P.limit_us;
    for (const bmq::PersistArgs &pa : P.pa) g->flag_offs.push_back((uint64_t)((uint8_t *)(pa.sync + 1) - g->ws));
    sv->cur = cur_begin;                          // capture runs nothing
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        e = persist_enqueue(states, 1, P, cs);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (e == hipSuccess) e = e2;
        g->g = graph;
        if (e == hipSuccess) e = hipGraphInstantiate(&g->x, g->g, nullptr, nullptr, 0);
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        sv_graph_destroy(g);
        return fail(SV_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    }
    *out = g;
    return SV_OK;
}

int sv_fidelity(const sv_t *sv, const double *ref_host, const double *ref_dev, const sv_t *ref_sv, sv_fidelity_t *out)
{
    if (int rc = check_state(sv)) return rc;
    if (!out) return fail(SV_ERR_INVALID, "out is NULL");
    if ((ref_host != nullptr) + (ref_dev != nullptr) + (ref_sv != nullptr) > 1)
        return fail(SV_ERR_INVALID, "give at most one reference");
    if (ref_sv) {
        if (int rc = check_state(ref_sv)) return rc;
        if (ref_sv->n != sv->n) return fail(SV_ERR_INVALID, "reference state has %d qubits, state %d", ref_sv->n, sv->n);
        if (ref_sv->stream != sv->stream) HIP_TRY(hipStreamSynchronize(ref_sv->stream));
    }
    const uint64_t nch = 1ull << (sv->n - 6);
    const int np = (int)std::min<uint64_t>(kPartials, (nch + 63) / 64);
    const bmq::CodecParams cp = codec_params(sv->cfg);
    HIP_TRY(bmq::launch_fill_u64((uint64_t *)sv->partials, (uint64_t)np * 5, 0ull, sv->stream));
    bmq::RefView rv{};
    rv.kind = bmq::REF_NONE;
    if (ref_dev) {
        rv.kind = bmq::REF_C128;
        rv.c128 = (const double2 *)ref_dev;
    } else if (ref_sv) {
        rv.kind = bmq::REF_STATE;
        rv.dir = ref_sv->dir[ref_sv->cur];
        rv.pv = pool_view(ref_sv, ref_sv->cur);
        rv.cp = codec_params(ref_sv->cfg);
    }
    if (ref_host) {
        // stream the host reference through the staging area, slice by slice
        const uint64_t slice = kStageBytes / (64 * 16);        // chunks per slice
        rv.kind = bmq::REF_C128;
        rv.c128 = (const double2 *)sv->stage;
        for (uint64_t c0 = 0; c0 < nch; c0 += slice) {
            const uint64_t nc = std::min(slice, nch - c0);
            HIP_TRY(hipMemcpyAsync(sv->stage, ref_host + 2 * 64 * c0, nc * 64 * 16, hipMemcpyHostToDevice, sv->stream));
            HIP_TRY(bmq::launch_fidelity_partial(sv->dir[sv->cur], pool_view(sv, sv->cur), cp, c0, nc, rv, sv->partials,
                                                 np, sv->stream));
        }
    } else {
        HIP_TRY(bmq::launch_fidelity_partial(sv->dir[sv->cur], pool_view(sv, sv->cur), cp, 0, nch, rv, sv->partials, np,
                                             sv->stream));
    }
    HIP_TRY(bmq::launch_fidelity_final(sv->partials, np, sv->out5, sv->stream));
    double h[5];
    HIP_TRY(hipMemcpyAsync(h, sv->out5, sizeof(h), hipMemcpyDeviceToHost, sv->stream));
    HIP_TRY(hipStreamSynchronize(sv->stream));
    out->norm2 = h[2];
    if (rv.kind != bmq::REF_NONE) {
        out->overlap_re = h[0];
        out->overlap_im = h[1];
        out->overlap2 = h[0] * h[0] + h[1] * h[1];
        out->ref_norm2 = h[3];
        out->fidelity = out->overlap2 / (h[2] * h[3]);
        out->max_abs_err = h[4];
    } else {
        out->overlap_re = out->overlap_im = out->overlap2 = out->ref_norm2 = NAN;
        out->fidelity = out->max_abs_err = NAN;
    }
    return SV_OK;
}

namespace {
// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): output i of the sequence whose state starts at
// seed, as a double in [0, 1) from its top 53 bits.
static double splitmix_uniform(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}
}  // namespace

int sv_sample(const sv_t *sv, uint64_t k, uint64_t seed, uint64_t *idx_host)
{
    if (int rc = check_state(sv)) return rc;
    if (!k) return SV_OK;
    if (!idx_host) return fail(SV_ERR_INVALID, "idx_host is NULL");
    const int n = sv->n;
    // groups of 2^gq amplitudes, at least 16 chunks and at most 2^16 groups
    const int gq = std::max(10, n - 16);
    const uint32_t cpg = 1u << (gq - 6);
    const uint64_t ng = 1ull << (n - gq);
    const bmq::PoolView pv = pool_view(sv, sv->cur);
    const bmq::CodecParams cp = codec_params(sv->cfg);
    double *gnorm = (double *)sv->stage;
    uint32_t *grp = (uint32_t *)(sv->stage + kMaxSampleGroups * 8);
    double *resid = (double *)(sv->stage + kMaxSampleGroups * 8 + kSampleBatch * 4);
    uint64_t *outd = (uint64_t *)(sv->stage + kMaxSampleGroups * 8 + kSampleBatch * 12);
    HIP_TRY(bmq::launch_group_norm(sv->dir[sv->cur], pv, cp, cpg, ng, gnorm, sv->stream));
    std::vector<double> gn(ng), pre(ng + 1);
    HIP_TRY(hipMemcpyAsync(gn.data(), gnorm, ng * 8, hipMemcpyDeviceToHost, sv->stream));
    HIP_TRY(hipStreamSynchronize(sv->stream));
    pre[0] = 0;
    for (uint64_t g = 0; g < ng; ++g) pre[g + 1] = pre[g] + gn[g];
    const double total = pre[ng];
    if (!(total > 0) || !std::isfinite(total)) return fail(SV_ERR_INVALID, "state has no finite, positive norm");
    std::vector<uint32_t> hg(kSampleBatch);
    std::vector<double> hr(kSampleBatch);
    for (uint64_t s0 = 0; s0 < k; s0 += kSampleBatch) {
        const uint64_t nb = std::min(kSampleBatch, k - s0);
        for (uint64_t i = 0; i < nb; ++i) {
            const double u = splitmix_uniform(seed, s0 + i) * total;
            // the group g with pre[g] <= u < pre[g + 1] (groups of zero norm are never chosen)
            uint64_t g = (uint64_t)(std::upper_bound(pre.begin(), pre.end(), u) - pre.begin()) - 1;
            if (g >= ng) g = ng - 1;
            while (g > 0 && gn[g] == 0.0) --g;
            hg[i] = (uint32_t)g;
            hr[i] = std::min(std::max(u - pre[g], 0.0), gn[g]);
        }
        HIP_TRY(hipMemcpyAsync(grp, hg.data(), nb * 4, hipMemcpyHostToDevice, sv->stream));
        HIP_TRY(hipMemcpyAsync(resid, hr.data(), nb * 8, hipMemcpyHostToDevice, sv->stream));
        HIP_TRY(bmq::launch_sample(sv->dir[sv->cur], pv, cp, cpg, grp, resid, nb, outd, sv->stream));
        HIP_TRY(hipMemcpyAsync(idx_host + s0, outd, nb * 8, hipMemcpyDeviceToHost, sv->stream));
        HIP_TRY(hipStreamSynchronize(sv->stream));     // the host tables are reused by the next batch
    }
    return SV_OK;
}

int sv_export(const sv_t *sv, uint64_t start, uint64_t count, void *dst_dev)
{
    if (int rc = check_state(sv)) return rc;
    const uint64_t dim = 1ull << sv->n;
    if ((start & 63) || (count & 63) || start > dim || count > dim - start || (count && !dst_dev))
        return fail(SV_ERR_INVALID, "export range must be 64-aligned and inside the state");
    if (!count) return SV_OK;
    HIP_TRY(bmq::launch_export(sv->dir[sv->cur], pool_view(sv, sv->cur), codec_params(sv->cfg), start >> 6, count >> 6,
                               (float2 *)dst_dev, sv->stream));
    return SV_OK;
}

int sv_amplitudes(const sv_t *sv, const uint64_t *idx_dev, uint64_t k, void *out_dev)
{
    if (int rc = check_state(sv)) return rc;
    if (k && (!idx_dev || !out_dev)) return fail(SV_ERR_INVALID, "NULL pointer");
    if (!k) return SV_OK;
    HIP_TRY(bmq::launch_amplitudes(sv->dir[sv->cur], pool_view(sv, sv->cur), codec_params(sv->cfg), idx_dev, k,
                                   1ull << (sv->n - 6), (float2 *)out_dev, sv->stream));
    return SV_OK;
}

int sv_footprint(const sv_t *sv, uint64_t *record_bytes, uint64_t *host_bytes, uint64_t *dir_bytes)
{
    if (int rc = check_state(sv)) return rc;
    if (int rc = resolve_graph(const_cast<sv_t *>(sv))) return rc;
    if (sv->reset_pending) {
        unsigned long long c = 0;
        HIP_TRY(hipMemcpyAsync(&c, sv->counters + kMaxLaunchesPerBatch * kStageCounters + bmq::C_CURSOR, 8,
                               hipMemcpyDeviceToHost, sv->stream));
        HIP_TRY(hipStreamSynchronize(sv->stream));
        const_cast<sv_t *>(sv)->live_bytes = c;
        const_cast<sv_t *>(sv)->reset_pending = false;
    }
    if (record_bytes) *record_bytes = sv->live_bytes;
    if (host_bytes) *host_bytes = sv->live_host;
    if (dir_bytes) *dir_bytes = (1ull << (sv->n - 6)) * 8ull;
    return SV_OK;
}

int sv_directory(const sv_t *sv, const uint64_t **dir_dev, uint64_t *n_entries)
{
    if (int rc = check_state(sv)) return rc;
    if (int rc = resolve_graph(const_cast<sv_t *>(sv))) return rc;
    if (dir_dev) *dir_dev = sv->dir[sv->cur];
    if (n_entries) *n_entries = 1ull << (sv->n - 6);
    return SV_OK;
}

int sv_check(sv_t *sv, uint64_t *n_bad)
{
    if (n_bad) *n_bad = 0;
    if (int rc = check_state(sv)) return rc;
    if (int rc = resolve_graph(sv)) return rc;
    unsigned long long *bad = (unsigned long long *)sv->out5;
    HIP_TRY(bmq::launch_fill_u64((uint64_t *)bad, 1, 0, sv->stream));
    HIP_TRY(bmq::launch_check_dir(sv->dir[sv->cur], 1ull << (sv->n - 6), sv->pool_cap,
                                  sv->host[sv->cur] ? sv->host_cap : 0, sv->cfg.domain, bad, sv->stream));
    unsigned long long h = 0;
    HIP_TRY(hipMemcpyAsync(&h, bad, 8, hipMemcpyDeviceToHost, sv->stream));
    HIP_TRY(hipStreamSynchronize(sv->stream));
    if (n_bad) *n_bad = h;
    if (h) {
        sv->poisoned = true;
        return fail(SV_ERR_CORRUPT, "%llu malformed directory entries", h);
    }
    return SV_OK;
}

int sv_block_features(const sv_t *sv, const sv_plan_t *p, size_t stage, float *feats_dev)
{
    if (int rc = check_state(sv)) return rc;
    if (!p || !feats_dev) return fail(SV_ERR_INVALID, "NULL argument");
    if (p->cfg.n_qubits != sv->cfg.n_qubits || p->cfg.block_qubits != sv->cfg.block_qubits)
        return fail(SV_ERR_INVALID, "plan and state configurations differ");
    if (stage >= p->stages.size()) return fail(SV_ERR_INVALID, "stage %zu outside the plan", stage);
    if (sv->n - sv->b > 30) return fail(SV_ERR_UNSUPPORTED, "more than 2^30 blocks");
    const bmq::StageFeats sf = stage_feats(p, stage);
    HIP_TRY(bmq::launch_block_stats(sv->dir[sv->cur], 1ull << (sv->b - 6), 1ull << (sv->n - sv->b), sf, feats_dev,
                                    nullptr, nullptr, sv->stream));
    return SV_OK;
}

int sv_plan_features(const sv_t *sv, const sv_plan_t *p, size_t stage, float *feats_dev)
{
    if (int rc = sv_block_features(sv, p, stage, feats_dev)) return rc;
    HIP_TRY(bmq::launch_plan_form(feats_dev, nullptr, (uint32_t)(1ull << (sv->n - sv->b)), sv->b, sv->stream));
    return SV_OK;
}

int sv_plan_labels(const sv_t *sv, float *log2_bytes_dev, int32_t *mode_dev)
{
    if (int rc = sv_block_labels(sv, log2_bytes_dev, mode_dev)) return rc;
    HIP_TRY(bmq::launch_plan_form(nullptr, log2_bytes_dev, (uint32_t)(1ull << (sv->n - sv->b)), sv->b, sv->stream));
    return SV_OK;
}

int mlp_predict_work(const sv_plan_t *p, uint64_t *bytes)
{
    if (!p || !bytes) return fail(SV_ERR_INVALID, "NULL argument");
    if (p->cfg.n_qubits - p->cfg.block_qubits > 20) return fail(SV_ERR_UNSUPPORTED, "more than 2^20 blocks");
    *bytes = predict_work(p->cfg, p->stages.size()).total;
    return SV_OK;
}

int mlp_predict_bytes(const float *params_dev, const sv_plan_t *p, void *work_dev, uint64_t work_bytes,
                      double *bytes_host, void *hip_stream)
{
    if (!params_dev || !p || !work_dev || (!bytes_host && !p->stages.empty())) return fail(SV_ERR_INVALID, "NULL argument");
    if ((uintptr_t)work_dev & 255u) return fail(SV_ERR_INVALID, "work must be 256-byte aligned");
    const sv_config_t &c = p->cfg;
    if (c.n_qubits - c.block_qubits > 20) return fail(SV_ERR_UNSUPPORTED, "more than 2^20 blocks");
    const size_t ns = p->stages.size();
    const PredictWork w = predict_work(c, ns);
    if (work_bytes < w.total)
        return fail(SV_ERR_INVALID, "work space of %llu bytes < %llu", (unsigned long long)work_bytes,
                    (unsigned long long)w.total);
    if (!ns) return SV_OK;
    const hipStream_t st = (hipStream_t)hip_stream;
    uint8_t *W = (uint8_t *)work_dev;
    uint64_t *dir = (uint64_t *)(W + w.off_dir);
    float *X = (float *)(W + w.off_x), *out = (float *)(W + w.off_out);
    double *tot = (double *)(W + w.off_tot);
    const uint64_t cpb = 1ull << (c.block_qubits - 6);
    const uint32_t nb = (uint32_t)(1ull << (c.n_qubits - c.block_qubits));
    // features of |0...0>: block 0 holds the encoded amplitude 1, every
    // other block is all zero; two blocks are built and the second copied
    HIP_TRY(bmq::launch_init_state(dir, 2 * cpb, W + w.off_pool, (unsigned long long *)(W + w.off_cnt),
                                   codec_params(c), st));
    HIP_TRY(bmq::launch_block_stats(dir, cpb, nb >= 2 ? 2 : 1, stage_feats(p, 0), X, nullptr, nullptr, st));
    HIP_TRY(bmq::launch_replicate_rows(X, nb, st));
    HIP_TRY(bmq::launch_plan_form(X, nullptr, nb, c.block_qubits, st));
    for (size_t s = 0; s < ns; ++s) {
        bmq::StageFeats next{};
        if (s + 1 < ns) next = stage_feats(p, s + 1);
        HIP_TRY(bmq::launch_mlp_forward(params_dev, X, nb, out, st));
        HIP_TRY(bmq::launch_rollout_step(X, out, nb, next, c.block_qubits, tot + s, st));
    }
    HIP_TRY(hipMemcpyAsync(bytes_host, tot, ns * 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return SV_OK;
}

int sv_admit(const sv_config_t *cfgs, size_t count, const double *peak_bytes, double margin, uint64_t budget,
             uint8_t *admit_out, uint64_t *pool_bytes_out, uint64_t *arena_bytes_out)
{
    if (count && (!cfgs || !admit_out)) return fail(SV_ERR_INVALID, "NULL argument");
    if (!(margin >= 0.0) || !std::isfinite(margin)) return fail(SV_ERR_INVALID, "margin must be finite and >= 0");
    for (size_t i = 0; i < count; ++i)
        if (int rc = validate_cfg(&cfgs[i])) return rc;
    uint64_t used = 0;
    for (size_t i = 0; i < count; ++i) {
        sv_config_t c = cfgs[i];
        c.pool_bytes = 0;
        const uint64_t worst = layout_for(c).pool_cap;
        uint64_t pool = worst;
        if (peak_bytes) {
            // record bodies: the stream bytes less the two 4-byte headers per
            // chunk (they live in the directory), with the margin and the
            // segment slack the worst case also carries
            const double nch = (double)(1ull << (c.n_qubits - 6));
            const double body = std::max(0.0, peak_bytes[i] - 8.0 * nch);
            const double want = std::ceil(body * (1.0 + margin)) + (double)bmq::kSegments * 256.0 + 1024.0;
            if (want < (double)worst) pool = align256((uint64_t)want);
        }
        c.pool_bytes = pool;
        const uint64_t arena = layout_for(c).total;
        const bool ok = used + arena <= budget;
        if (ok) used += arena;
        admit_out[i] = ok ? 1 : 0;
        if (pool_bytes_out) pool_bytes_out[i] = pool;
        if (arena_bytes_out) arena_bytes_out[i] = arena;
    }
    return SV_OK;
}

int sv_block_labels(const sv_t *sv, float *log2_bytes_dev, int32_t *mode_dev)
{
    if (int rc = check_state(sv)) return rc;
    if (!log2_bytes_dev || !mode_dev) return fail(SV_ERR_INVALID, "NULL argument");
    if (sv->n - sv->b > 30) return fail(SV_ERR_UNSUPPORTED, "more than 2^30 blocks");
    bmq::StageFeats sf{};
    HIP_TRY(bmq::launch_block_stats(sv->dir[sv->cur], 1ull << (sv->b - 6), 1ull << (sv->n - sv->b), sf, nullptr,
                                    log2_bytes_dev, mode_dev, sv->stream));
    return SV_OK;
}

int mlp_forward(const float *params_dev, const float *x_dev, uint32_t batch, float *out_dev, void *hip_stream)
{
    if (!params_dev || (batch && (!x_dev || !out_dev))) return fail(SV_ERR_INVALID, "NULL pointer");
    if (batch > (1u << 30)) return fail(SV_ERR_INVALID, "batch above 2^30");
    if (!batch) return SV_OK;
    HIP_TRY(bmq::launch_mlp_forward(params_dev, x_dev, batch, out_dev, (hipStream_t)hip_stream));
    return SV_OK;
}

uint64_t mlp_work_floats(uint32_t batch) { return bmq::mlp_work_floats(batch); }

int mlp_loss_grad(const float *params_dev, const float *x_dev, const float *y_log2_bytes_dev,
                  const int32_t *y_mode_dev, uint32_t batch, float *work_dev, float *grad_dev, float *loss_dev,
                  void *hip_stream)
{
    if (!params_dev || !x_dev || !y_log2_bytes_dev || !y_mode_dev || !work_dev || !grad_dev || !loss_dev)
        return fail(SV_ERR_INVALID, "NULL pointer");
    if (batch == 0 || batch > (1u << 30)) return fail(SV_ERR_INVALID, "batch must be in [1, 2^30]");
    HIP_TRY(bmq::launch_mlp_loss_grad(params_dev, x_dev, y_log2_bytes_dev, y_mode_dev, batch, work_dev, grad_dev,
                                      loss_dev, (hipStream_t)hip_stream));
    return SV_OK;
}

int mlp_adam_update(float *params_dev, const float *grad_dev, float *m_dev, float *v_dev, uint32_t step, float lr,
                    void *hip_stream)
{
    if (!params_dev || !grad_dev || !m_dev || !v_dev) return fail(SV_ERR_INVALID, "NULL pointer");
    if (step == 0) return fail(SV_ERR_INVALID, "Adam steps count from 1");
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return fail(SV_ERR_INVALID, "learning rate must be finite and >= 0");
    const double c1 = 1.0 / (1.0 - std::pow((double)SV_MLP_BETA1, (double)step));
    const double c2 = 1.0 / (1.0 - std::pow((double)SV_MLP_BETA2, (double)step));
    HIP_TRY(bmq::launch_mlp_adam(params_dev, grad_dev, m_dev, v_dev, lr, SV_MLP_BETA1, SV_MLP_BETA2, SV_MLP_EPS,
                                 (float)c1, (float)c2, (hipStream_t)hip_stream));
    return SV_OK;
}

int sv_block_stream(const sv_t *sv, uint64_t block, void *dst_host, uint64_t cap, uint64_t *bytes)
{
    if (int rc = check_state(sv)) return rc;
    if (!bytes) return fail(SV_ERR_INVALID, "bytes is NULL");
    const int b = sv->b;
    if (block >= (1ull << (sv->n - b))) return fail(SV_ERR_INVALID, "block %llu out of range", (unsigned long long)block);
    const uint64_t nchb = 1ull << (b - 6);
    const uint64_t chunk0 = block * nchb;
    // the directory holds each chunk's two headers and its body offset; the
    // canonical record is the headers followed by the body
    std::vector<uint64_t> dir(nchb);
    HIP_TRY(hipMemcpyAsync(dir.data(), sv->dir[sv->cur] + chunk0, nchb * 8, hipMemcpyDeviceToHost, sv->stream));
    HIP_TRY(hipStreamSynchronize(sv->stream));
    std::vector<uint32_t> sizes(nchb);
    uint64_t total = 16;
    for (uint64_t c = 0; c < nchb; ++c) {
        if (dir[c] == bmq::kDirInvalid) return fail(SV_ERR_CORRUPT, "chunk %llu lost to an overflow", (unsigned long long)(chunk0 + c));
        sizes[c] = body_bytes_host((uint32_t)(dir[c] >> 40) & 0xFFFu) + body_bytes_host((uint32_t)(dir[c] >> 52));
        total += 8 + sizes[c];
    }
    *bytes = total;
    if (!dst_host || cap < total) return fail(SV_ERR_INVALID, "buffer of %llu bytes < stream of %llu", (unsigned long long)cap,
                                             (unsigned long long)total);
    uint8_t *d = (uint8_t *)dst_host;
    const float ebf = (float)sv->cfg.eb;
    uint32_t ebbits;
    std::memcpy(&ebbits, &ebf, 4);
    const uint32_t nv = (uint32_t)(1ull << b), nc = (uint32_t)nchb;
    d[0] = 0x51; d[1] = 1; d[2] = (uint8_t)sv->cfg.domain; d[3] = 6;
    std::memcpy(d + 4, &ebbits, 4);
    std::memcpy(d + 8, &nv, 4);
    std::memcpy(d + 12, &nc, 4);
    // bodies that lie back to back in the device pool (a wave writes its
    // chunks' bodies contiguously) are fetched with one copy and scattered
    // between the headers on the host
    struct Piece { uint64_t dst; uint32_t len; };
    struct Run { uint64_t src, len; size_t p0, np; };
    std::vector<Piece> pieces;
    std::vector<Run> runs;
    uint64_t o = 16;
    for (uint64_t c = 0; c < nchb; ++c) {
        const uint32_t h0 = (uint32_t)(dir[c] >> 40) & 0xFFFu, h1 = (uint32_t)(dir[c] >> 52);
        std::memcpy(d + o, &h0, 4);
        std::memcpy(d + o + 4, &h1, 4);
        o += 8;
        if (sizes[c]) {
            const uint64_t off = dir[c] & bmq::kDirOffsetMask;
            if (off < sv->pool_cap) {
                if (runs.empty() || runs.back().src + runs.back().len != off)
                    runs.push_back(Run{off, 0, pieces.size(), 0});
                runs.back().len += sizes[c];
                runs.back().np++;
                pieces.push_back(Piece{o, sizes[c]});
            } else {
                std::memcpy(d + o, sv->host_h[sv->cur] + (off - sv->pool_cap), sizes[c]);
            }
            o += sizes[c];
        }
    }
    std::vector<uint8_t> tmp;
    for (const Run &r : runs) {
        tmp.resize(r.len);
        HIP_TRY(hipMemcpy(tmp.data(), sv->pool[sv->cur] + r.src, r.len, hipMemcpyDeviceToHost));
        uint64_t t = 0;
        for (size_t i = r.p0; i < r.p0 + r.np; ++i) {
            std::memcpy(d + pieces[i].dst, tmp.data() + t, pieces[i].len);
            t += pieces[i].len;
        }
    }
    return SV_OK;
}

int sv_debug_dump(sv_t *sv, uint64_t start, uint64_t count, float *pre_re, float *pre_im, float *post_re,
                  float *post_im)
{
    if (int rc = check_state(sv)) return rc;
    if ((pre_re == nullptr) != (pre_im == nullptr) || (post_re == nullptr) != (post_im == nullptr))
        return fail(SV_ERR_INVALID, "give both planes or neither");
    const uint64_t dim = 1ull << sv->n;
    if ((start & 63) || (count & 63) || start > dim || count > dim - start)
        return fail(SV_ERR_INVALID, "dump range must be 64-aligned and inside the state");
    sv->dump_re = pre_re;
    sv->dump_im = pre_im;
    sv->dumpd_re = post_re;
    sv->dumpd_im = post_im;
    sv->dump_lo = start;
    sv->dump_n = count;
    return SV_OK;
}

namespace {
static int check_codec_args(const sv_config_t *cfg, uint64_t n_values)
{
    if (!cfg || !(cfg->eb > 0) || (cfg->domain < SV_DOMAIN_LIN || cfg->domain > SV_DOMAIN_RAW))
        return fail(SV_ERR_INVALID, "bad codec config");
    if (n_values % 64) return fail(SV_ERR_INVALID, "n_values must be a multiple of 64 (whole chunks)");
    if (n_values > (1ull << 31)) return fail(SV_ERR_INVALID, "n_values above 2^31");
    return SV_OK;
}

// codec workspace: record sizes (u32 per chunk), record offsets (u64 per
// chunk + 1), one flag word
struct CodecWork {
    uint64_t off_sizes, off_offs, off_flag, total;
};
static CodecWork codec_work(uint64_t nch)
{
    CodecWork w{};
    w.off_sizes = 0;
    w.off_offs = align256(nch * 4);
    w.off_flag = w.off_offs + align256((nch + 1) * 8);
    w.total = w.off_flag + 256;
    return w;
}

static int codec_encode_impl(const float *re_dev, const float *im_dev, uint64_t n_values, const sv_config_t *cfg,
                      void *dst_dev, uint64_t cap, uint64_t *bytes, uint8_t *work, hipStream_t st)
{
    const uint64_t nch = n_values / 64;
    const CodecWork w = codec_work(nch);
    uint64_t *off = (uint64_t *)(work + w.off_offs);
    const float ebf = (float)cfg->eb;
    uint32_t ebbits;
    std::memcpy(&ebbits, &ebf, 4);
    HIP_TRY(bmq::launch_codec_stream_encode(re_dev, im_dev, nch, codec_params(*cfg), (uint32_t *)(work + w.off_sizes),
                                            off, (uint8_t *)dst_dev, cap, ebbits, st));
    uint64_t total = 0;
    HIP_TRY(hipMemcpyAsync(&total, off + nch, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *bytes = 16 + total;
    if (16 + total > cap)
        return fail(SV_ERR_INVALID, "stream of %llu bytes > capacity %llu (nothing written)",
                    (unsigned long long)(16 + total), (unsigned long long)cap);
    return SV_OK;
}
}  // namespace

int codec_encode_chunks(const float *re_dev, const float *im_dev, uint64_t n_values, const sv_config_t *cfg,
                        void *slots_dev, uint32_t *sizes_dev, void *hip_stream)
{
    if (int rc = check_codec_args(cfg, n_values)) return rc;
    if (!n_values) return SV_OK;
    if (!re_dev || !im_dev || !slots_dev || !sizes_dev) return fail(SV_ERR_INVALID, "NULL pointer");
    HIP_TRY(bmq::launch_codec_slots_encode(re_dev, im_dev, n_values / 64, codec_params(*cfg), (uint8_t *)slots_dev,
                                           sizes_dev, (hipStream_t)hip_stream));
    return SV_OK;
}

int codec_decode_chunks(const void *slots_dev, uint64_t n_values, const sv_config_t *cfg, float *re_dev, float *im_dev,
                        void *hip_stream)
{
    if (int rc = check_codec_args(cfg, n_values)) return rc;
    if (!n_values) return SV_OK;
    if (!re_dev || !im_dev || !slots_dev) return fail(SV_ERR_INVALID, "NULL pointer");
    HIP_TRY(bmq::launch_codec_slots_decode((const uint8_t *)slots_dev, n_values / 64, codec_params(*cfg), re_dev,
                                           im_dev, (hipStream_t)hip_stream));
    return SV_OK;
}

int codec_workspace(uint64_t n_values, uint64_t *bytes)
{
    if (!bytes) return fail(SV_ERR_INVALID, "bytes is NULL");
    if (n_values % 64 || n_values > (1ull << 31)) return fail(SV_ERR_INVALID, "n_values must be a multiple of 64, <= 2^31");
    *bytes = codec_work(n_values / 64).total;
    return SV_OK;
}

int codec_encode(const float *re_dev, const float *im_dev, uint64_t n_values, const sv_config_t *cfg, void *dst_dev,
                 uint64_t cap, uint64_t *bytes, void *work_dev, uint64_t work_bytes, void *hip_stream)
{
    if (int rc = check_codec_args(cfg, n_values)) return rc;
    if (!n_values) return fail(SV_ERR_INVALID, "empty input");
    if (!re_dev || !im_dev || !dst_dev || !bytes || !work_dev) return fail(SV_ERR_INVALID, "NULL pointer");
    if (((uintptr_t)dst_dev & 3u) || ((uintptr_t)work_dev & 255u))
        return fail(SV_ERR_INVALID, "dst must be 4-byte and work 256-byte aligned");
    if (work_bytes < codec_work(n_values / 64).total)
        return fail(SV_ERR_INVALID, "workspace of %llu bytes < %llu", (unsigned long long)work_bytes,
                    (unsigned long long)codec_work(n_values / 64).total);
    return codec_encode_impl(re_dev, im_dev, n_values, cfg, dst_dev, cap, bytes, (uint8_t *)work_dev,
                             (hipStream_t)hip_stream);
}

int codec_encode_noalloc(const float *re_dev, const float *im_dev, uint64_t n_values, const sv_config_t *cfg,
                         void *dst_dev, uint64_t cap, uint64_t *bytes, void *hip_stream)
{
    if (int rc = check_codec_args(cfg, n_values)) return rc;
    if (!n_values) return fail(SV_ERR_INVALID, "empty input");
    if (n_values > bmq::kNoAllocMaxValues)
        return fail(SV_ERR_INVALID, "n_values %llu above %llu, the most the static scratch holds",
                    (unsigned long long)n_values, (unsigned long long)bmq::kNoAllocMaxValues);
    if (!re_dev || !im_dev || !dst_dev || !bytes) return fail(SV_ERR_INVALID, "NULL pointer");
    if ((uintptr_t)dst_dev & 3u) return fail(SV_ERR_INVALID, "dst must be 4-byte aligned");
    static_assert(bmq::kNoAllocMaxValues % 64 == 0, "whole chunks");
    if (codec_work(bmq::kNoAllocMaxValues / 64).total > bmq::kNoAllocScratchBytes)
        return fail(SV_ERR_UNSUPPORTED, "static scratch smaller than the codec workspace");
    void *work = nullptr;
    HIP_TRY(bmq::noalloc_scratch(&work));
    return codec_encode_impl(re_dev, im_dev, n_values, cfg, dst_dev, cap, bytes, (uint8_t *)work,
                             (hipStream_t)hip_stream);
}

int codec_decode(const void *src_dev, uint64_t bytes, const sv_config_t *cfg, uint64_t n_values, float *re_dev,
                 float *im_dev, void *work_dev, uint64_t work_bytes, void *hip_stream)
{
    if (int rc = check_codec_args(cfg, n_values)) return rc;
    if (!n_values) return fail(SV_ERR_INVALID, "empty output");
    if (!src_dev || !re_dev || !im_dev || !work_dev) return fail(SV_ERR_INVALID, "NULL pointer");
    if (((uintptr_t)src_dev & 3u) || ((uintptr_t)work_dev & 255u))
        return fail(SV_ERR_INVALID, "src must be 4-byte and work 256-byte aligned");
    const uint64_t nch = n_values / 64;
    const CodecWork w = codec_work(nch);
    if (work_bytes < w.total)
        return fail(SV_ERR_INVALID, "workspace of %llu bytes < %llu", (unsigned long long)work_bytes,
                    (unsigned long long)w.total);
    if (bytes < 16) return fail(SV_ERR_CORRUPT, "stream shorter than its header");
    const hipStream_t st = (hipStream_t)hip_stream;
    uint8_t *work = (uint8_t *)work_dev;
    uint32_t hdr[4];
    HIP_TRY(hipMemcpyAsync(hdr, src_dev, 16, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const float ebf = (float)cfg->eb;
    uint32_t ebbits;
    std::memcpy(&ebbits, &ebf, 4);
    const uint32_t want = 0x51u | (1u << 8) | ((uint32_t)cfg->domain << 16) | (6u << 24);
    if (hdr[0] != want || hdr[1] != ebbits || hdr[2] != (uint32_t)n_values || hdr[3] != (uint32_t)nch)
        return fail(SV_ERR_CORRUPT, "stream header does not match the configuration and n_values");
    uint32_t *flag = (uint32_t *)(work + w.off_flag);
    uint64_t *off = (uint64_t *)(work + w.off_offs);
    HIP_TRY(bmq::launch_fill_u64((uint64_t *)flag, 1, 0ull, st));
    HIP_TRY(bmq::launch_codec_stream_decode((const uint8_t *)src_dev, bytes, nch, codec_params(*cfg), off, flag, st));
    uint32_t bad = 0;
    HIP_TRY(hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (bad) return fail(SV_ERR_CORRUPT, "malformed record in the stream");
    HIP_TRY(bmq::launch_codec_read((const uint8_t *)src_dev, off, nch, codec_params(*cfg), re_dev, im_dev, st));
    return SV_OK;
}

}  // extern "C"

// ====================================================================== host-resident pipeline
//
// The compressed state lives in the caller's pinned host memory as one image
// per SV block ([the block's chunk directory, body offsets relative to the
// image's body area] [bodies in chunk order]).  Every stage moves each SV
// group through the device on one of S streams (Section 4.2, Fig. 6): the
// group's block images are copied in (H2D), their directories rebased into
// one staging pool, the stage's tile passes run on the group alone (its
// outer bits fixed, directory and scratch in the group's packed order), the
// output is packed into new block images and copied back (D2H).  Groups of a
// stage are independent, so while one stream computes, the others copy.

namespace {

struct PipeStream {
    hipStream_t s = nullptr;
    hipEvent_t packed = nullptr;
    uint64_t *dir[2] = {nullptr, nullptr};   // staging directories (packed order); [0] receives the input
    uint8_t *pool[2] = {nullptr, nullptr};   // staging record pools
    uint64_t *body_off = nullptr;            // per block of the group: its bodies' offset in pool[0]
    float *scr_re = nullptr, *scr_im = nullptr;
    unsigned long long *counters = nullptr;  // kMaxPipePasses counter blocks
    uint32_t *rel = nullptr;
    uint64_t *segsum = nullptr, *img_off = nullptr;
    uint8_t *img = nullptr;
    uint64_t *h_off = nullptr, *h_img = nullptr;   // pinned host: body offsets (in), image offsets (out)
    bool pending = false;
    std::vector<uint64_t> pend_blocks;
};

constexpr int kMaxPipeStreams = 8;
constexpr size_t kMaxPipePasses = 64;

struct PipeLayout {
    int gq = 0;                     // log2 amplitudes of the largest group
    uint64_t gch = 0, gblocks = 0;  // its chunks and blocks
    uint64_t pool_cap = 0, seg = 0;
    uint64_t per_stream = 0, total = 0;
    uint64_t off_dir[2], off_pool[2], off_body, off_scr_re, off_scr_im, off_counters, off_rel, off_segsum, off_img_off,
        off_img;
    uint64_t off_ops, off_load_off;
    uint64_t host_small = 0;        // pinned bytes of the per-stream arrays
};

PipeLayout pipe_layout(const sv_config_t &c, int S)
{
    PipeLayout L;
    const int n = c.n_qubits, b = c.block_qubits;
    const int t = c.tile_qubits ? c.tile_qubits : kDefaultTile;
    L.gq = std::min(n, std::max(b + std::max(c.inner_size, 2), t));
    L.gch = 1ull << (L.gq - 6);
    L.gblocks = 1ull << (L.gq - b);
    L.pool_cap = L.gch * bmq::kMaxBodyBytes + bmq::kSegments * 256ull;
    L.seg = std::min<uint64_t>(1024, 1ull << (b - 6));
    uint64_t o = 0;
    L.off_dir[0] = o; o += align256(L.gch * 8);
    L.off_dir[1] = o; o += align256(L.gch * 8);
    L.off_pool[0] = o; o += align256(L.pool_cap + 1024);
    L.off_pool[1] = o; o += align256(L.pool_cap + 1024);
    L.off_body = o; o += align256(L.gblocks * 8);
    const uint64_t scr = (c.flags & SV_FLAG_NO_SCRATCH) ? 0 : align256((1ull << L.gq) * 4);
    L.off_scr_re = o; o += scr;
    L.off_scr_im = o; o += scr;
    L.off_counters = o; o += align256(kMaxPipePasses * kStageCounters * 8);
    L.off_rel = o; o += align256(L.gch * 4);
    L.off_segsum = o; o += align256(L.gch / L.seg * 8 + 8);
    L.off_img_off = o; o += align256((2 * L.gblocks + 1) * 8);
    L.off_img = o; o += align256(L.gch * (8 + bmq::kMaxBodyBytes) + 16 * L.gblocks);
    L.per_stream = o;
    L.off_ops = (uint64_t)S * L.per_stream;
    L.off_load_off = L.off_ops + kOpsArenaBytes;
    L.total = L.off_load_off + align256((1ull << (n - b)) * 8);
    L.host_small = align256((uint64_t)S * 3 * (L.gblocks + 1) * 8);
    return L;
}

}  // namespace

struct sv_pipe {
    sv_config_t cfg{};
    int n = 0, b = 0, S = 0;
    hipStream_t user = nullptr;
    uint8_t *ws = nullptr;
    PipeLayout L;
    uint8_t *host = nullptr;
    uint64_t host_bytes = 0, host_used = 0;
    struct Slot {
        uint64_t off = 0, cap = 0, size = 0;    // image: host offset, room, bytes (16-byte multiple)
        uint64_t body = 0;                      // its record bodies' bytes
    };
    std::vector<Slot> slots;          // block images in the host buffer
    std::vector<PipeStream> st;
    uint8_t *ops = nullptr;
    uint64_t uploaded_uid = 0;
    uint64_t h2d = 0, d2h = 0;        // bytes moved since the last reset
    bool poisoned = false;
};

namespace {

// Reserve host room for block k's next image of `size` bytes: in place when
// it fits (the old image is dead once the group's copy-in has run, which
// precedes its copy-out on the same stream), else a new slot with a quarter
// of headroom.
int pipe_slot(sv_pipe *pp, uint64_t k, uint64_t size, uint64_t body)
{
    sv_pipe::Slot &sl = pp->slots[k];
    if (size > sl.cap) {
        const uint64_t cap = align256(size + size / 4);
        if (pp->host_used + cap > pp->host_bytes) {
            pp->poisoned = true;
            return fail(SV_ERR_CAPACITY, "host store full: block %llu needs %llu bytes, %llu of %llu in use",
                        (unsigned long long)k, (unsigned long long)cap, (unsigned long long)pp->host_used,
                        (unsigned long long)pp->host_bytes);
        }
        sl.off = pp->host_used;
        sl.cap = cap;
        pp->host_used += cap;
    }
    sl.size = size;
    sl.body = body;
    return SV_OK;
}

// The group on stream ps has been packed: read its image offsets, place the
// images in the host store and copy them out (asynchronously).
int pipe_finish(sv_pipe *pp, PipeStream &ps)
{
    if (!ps.pending) return SV_OK;
    ps.pending = false;
    HIP_TRY(hipEventSynchronize(ps.packed));
    for (size_t j = 0; j < ps.pend_blocks.size(); ++j) {
        const uint64_t size = ps.h_img[j + 1] - ps.h_img[j];
        const uint64_t k = ps.pend_blocks[j];
        if (int rc = pipe_slot(pp, k, size, ps.h_img[ps.pend_blocks.size() + 1 + j])) return rc;
        HIP_TRY(hipMemcpyAsync(pp->host + pp->slots[k].off, ps.img + ps.h_img[j], size, hipMemcpyDeviceToHost, ps.s));
        pp->d2h += 8 * (1ull << (pp->b - 6)) + pp->slots[k].body;
    }
    return SV_OK;
}

// Pack the n_blk blocks of the staged output (dir, pool) on ps into images,
// their offsets copied to the pinned h_img; blocks receives their ids.
int pipe_pack(sv_pipe *pp, PipeStream &ps, const uint64_t *dir, const uint8_t *pool, uint64_t n_blk,
              std::vector<uint64_t> &&blocks)
{
    const uint32_t cpb = 1u << (pp->b - 6);
    const uint64_t nch = n_blk * cpb;
    const uint32_t seg = (uint32_t)pp->L.seg;
    HIP_TRY(bmq::launch_pack_sizes(dir, nch, seg, ps.rel, ps.segsum, ps.s));
    HIP_TRY(bmq::launch_pack_offsets(ps.segsum, cpb, seg, (uint32_t)n_blk, ps.img_off, ps.s));
    HIP_TRY(bmq::launch_pack_write(dir, pool, cpb, seg, nch, ps.rel, ps.segsum, ps.img_off, ps.img, ps.s));
    HIP_TRY(hipMemcpyAsync(ps.h_img, ps.img_off, (2 * n_blk + 1) * 8, hipMemcpyDeviceToHost, ps.s));
    HIP_TRY(hipEventRecord(ps.packed, ps.s));
    ps.pending = true;
    ps.pend_blocks = std::move(blocks);
    return SV_OK;
}

int pipe_check(const sv_pipe *pp)
{
    if (!pp) return fail(SV_ERR_INVALID, "pipeline is NULL");
    if (pp->poisoned) return fail(SV_ERR_CAPACITY, "pipeline is poisoned by an earlier overflow");
    return SV_OK;
}

}  // namespace

extern "C" {

int sv_pipe_required(const sv_config_t *cfg, int32_t streams, uint64_t *dev_bytes, uint64_t *host_min_bytes)
{
    if (int rc = validate_cfg(cfg)) return rc;
    if (streams < 1 || streams > kMaxPipeStreams) return fail(SV_ERR_INVALID, "streams %d outside [1, 8]", streams);
    const PipeLayout L = pipe_layout(*cfg, streams);
    if (dev_bytes) *dev_bytes = L.total;
    const uint64_t nblk = 1ull << (cfg->n_qubits - cfg->block_qubits);
    const uint64_t cpb = 1ull << (cfg->block_qubits - 6);
    if (host_min_bytes) *host_min_bytes = L.host_small + nblk * align256((8 * cpb + 16) * 5 / 4) + 4096;
    return SV_OK;
}

int sv_pipe_reset(sv_pipe_t *pp);

int sv_pipe_create(const sv_config_t *cfg, int32_t streams, void *dev_ws, uint64_t dev_bytes, void *host_pinned,
                   uint64_t host_bytes, void *hip_stream, sv_pipe_t **out)
{
    if (int rc = validate_cfg(cfg)) return rc;
    if (!out) return fail(SV_ERR_INVALID, "out is NULL");
    if (streams < 1 || streams > kMaxPipeStreams) return fail(SV_ERR_INVALID, "streams %d outside [1, 8]", streams);
    if (cfg->domain == SV_DOMAIN_RAW) return fail(SV_ERR_UNSUPPORTED, "the pipeline stores compressed images only");
    const PipeLayout L = pipe_layout(*cfg, streams);
    if (!dev_ws || ((uintptr_t)dev_ws & 255u) || dev_bytes < L.total)
        return fail(SV_ERR_INVALID, "device workspace must be 256-byte aligned and hold %llu bytes",
                    (unsigned long long)L.total);
    if (!host_pinned || ((uintptr_t)host_pinned & 255u) || host_bytes < L.host_small)
        return fail(SV_ERR_INVALID, "host store must be 256-byte aligned pinned memory of at least %llu bytes",
                    (unsigned long long)L.host_small);
    sv_pipe *pp = new (std::nothrow) sv_pipe;
    if (!pp) return fail(SV_ERR_OOM, "host allocation failed");
    pp->cfg = *cfg;
    pp->n = cfg->n_qubits;
    pp->b = cfg->block_qubits;
    pp->S = streams;
    pp->user = (hipStream_t)hip_stream;
    pp->ws = (uint8_t *)dev_ws;
    pp->L = L;
    pp->host = (uint8_t *)host_pinned + L.host_small;
    pp->host_bytes = host_bytes - L.host_small;
    pp->ops = pp->ws + L.off_ops;
    pp->st.resize(streams);
    const bool scratch = !(cfg->flags & SV_FLAG_NO_SCRATCH);
    for (int i = 0; i < streams; ++i) {
        PipeStream &ps = pp->st[i];
        uint8_t *w = pp->ws + (uint64_t)i * L.per_stream;
        ps.dir[0] = (uint64_t *)(w + L.off_dir[0]);
        ps.dir[1] = (uint64_t *)(w + L.off_dir[1]);
        ps.pool[0] = w + L.off_pool[0];
        ps.pool[1] = w + L.off_pool[1];
        ps.body_off = (uint64_t *)(w + L.off_body);
        if (scratch) {
            ps.scr_re = (float *)(w + L.off_scr_re);
            ps.scr_im = (float *)(w + L.off_scr_im);
        }
        ps.counters = (unsigned long long *)(w + L.off_counters);
        ps.rel = (uint32_t *)(w + L.off_rel);
        ps.segsum = (uint64_t *)(w + L.off_segsum);
        ps.img_off = (uint64_t *)(w + L.off_img_off);
        ps.img = w + L.off_img;
        ps.h_off = (uint64_t *)host_pinned + (uint64_t)i * 3 * (L.gblocks + 1);
        ps.h_img = ps.h_off + (L.gblocks + 1);
        hipError_t e = hipStreamCreateWithFlags(&ps.s, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ps.packed, hipEventDisableTiming);
        if (e != hipSuccess) {
            sv_pipe_destroy(pp);
            return fail(SV_ERR_HIP, "pipeline streams: %s", hipGetErrorString(e));
        }
    }
    if (int rc = sv_pipe_reset(pp)) {
        sv_pipe_destroy(pp);
        return rc;
    }
    *out = pp;
    return SV_OK;
}

// |0...0> (Section 4.2): block 0's image holds the encoded first chunk, every
// other block's image is an all-zero directory.
int sv_pipe_reset(sv_pipe_t *pp)
{
    if (!pp) return fail(SV_ERR_INVALID, "pipeline is NULL");
    for (PipeStream &ps : pp->st) {
        HIP_TRY(hipStreamSynchronize(ps.s));
        ps.pending = false;
    }
    pp->poisoned = false;
    pp->host_used = 0;
    pp->h2d = pp->d2h = 0;
    const uint64_t nblk = 1ull << (pp->n - pp->b);
    const uint64_t cpb = 1ull << (pp->b - 6);
    pp->slots.assign(nblk, sv_pipe::Slot{});
    // block 0 through the device (the encoder's record of amplitude 1)
    PipeStream &ps = pp->st[0];
    HIP_TRY(bmq::launch_fill_u64((uint64_t *)ps.counters, kStageCounters, 0, ps.s));
    HIP_TRY(bmq::launch_init_state(ps.dir[0], cpb, ps.pool[0], ps.counters, codec_params(pp->cfg), ps.s));
    if (int rc = pipe_pack(pp, ps, ps.dir[0], ps.pool[0], 1, std::vector<uint64_t>{0})) return rc;
    if (int rc = pipe_finish(pp, ps)) return rc;
    for (uint64_t k = 1; k < nblk; ++k) {
        if (int rc = pipe_slot(pp, k, 8 * cpb, 0)) return rc;
        std::memset(pp->host + pp->slots[k].off, 0, 8 * cpb);
    }
    HIP_TRY(hipStreamSynchronize(ps.s));
    pp->d2h = 0;
    return SV_OK;
}

int sv_pipe_apply(sv_pipe_t *pp, const sv_plan_t *p, size_t first, size_t count, sv_stage_stats_t *stats)
{
    if (int rc = pipe_check(pp)) return rc;
    if (!p) return fail(SV_ERR_INVALID, "plan is NULL");
    if (p->cfg.n_qubits != pp->n || p->cfg.block_qubits != pp->b || p->cfg.domain != pp->cfg.domain ||
        p->cfg.eb != pp->cfg.eb)
        return fail(SV_ERR_INVALID, "plan and pipeline configurations differ");
    if (first > p->stages.size() || count > p->stages.size() - first)
        return fail(SV_ERR_INVALID, "stage range outside the plan");
    if (pp->cfg.flags & SV_FLAG_NO_SCRATCH)
        for (size_t i = 0; i < count; ++i)
            if (p->stages[first + i].passes.size() > 1)
                return fail(SV_ERR_UNSUPPORTED, "the pipeline runs multi-pass stages through its scratch planes");
    // the plan's operations, once per plan
    if (pp->uploaded_uid != p->uid) {
        const uint64_t ob = p->ops.size() * sizeof(OpDesc);
        if (align256(ob) + p->data.size() * sizeof(float2) > kOpsArenaBytes)
            return fail(SV_ERR_UNSUPPORTED, "plan's fused operations exceed the operation arena");
        if (ob) HIP_TRY(hipMemcpyAsync(pp->ops, p->ops.data(), ob, hipMemcpyHostToDevice, pp->user));
        if (!p->data.empty())
            HIP_TRY(hipMemcpyAsync(pp->ops + align256(ob), p->data.data(), p->data.size() * sizeof(float2),
                                   hipMemcpyHostToDevice, pp->user));
        HIP_TRY(hipStreamSynchronize(pp->user));
        pp->uploaded_uid = p->uid;
    }
    HIP_TRY(hipStreamSynchronize(pp->user));       // earlier work of the caller's stream
    const int n = pp->n, b = pp->b;
    const uint64_t cpb = 1ull << (b - 6);
    const bmq::CodecParams cp = codec_params(pp->cfg);
    const bool scratch = !(pp->cfg.flags & SV_FLAG_NO_SCRATCH);
    for (size_t si = 0; si < count; ++si) {
        const StagePlan &st = p->stages[first + si];
        const auto t0 = std::chrono::steady_clock::now();
        const uint64_t h2d0 = pp->h2d, d2h0 = pp->d2h;
        const int np = (int)st.passes.size();
        if ((size_t)np > kMaxPipePasses) return fail(SV_ERR_UNSUPPORTED, "stage with %d passes", np);
        GroupRun gr;
        group_qubits(n, b, st, gr);
        if ((int)gr.qubits.size() > pp->L.gq)
            return fail(SV_ERR_INVALID, "stage %zu spans %zu qubits; the pipeline stages groups of %d (create it "
                                        "with this inner size and tile)", first + si, gr.qubits.size(), pp->L.gq);
        const int gq = (int)gr.qubits.size();
        const uint64_t nblk = 1ull << (gq - b), nch = 1ull << (gq - 6);
        const uint64_t ngroups = 1ull << gr.outer.size();
        const uint64_t waves = (1ull << (gq - p->t)) * (p->t == 13 ? 8u : 4u);
        const int n_seg = (int)std::min<uint64_t>((uint64_t)bmq::kSegments, waves);
        for (gr.g = 0; gr.g < ngroups; ++gr.g) {
            PipeStream &ps = pp->st[gr.g % pp->S];
            if (int rc = pipe_finish(pp, ps)) return rc;
            // the group's blocks in packed order: block j holds the group
            // qubits above the block bits set to j
            uint64_t fixed = 0;
            for (size_t k = 0; k < gr.outer.size(); ++k) fixed |= ((gr.g >> k) & 1ull) << gr.outer[k];
            std::vector<uint64_t> blocks(nblk);
            uint64_t boff = 0;
            for (uint64_t j = 0; j < nblk; ++j) {
                uint64_t idx = fixed;
                for (int k = 0; k < gq - b; ++k) idx |= ((j >> k) & 1ull) << gr.qubits[b + k];
                const uint64_t blk = idx >> b;
                blocks[j] = blk;
                const sv_pipe::Slot &sl = pp->slots[blk];
                const uint64_t body = sl.body;
                HIP_TRY(hipMemcpyAsync(ps.dir[0] + j * cpb, pp->host + sl.off, 8 * cpb, hipMemcpyHostToDevice, ps.s));
                if (body)
                    HIP_TRY(hipMemcpyAsync(ps.pool[0] + boff, pp->host + sl.off + 8 * cpb, body,
                                           hipMemcpyHostToDevice, ps.s));
                ps.h_off[j] = boff;
                boff += (body + 15) & ~15ull;
                pp->h2d += 8 * cpb + body;
            }
            HIP_TRY(hipMemcpyAsync(ps.body_off, ps.h_off, nblk * 8, hipMemcpyHostToDevice, ps.s));
            HIP_TRY(bmq::launch_rebase_dir(ps.dir[0], nch, (uint32_t)cpb, ps.body_off, ps.s));
            HIP_TRY(bmq::launch_fill_u64((uint64_t *)ps.counters, (uint64_t)np * kStageCounters, 0, ps.s));
            int cur = 0;
            for (int pi = 0; pi < np; ++pi) {
                const PassPlan &pl = st.passes[pi];
                bmq::PassArgs a;
                std::memset(&a, 0, sizeof(a));
                a.n = n;
                a.t = p->t;
                fill_geometry(a, n, p->t, pl, &gr);
                a.dir_packed = 1;
                a.op_begin = pl.op_begin;
                a.op_end = pl.op_end;
                a.in_mode = (!scratch || pi == 0) ? bmq::IO_COMPRESSED : bmq::IO_SCRATCH;
                a.out_mode = (!scratch || pi == np - 1) ? bmq::IO_COMPRESSED : bmq::IO_SCRATCH;
                a.cp = cp;
                a.dir_in = ps.dir[cur];
                a.pool_in = ps.pool[cur];
                a.dir_out = ps.dir[cur ^ 1];
                a.pool_out = ps.pool[cur ^ 1];
                a.pool_cap = pp->L.pool_cap;
                a.n_seg = n_seg;
                a.seg_cap = (pp->L.pool_cap / (uint64_t)n_seg) & ~3ull;
                a.seg_base = 0;
                a.counters = ps.counters + (size_t)pi * kStageCounters;
                a.scr_re = ps.scr_re;
                a.scr_im = ps.scr_im;
                a.ops = (const OpDesc *)pp->ops;
                a.opdata = (const float2 *)(pp->ops + align256(p->ops.size() * sizeof(OpDesc)));
                a.mfma = (pp->cfg.flags & SV_FLAG_NO_MFMA) ? 0 : 1;
                HIP_TRY(bmq::launch_pass(a, ps.s));
                if (a.out_mode == bmq::IO_COMPRESSED) cur ^= 1;
            }
            if (int rc = pipe_pack(pp, ps, ps.dir[cur], ps.pool[cur], nblk, std::move(blocks))) return rc;
        }
        // stage barrier: every group's images are in the host store
        for (PipeStream &ps : pp->st)
            if (int rc = pipe_finish(pp, ps)) return rc;
        for (PipeStream &ps : pp->st) HIP_TRY(hipStreamSynchronize(ps.s));
        if (stats) {
            sv_stage_stats_t &s = stats[si];
            std::memset(&s, 0, sizeof(s));
            s.ms = (float)std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            s.bytes_in = pp->h2d - h2d0;
            s.bytes_out = pp->d2h - d2h0;
            s.bytes_out_host = s.bytes_out;
            s.passes = (uint32_t)np;
            s.launches = (uint32_t)(np << gr.outer.size());
            s.n_gates = (uint32_t)(st.g1 - st.g0);
            s.n_inner = (uint32_t)st.inner.size();
            uint32_t nops = 0;
            for (const auto &pl : st.passes) nops += (uint32_t)(pl.op_end - pl.op_begin);
            s.n_ops = nops;
        }
    }
    return SV_OK;
}

// Copy the host-resident state into a device state of the same
// configuration (its current copy; bodies packed block after block).
int sv_pipe_load(sv_pipe_t *pp, sv_t *sv)
{
    if (int rc = pipe_check(pp)) return rc;
    if (int rc = check_state(sv)) return rc;
    if (sv->n != pp->n || sv->b != pp->b || sv->cfg.domain != pp->cfg.domain || sv->cfg.eb != pp->cfg.eb)
        return fail(SV_ERR_INVALID, "state and pipeline configurations differ");
    if (int rc = resolve_graph(sv)) return rc;
    const uint64_t nblk = 1ull << (pp->n - pp->b), cpb = 1ull << (pp->b - 6);
    uint64_t total = 0;
    for (const auto &sl : pp->slots) total += sl.body;
    if (total > sv->pool_cap) return fail(SV_ERR_CAPACITY, "state's device pool holds %llu bytes, the records %llu",
                                          (unsigned long long)sv->pool_cap, (unsigned long long)total);
    std::vector<uint64_t> off(nblk);
    uint64_t o = 0;
    for (uint64_t k = 0; k < nblk; ++k) {
        const auto &sl = pp->slots[k];
        HIP_TRY(hipMemcpyAsync(sv->dir[sv->cur] + k * cpb, pp->host + sl.off, 8 * cpb, hipMemcpyHostToDevice,
                               sv->stream));
        if (sl.body)
            HIP_TRY(hipMemcpyAsync(sv->pool[sv->cur] + o, pp->host + sl.off + 8 * cpb, sl.body,
                                   hipMemcpyHostToDevice, sv->stream));
        off[k] = o;
        o += sl.body;
    }
    uint64_t *doff = (uint64_t *)(pp->ws + pp->L.off_load_off);
    HIP_TRY(hipMemcpyAsync(doff, off.data(), nblk * 8, hipMemcpyHostToDevice, sv->stream));
    HIP_TRY(bmq::launch_rebase_dir(sv->dir[sv->cur], nblk * cpb, (uint32_t)cpb, doff, sv->stream));
    HIP_TRY(hipStreamSynchronize(sv->stream));
    sv->live_bytes = total;
    sv->live_host = 0;
    sv->reset_pending = false;
    return SV_OK;
}

int sv_pipe_footprint(const sv_pipe_t *pp, uint64_t *record_bytes, uint64_t *image_bytes, uint64_t *host_used,
                      uint64_t *h2d_bytes, uint64_t *d2h_bytes)
{
    if (!pp) return fail(SV_ERR_INVALID, "pipeline is NULL");
    const uint64_t cpb = 1ull << (pp->b - 6);
    uint64_t rec = 0, img = 0;
    for (const auto &sl : pp->slots) {
        rec += sl.body;
        img += 8 * cpb + sl.body;
    }
    if (record_bytes) *record_bytes = rec;
    if (image_bytes) *image_bytes = img;
    if (host_used) *host_used = pp->host_used;
    if (h2d_bytes) *h2d_bytes = pp->h2d;
    if (d2h_bytes) *d2h_bytes = pp->d2h;
    return SV_OK;
}

void sv_pipe_destroy(sv_pipe_t *pp)
{
    if (!pp) return;
    for (PipeStream &ps : pp->st) {
        if (ps.s) (void)hipStreamSynchronize(ps.s);
        if (ps.packed) (void)hipEventDestroy(ps.packed);
        if (ps.s) (void)hipStreamDestroy(ps.s);
    }
    delete pp;
}

}  // extern "C"
