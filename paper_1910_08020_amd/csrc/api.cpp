// C ABI of the engine: contexts, evolution, pseudo-measurement, sampling,
// batching.  See include/lgt.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "lgt_internal.hpp"

using namespace lgt;

namespace {

thread_local std::string g_err;   // errors of calls without a context

struct ProfEvent {
    int kf;
    hipEvent_t a, b;
};

}  // namespace

struct lgt_ctx {
    Lattice lat;
    int dtype = LGT_C64;
    int device = 0;
    void *state = nullptr;
    size_t state_bytes = 0;
    bool own_state = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint32_t ptab[kParityBytes][256];
    uint32_t *ptab_dev = nullptr;
    // per-call tables (device) and their pinned staging buffer
    void *rot_dev = nullptr, *ph_dev = nullptr;
    size_t rot_cap = 0, ph_cap = 0;
    void *stage = nullptr;
    size_t stage_cap = 0;
    hipEvent_t stage_free = nullptr;
    DevInst *inst_dev = nullptr;
    int inst_cap = 0;
    // reductions
    double *partials = nullptr;
    uint64_t *masks_dev = nullptr;
    std::vector<double> partials_host;
    // profiling
    bool profiling = false;
    int prof_stride = 1;
    int64_t prof_seen[KF_COUNT] = {0};
    std::vector<ProfEvent> pending;
    std::vector<hipEvent_t> pool;
    int64_t prof_launches[KF_COUNT] = {0};
    double prof_ms[KF_COUNT] = {0};
    int plan = 0;   // pass plan code (plan_passes), 0 = built-in rule
    int batch_group = 0;   // instances per launch group of batches led by this context, 0 = rule
    int n_anc = 0;  // 1: one ancilla qubit on bit N_l above the links
    // captured launch sequences of batched evolutions, by structure (lgt_set_graphs)
    bool use_graphs = false;
    std::map<std::string, hipGraphExec_t> graphs;
    // X density of states: a state-sized buffer and its one-step tables, made at the first
    // LGT_OBS_XDOS and kept until lgt_destroy
    void *xdos_buf = nullptr;
    void *xdos_tab = nullptr;
    std::string err;
};

namespace {

// qubits of the state: the links, plus the ancilla of an ancilla context
int nq(const lgt_ctx *c) { return c->lat.n_links + c->n_anc; }

constexpr int kMaxPartialBlocks = 2048;
constexpr int kPartialWidth = kMaxPlaq + 1;
constexpr int kMaskChunk = 32;
constexpr int kFlipChunk = 8;

lgt_status fail(lgt_ctx *c, lgt_status s, const std::string &msg)
{
    if (c) c->err = msg;
    else g_err = msg;
    return s;
}

#define HIPCHK(ctx, expr)                                                                      \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail((ctx), LGT_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t elem_bytes(int dtype) { return dtype == LGT_C64 ? 8 : 16; }

// grow a device buffer (stream-ordered: free after the stream drains)
hipError_t ensure_dev(lgt_ctx *c, void **p, size_t *cap, size_t need)
{
    if (*cap >= need) return hipSuccess;
    if (*p) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return e;
        (void)hipFree(*p);
        *p = nullptr;
        *cap = 0;
    }
    size_t sz = std::max(need, (size_t)4096);
    hipError_t e = hipMalloc(p, sz);
    if (e == hipSuccess) *cap = sz;
    return e;
}

hipError_t ensure_stage(lgt_ctx *c, size_t need)
{
    // the previous call's copies out of the staging buffer must have finished
    hipError_t e = hipEventSynchronize(c->stage_free);
    if (e != hipSuccess) return e;
    if (c->stage_cap >= need) return hipSuccess;
    if (c->stage) (void)hipHostFree(c->stage);
    c->stage = nullptr;
    c->stage_cap = 0;
    size_t sz = std::max(need, (size_t)65536);
    e = hipHostMalloc(&c->stage, sz, hipHostMallocDefault);
    if (e == hipSuccess) c->stage_cap = sz;
    return e;
}

// --- profiling: HIP events around launches on the context stream ----------
// two events from the context's pool for one timed launch
hipError_t prof_take(lgt_ctx *c, int kf, ProfEvent &pe)
{
    pe.kf = kf;
    if (c->pool.size() < 2) {
        for (int i = 0; i < 512; ++i) {
            hipEvent_t ev;
            hipError_t e = hipEventCreate(&ev);
            if (e != hipSuccess) return e;
            c->pool.push_back(ev);
        }
    }
    pe.a = c->pool.back(); c->pool.pop_back();
    pe.b = c->pool.back(); c->pool.pop_back();
    return hipSuccess;
}

hipError_t prof_harvest(lgt_ctx *c)
{
    for (auto &pe : c->pending) {
        hipError_t e = hipEventSynchronize(pe.b);
        if (e != hipSuccess) return e;
        float ms = 0;
        e = hipEventElapsedTime(&ms, pe.a, pe.b);
        if (e != hipSuccess) return e;
        c->prof_launches[pe.kf] += 1;
        c->prof_ms[pe.kf] += ms;
        c->pool.push_back(pe.a);
        c->pool.push_back(pe.b);
    }
    c->pending.clear();
    return hipSuccess;
}

template <typename F>
hipError_t timed(lgt_ctx *c, int kf, F &&launch)
{
    if (!c->profiling) return launch();
    if (c->prof_seen[kf]++ % c->prof_stride) return launch();
    ProfEvent pe;
    hipError_t e;
    if (kf == KF_TILE_LOW || kf == KF_TILE_HIGH) {
        // the tile launchers time their kernels themselves, on the dispatch
        e = prof_take(c, kf, pe);
        if (e != hipSuccess) return e;
        LaunchTiming lt{pe.a, pe.b, false};
        g_launch_timing = &lt;
        e = launch();
        g_launch_timing = nullptr;
        if (e != hipSuccess || !lt.used) {
            c->pool.push_back(pe.a);
            c->pool.push_back(pe.b);
            return e;
        }
    } else {
        e = prof_take(c, kf, pe);
        if (e == hipSuccess) e = hipEventRecord(pe.a, c->stream);
        if (e != hipSuccess) return e;
        e = launch();
        if (e != hipSuccess) return e;
        e = hipEventRecord(pe.b, c->stream);
        if (e != hipSuccess) return e;
    }
    c->pending.push_back(pe);
    if (c->pending.size() >= 4096) return prof_harvest(c);
    return hipSuccess;
}

lgt_status check_ctx(lgt_ctx *c)
{
    if (!c) return fail(nullptr, LGT_E_INVALID, "null context");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, LGT_E_DEVICE, "hipSetDevice failed");
    return LGT_OK;
}

// upload rot/phase tables of one instance into dst buffers through the staging buffer
struct Tables {
    std::vector<RotParam<float>> rf;
    std::vector<Cplx<float>> pf;
    std::vector<RotParam<double>> rd;
    std::vector<Cplx<double>> pd;
    size_t rot_bytes = 0, ph_bytes = 0;
};

void make_tables(const Lattice &lat, int dtype, double dt, const std::vector<double> &cx,
                 const std::vector<double> &cz, int order, StepTables &st, Tables &tb)
{
    build_step_tables(lat.n_links, lat.n_plaq, dt, cx.data(), cz.data(), (int)cx.size(), order, st);
    if (dtype == LGT_C64) {
        round_tables_f32(st, lat.n_links, lat.n_plaq, tb.rf, tb.pf);
        tb.rot_bytes = tb.rf.size() * sizeof(RotParam<float>);
        tb.ph_bytes = tb.pf.size() * sizeof(Cplx<float>);
    } else {
        round_tables_f64(st, lat.n_plaq, tb.rd, tb.pd);
        tb.rot_bytes = tb.rd.size() * sizeof(RotParam<double>);
        tb.ph_bytes = tb.pd.size() * sizeof(Cplx<double>);
    }
}

const void *rot_ptr(const Tables &tb, int dtype)
{
    return dtype == LGT_C64 ? (const void *)tb.rf.data() : (const void *)tb.rd.data();
}
const void *ph_ptr(const Tables &tb, int dtype)
{
    return dtype == LGT_C64 ? (const void *)tb.pf.data() : (const void *)tb.pd.data();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// f(0) .. f(n-1) on up to 16 host threads (independent items, any order)
template <typename F>
void parallel_for(int n, F &&f)
{
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nt = std::min(n, (int)std::min(16u, hw));
    if (nt <= 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int> next{0};
    std::vector<std::thread> pool;
    pool.reserve(nt);
    for (int t = 0; t < nt; ++t)
        pool.emplace_back([&] {
            for (int i; (i = next.fetch_add(1)) < n;) f(i);
        });
    for (auto &th : pool) th.join();
}

}  // namespace

namespace lgt {

PassPlan plan_passes(int n_links, int dtype, int plan, int n_inst)
{
    PassPlan p;
    if (n_links <= 12) return p;   // handled on chip by the small-state kernels
    const int big = dtype == LGT_C64 ? 14 : 13;
    // The default depends on the lattice only, so batched and single runs round
    // identically: big low tiles when they give at least 64 workgroups, else 12-bit ones.
    (void)n_inst;
    const bool merge = !(plan & kPlanNoMerge);
    plan &= ~kPlanNoMerge;
    if (plan == 0) {
        // big low tiles when they give at least 64 workgroups and need no register pass
        plan = (n_links >= big && (1 << (n_links - big)) >= 64) ? 2 : 1;
        if (plan == 2) {
            const PassPlan p2 = plan_passes(n_links, dtype, 2 | (merge ? 0 : kPlanNoMerge), n_inst);
            for (int i = 0; i < p2.n_passes; ++i)
                if (p2.pass[i].kind == PASS_HIGH_REG) plan = 1;
            // Complex128 states beyond the Infinity Cache: a high pass over rows of 8
            // amplitudes (128 bytes) streams HBM 10-20% slower than one over rows of 16;
            // where the 14-bit register-bit low tile leaves only rows of 16, take it
            // (32 links: 64.1 instead of 67.4 ms per step)
            if (plan == 2 && dtype != LGT_C64 && n_links >= 26) {
                auto short_rows = [](const PassPlan &q) {
                    for (int i = 0; i < q.n_passes; ++i)
                        if (q.pass[i].kind == PASS_TILE_HIGH && q.pass[i].cb < 4 &&
                            !(q.pass[i].cb == 3 && q.pass[i].h == 11))
                            return true;
                    return false;
                };
                const PassPlan p5 = plan_passes(n_links, dtype, 5 | (merge ? 0 : kPlanNoMerge), n_inst);
                bool p5_ok = !short_rows(p5);
                for (int i = 0; i < p5.n_passes; ++i)
                    if (p5.pass[i].kind == PASS_HIGH_REG) p5_ok = false;
                if (short_rows(p2) && p5_ok) return p5;
            }
            if (plan == 2) return p2;
        }
    }
    if (plan == 4) {
        // the 12-bit LDS tile with 256 threads followed by register passes of <= 6 bits
        p.pass[p.n_passes++] = Pass{PASS_LOW12, 0, 12, 0};
        const int rest = n_links - 12, hmax = dtype == LGT_C64 ? 6 : 5;
        const int nh = (rest + hmax - 1) / hmax;
        int q = 12;
        for (int i = 0; i < nh; ++i) {
            const int h = rest / nh + (i < rest % nh ? 1 : 0);
            p.pass[p.n_passes++] = Pass{PASS_HIGH_REG, q, h, 0};
            q += h;
        }
        return p;
    }
    // persistent tile passes: one low tile (12 bits for plan 1, the largest otherwise), then
    // as few high tiles as possible with the longest (plans 1, 2) or shortest (3) rows;
    // chunks no tile pass takes go to register passes
    // plan 5: complex128 low tiles of 14 bits (one bit in registers)
    int low = (plan == 1 || n_links < big) ? 12 : big;
    if (plan == 5 && dtype != LGT_C64 && n_links >= 15) low = 14;
    p.pass[p.n_passes++] = Pass{PASS_TILE_LOW, 0, low, 0};
    const bool long_rows = plan != 3;
    const int rest = n_links - low, reg_max = dtype == LGT_C64 ? 6 : 5;
    // complex128 high tiles may keep rows of 64 bytes, which lets one tile rotate 11 bits
    const int cb_lo = dtype == LGT_C64 ? 4 : 2;
    // 512-byte rows only for complex64 states beyond the 256 MB Infinity Cache, where the
    // passes stream HBM (one of the 28-link high passes runs 7-13% faster with them)
    const int cb_hi = dtype == LGT_C64 ? (n_links >= 26 ? 6 : 5) : 4;
    // most bits one high tile rotates: 10 (complex64, 128-byte rows, 16 waves), 11
    // (complex128: 128-byte rows with one bit in registers, or 64-byte rows; 8 waves)
    const int hmax = dtype == LGT_C64 ? 10 : 11;
    const int nh = (rest + hmax - 1) / hmax;
    int q = low;
    for (int i = 0; i < nh; ++i) {
        const int h = rest / nh + (i < rest % nh ? 1 : 0);
        int cb = -1;
        for (int k = 0; k <= cb_hi - cb_lo && cb < 0; ++k) {
            const int c = long_rows ? cb_hi - k : cb_lo + k;
            if (pass_wave_bits(dtype, 0, h, c) >= 0 && pass_offsets_fit(dtype, n_links, 0, q, h, c)) cb = c;
        }
        if (cb >= 0) p.pass[p.n_passes++] = Pass{PASS_TILE_HIGH, q, h, cb};
        else if (h <= reg_max) p.pass[p.n_passes++] = Pass{PASS_HIGH_REG, q, h, 0};
        else return plan_passes(n_links, dtype, 4, n_inst);
        q += h;
    }
    // steps merge at the first and the last pass: keep a register pass out of those places
    const int last = p.n_passes - 1;
    if (last >= 2 && p.pass[last].kind == PASS_HIGH_REG)
        for (int i = last - 1; i >= 1; --i)
            if (p.pass[i].kind == PASS_TILE_HIGH) {
                std::swap(p.pass[i], p.pass[last]);
                break;
            }
    p.merge = merge && last >= 1 && p.pass[last].kind != PASS_HIGH_REG;
    return p;
}

std::string describe_plan(const PassPlan &p, int n_links)
{
    if (p.n_passes == 0) return "small(" + std::to_string(n_links) + " links on chip)";
    std::string s;
    for (int i = 0; i < p.n_passes; ++i) {
        const Pass &ps = p.pass[i];
        if (i) s += " | ";
        switch (ps.kind) {
        case PASS_LOW12: s += "low12"; break;
        case PASS_TILE_LOW: s += "tile_low" + std::to_string(ps.h); break;
        case PASS_TILE_HIGH:
            s += "tile_high(q" + std::to_string(ps.q0) + ",h" + std::to_string(ps.h) + ",rows" +
                 std::to_string(1 << ps.cb) + ")";
            break;
        default: s += "reg_high(q" + std::to_string(ps.q0) + ",h" + std::to_string(ps.h) + ")";
        }
    }
    if (p.merge) s += " ; steps merged";
    return s;
}

hipError_t enqueue_fused_steps(int dtype, int n, int n_plaq, const DevInst *dev_inst, int n_inst,
                               int count, int pre_first, int post_off, const uint8_t *forms,
                               int plan_sel, hipStream_t st, void *prof_ctx)
{
    FusedCursor cur;
    return enqueue_fused_range(dtype, n, n_plaq, dev_inst, n_inst, count, 0, count, pre_first,
                               post_off, forms, plan_sel, st, prof_ctx, cur);
}

hipError_t enqueue_fused_range(int dtype, int n, int n_plaq, const DevInst *dev_inst, int n_inst,
                               int count, int j_begin, int j_end, int pre_first, int post_off,
                               const uint8_t *forms, int plan_sel, hipStream_t st,
                               void *prof_ctx, FusedCursor &cur)
{
    lgt_ctx *pc = (lgt_ctx *)prof_ctx;
    auto run = [&](int kf, auto &&launch) -> hipError_t {
        if (pc && pc->profiling) return timed(pc, kf, launch);
        return launch();
    };
    if (j_begin < 0 || j_end > count || j_begin > j_end) return hipErrorInvalidValue;
    if (small_supported(dtype, n)) {
        // one kernel runs every step: no partial ranges
        if (j_begin != 0 || j_end != count) return hipErrorInvalidValue;
        // the small kernel reads phase[ph0] first when pre_first >= 0
        return run(KF_SMALL, [&] {
            return launch_small(dtype, dev_inst, n_inst, n, count, pre_first >= 0 ? 1 : 0, n_plaq, st);
        });
    }
    const PassPlan plan = plan_passes(n, dtype, plan_sel, n_inst);
    const int np = plan.n_passes;
    // merged plans walk the passes forwards and backwards in turn, so a step's last pass
    // is the next step's first: one launch applies both rotations around the phase
    bool fwd = cur.fwd, merged_in = cur.merged_in;
    for (int j = j_begin; j < j_end; ++j) {
        auto form_at = [&](int i) { return forms ? ((forms[i] & 3) ? (forms[i] & 3) : 1) : 3; };
        const bool merge_out = plan.merge && j + 1 < count;
        const int fm = form_at(j) | (merge_out ? form_at(j + 1) << 2 : 0);
        for (int k = merged_in ? 1 : 0; k < np; ++k) {
            const Pass &ps = plan.pass[fwd ? k : np - 1 - k];
            const bool last = (k == np - 1);
            const int post = last ? j + post_off : -1;
            const int pre = (k == 0 && j == 0) ? pre_first : -1;
            const int mg = (last && merge_out) ? 1 : 0;
            hipError_t e;
            switch (ps.kind) {
            case PASS_LOW12:
                if (mg) return hipErrorInvalidValue;   // only tile passes merge steps
                e = run(KF_LOW, [&] {
                    return launch_low(dtype, dev_inst, n_inst, n, 12, j, pre, post, n_plaq, st);
                });
                break;
            case PASS_TILE_LOW:
                e = run(KF_TILE_LOW, [&] {
                    return launch_tile(dtype, dev_inst, n_inst, n, 1, 0, ps.h, 0, j, pre, post, n_plaq, fm, mg, st);
                });
                break;
            case PASS_TILE_HIGH:
                e = run(KF_TILE_HIGH, [&] {
                    return launch_tile(dtype, dev_inst, n_inst, n, 0, ps.q0, ps.h, ps.cb, j, pre, post, n_plaq, fm, mg, st);
                });
                break;
            default:
                // register passes never come first and never merge steps
                if (pre >= 0 || mg) return hipErrorInvalidValue;
                e = run(KF_HIGH, [&] {
                    return launch_high(dtype, dev_inst, n_inst, n, ps.q0, ps.h, j, post, n_plaq, st);
                });
            }
            if (e != hipSuccess) return e;
        }
        merged_in = merge_out;
        if (plan.merge) fwd = !fwd;
    }
    cur.fwd = fwd;
    cur.merged_in = merged_in;
    return hipSuccess;
}

}  // namespace lgt

// graphs kept per context for batched evolutions
static constexpr size_t kMaxGraphs = 64;
// steps in the first chunk of FP32 phase rows a run rounds and uploads (then 2x, 4x, ...)
static constexpr int kFirstChunk = 32;
// state bytes of a batch that stay in the Infinity Cache between its passes
static constexpr size_t kCacheStateBytes = (size_t)160 << 20;

static hipError_t enqueue_fused(lgt_ctx *c, const DevInst *dev_inst, int n_inst, int count,
                                int pre_phase, const uint8_t *forms)
{
    return enqueue_fused_steps(c->dtype, c->lat.n_links, c->lat.n_plaq, dev_inst, n_inst, count,
                               pre_phase ? 0 : -1, pre_phase, forms, c->plan, c->stream, c);
}

// kFormTan: tan form (u == 1) of the factored link rotation, kFormCot: cot form
static void or_forms(const StepTables &st, std::vector<uint8_t> &forms)
{
    if (forms.size() < (size_t)st.n_steps) forms.resize(st.n_steps, 0);
    for (int j = 0; j < st.n_steps; ++j) forms[j] |= (st.rot_u[j] == 1.0) ? kFormTan : kFormCot;
}

static lgt_status create_common(int d, const int *L, int periodic, lgt_dtype dtype, void *buf,
                                size_t bytes, void *stream, int n_anc, lgt_ctx **out)
{
    if (!out) return fail(nullptr, LGT_E_INVALID, "null output pointer");
    *out = nullptr;
    if (dtype != LGT_C64 && dtype != LGT_C128) return fail(nullptr, LGT_E_INVALID, "bad dtype");
    if (periodic != 1)
        return fail(nullptr, periodic == 0 ? LGT_E_UNSUPPORTED : LGT_E_INVALID,
                    "only periodic lattices (tori) are supported");
    Lattice lat;
    std::string why = build_lattice(d, L, lat);
    if (!why.empty()) {
        bool unsup = why.find("too many") != std::string::npos;
        return fail(nullptr, unsup ? LGT_E_UNSUPPORTED : LGT_E_INVALID, why);
    }
    std::unique_ptr<lgt_ctx> c(new (std::nothrow) lgt_ctx());
    if (!c) return fail(nullptr, LGT_E_OOM, "host allocation failed");
    c->lat = std::move(lat);
    c->dtype = dtype;
    c->n_anc = n_anc;
    c->state_bytes = ((size_t)1 << nq(c.get())) * elem_bytes(dtype);
    if (hipGetDevice(&c->device) != hipSuccess) return fail(nullptr, LGT_E_DEVICE, "no HIP device");
    if (buf) {
        if (bytes < c->state_bytes) return fail(nullptr, LGT_E_INVALID, "external buffer too small");
        if ((uintptr_t)buf % 256) return fail(nullptr, LGT_E_INVALID, "external buffer not 256-byte aligned");
        c->state = buf;
    } else {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && c->state_bytes + (64u << 20) > free_b)
            return fail(nullptr, LGT_E_OOM, "state does not fit in free device memory");
        if (hipMalloc(&c->state, c->state_bytes) != hipSuccess)
            return fail(nullptr, LGT_E_OOM, "hipMalloc of the state failed");
        c->own_state = true;
    }
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            lgt_destroy(c.release());
            return fail(nullptr, LGT_E_DEVICE, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    build_parity_tables(c->lat, c->ptab);
    if (const char *e = std::getenv("LGT_PASS_PLAN")) c->plan = std::atoi(e);   // debugging override
    lgt_ctx *raw = c.get();
    auto bail = [&](const char *m) {
        lgt_destroy(c.release());
        return fail(nullptr, LGT_E_DEVICE, m);
    };
    if (hipMalloc((void **)&raw->ptab_dev, sizeof(raw->ptab)) != hipSuccess) return bail("hipMalloc tables");
    if (hipMemcpy(raw->ptab_dev, raw->ptab, sizeof(raw->ptab), hipMemcpyHostToDevice) != hipSuccess)
        return bail("upload tables");
    if (hipMalloc((void **)&raw->partials, sizeof(double) * kMaxPartialBlocks * kPartialWidth) != hipSuccess)
        return bail("hipMalloc partials");
    if (hipMalloc((void **)&raw->masks_dev, sizeof(uint64_t) * 64) != hipSuccess) return bail("hipMalloc masks");
    if (hipEventCreateWithFlags(&raw->stage_free, hipEventDisableTiming) != hipSuccess) return bail("event");
    if (hipEventRecord(raw->stage_free, raw->stream) != hipSuccess) return bail("event record");
    raw->partials_host.resize((size_t)kMaxPartialBlocks * kPartialWidth);
    lgt_status s = lgt_reset(raw, LGT_INIT_PLUS, 0);
    if (s != LGT_OK) {
        std::string m = raw->err;
        lgt_destroy(c.release());
        return fail(nullptr, s, m);
    }
    *out = c.release();
    return LGT_OK;
}

extern "C" {

lgt_status lgt_create(int d, const int *L, int periodic, lgt_dtype dtype, lgt_ctx **out)
{
    return create_common(d, L, periodic, dtype, nullptr, 0, nullptr, 0, out);
}

lgt_status lgt_create_ancilla(int d, const int *L, int periodic, lgt_dtype dtype, lgt_ctx **out)
{
    return create_common(d, L, periodic, dtype, nullptr, 0, nullptr, 1, out);
}

lgt_status lgt_create_ex(int d, const int *L, int periodic, lgt_dtype dtype, void *dev_buf,
                         size_t bytes, void *stream, lgt_ctx **out)
{
    if (!dev_buf) return fail(nullptr, LGT_E_INVALID, "null device buffer");
    return create_common(d, L, periodic, dtype, dev_buf, bytes, stream, 0, out);
}

lgt_status lgt_destroy(lgt_ctx *c)
{
    if (!c) return LGT_OK;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto &pe : c->pending) {
        (void)hipEventDestroy(pe.a);
        (void)hipEventDestroy(pe.b);
    }
    for (auto ev : c->pool) (void)hipEventDestroy(ev);
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second);
    if (c->own_state && c->state) (void)hipFree(c->state);
    if (c->ptab_dev) (void)hipFree(c->ptab_dev);
    if (c->rot_dev) (void)hipFree(c->rot_dev);
    if (c->ph_dev) (void)hipFree(c->ph_dev);
    if (c->inst_dev) (void)hipFree(c->inst_dev);
    if (c->partials) (void)hipFree(c->partials);
    if (c->masks_dev) (void)hipFree(c->masks_dev);
    if (c->xdos_buf) (void)hipFree(c->xdos_buf);
    if (c->xdos_tab) (void)hipFree(c->xdos_tab);
    if (c->stage) (void)hipHostFree(c->stage);
    if (c->stage_free) (void)hipEventDestroy(c->stage_free);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return LGT_OK;
}

lgt_status lgt_info(const lgt_ctx *c, lgt_info_t *o)
{
    if (!c || !o) return fail(nullptr, LGT_E_INVALID, "null argument");
    const Lattice &l = c->lat;
    o->d = l.d;
    for (int i = 0; i < 3; ++i) o->L[i] = i < l.d ? l.L[i] : 1;
    o->n_links = l.n_links;
    o->n_qubits = nq(c);
    o->n_plaq = l.n_plaq;
    o->n_sites = l.n_sites;
    o->dtype = (lgt_dtype)c->dtype;
    o->state_bytes = c->state_bytes;
    o->state = c->state;
    o->stream = c->stream;
    o->plaq_masks = l.plaq_mask.data();
    o->plaq_links = l.plaq_links.data();
    o->star_masks = l.star_mask.data();
    o->link_plaqs = l.link_plaqs.data();
    return LGT_OK;
}

lgt_status lgt_lattice_query(int d, const int *L, int *n_links, int *n_plaq, int *n_sites,
                             int32_t *plaq_links, uint64_t *star_masks)
{
    Lattice lat;
    std::string why = build_lattice(d, L, lat);
    if (!why.empty())
        return fail(nullptr, why.find("too many") != std::string::npos ? LGT_E_UNSUPPORTED : LGT_E_INVALID, why);
    if (n_links) *n_links = lat.n_links;
    if (n_plaq) *n_plaq = lat.n_plaq;
    if (n_sites) *n_sites = lat.n_sites;
    if (plaq_links) std::memcpy(plaq_links, lat.plaq_links.data(), sizeof(int32_t) * lat.plaq_links.size());
    if (star_masks) std::memcpy(star_masks, lat.star_mask.data(), sizeof(uint64_t) * lat.star_mask.size());
    return LGT_OK;
}

lgt_status lgt_wilson_mask(const lgt_ctx *c, int site, int mu, int nu, int a, int b, uint64_t *mask)
{
    if (!c || !mask) return fail(nullptr, LGT_E_INVALID, "null argument");
    const Lattice &l = c->lat;
    if (site < 0 || site >= l.n_sites || mu < 0 || nu <= mu || nu >= l.d || a < 1 || b < 1 ||
        a > l.L[mu] || b > l.L[nu])
        return fail(const_cast<lgt_ctx *>(c), LGT_E_INVALID, "bad Wilson loop geometry");
    *mask = region_mask(l, site, mu, nu, a, b);
    return LGT_OK;
}

lgt_status lgt_line_mask(const lgt_ctx *c, int site, int mu, uint64_t *mask)
{
    if (!c || !mask) return fail(nullptr, LGT_E_INVALID, "null argument");
    if (site < 0 || site >= c->lat.n_sites || mu < 0 || mu >= c->lat.d)
        return fail(const_cast<lgt_ctx *>(c), LGT_E_INVALID, "bad line");
    *mask = line_mask(c->lat, site, mu);
    return LGT_OK;
}

lgt_status lgt_contour_mask(const lgt_ctx *c, int k, uint64_t *mask)
{
    if (!c || !mask) return fail(nullptr, LGT_E_INVALID, "null argument");
    if (k < 1 || k > 3) return fail(const_cast<lgt_ctx *>(c), LGT_E_INVALID, "contour index must be 1, 2 or 3");
    const uint64_t m = contour_mask(c->lat, k);
    if (!m) return fail(const_cast<lgt_ctx *>(c), LGT_E_UNSUPPORTED, "the contour wraps around this torus");
    *mask = m;
    return LGT_OK;
}

lgt_status lgt_thooft_mask(const lgt_ctx *c, int mu, uint64_t *mask)
{
    if (!c || !mask) return fail(nullptr, LGT_E_INVALID, "null argument");
    if (mu < 0 || mu >= c->lat.d) return fail(const_cast<lgt_ctx *>(c), LGT_E_INVALID, "bad direction");
    *mask = thooft_mask(c->lat, mu);
    return LGT_OK;
}

lgt_status lgt_apply_pauli(lgt_ctx *c, uint64_t xmask, uint64_t zmask)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    const int n = nq(c);
    if ((xmask >> n) || (zmask >> n)) return fail(c, LGT_E_INVALID, "mask has bits beyond N");
    HIPCHK(c, launch_pauli(c->dtype, c->state, n, xmask, zmask, c->stream));
    return LGT_OK;
}

lgt_status lgt_apply_gate(lgt_ctx *c, lgt_gate gate, int q0, int q1, double angle)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    const int n = nq(c);
    const bool two = gate == LGT_GATE_CNOT || gate == LGT_GATE_CZ;
    if (q0 < 0 || q0 >= n || (two && (q1 < 0 || q1 >= n || q1 == q0)))
        return fail(c, LGT_E_INVALID, "qubit index out of range");
    switch (gate) {
    case LGT_GATE_H:
        HIPCHK(c, timed(c, KF_GATE_H, [&] { return launch_gate_h(c->dtype, c->state, n, q0, c->stream); }));
        break;
    case LGT_GATE_X:
        HIPCHK(c, launch_pauli(c->dtype, c->state, n, 1ull << q0, 0, c->stream));
        break;
    case LGT_GATE_RX:
        HIPCHK(c, timed(c, KF_GATE_RX, [&] { return launch_gate_rx(c->dtype, c->state, n, q0, angle, c->stream); }));
        break;
    case LGT_GATE_RZ:
        HIPCHK(c, timed(c, KF_GATE_RZ, [&] { return launch_gate_rz(c->dtype, c->state, n, q0, angle, c->stream); }));
        break;
    case LGT_GATE_CNOT:
        HIPCHK(c, timed(c, KF_GATE_CNOT, [&] { return launch_gate_cnot(c->dtype, c->state, n, q0, q1, c->stream); }));
        break;
    case LGT_GATE_CZ:
        HIPCHK(c, timed(c, KF_GATE_CZ, [&] { return launch_gate_cz(c->dtype, c->state, n, q0, q1, c->stream); }));
        break;
    default:
        return fail(c, LGT_E_INVALID, "unknown gate");
    }
    return LGT_OK;
}

static lgt_status ground_circuit(lgt_ctx *c);

lgt_status lgt_reset(lgt_ctx *c, lgt_init init, uint64_t basis_index)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    const int n = c->lat.n_links;
    if (init == LGT_INIT_BASIS && (basis_index >> nq(c)))
        return fail(c, LGT_E_INVALID, "basis index >= 2^(number of qubits)");
    if (init == LGT_INIT_BASIS && c->n_anc) {
        HIPCHK(c, timed(c, KF_INIT, [&] {
            return launch_init(c->dtype, c->state, nq(c), init, basis_index, 0.0, c->ptab_dev, c->stream);
        }));
        return LGT_OK;
    }
    if (init == LGT_INIT_ZGROUND_CIRCUIT) {
        if (!c->n_anc) return fail(c, LGT_E_UNSUPPORTED, "the projection circuit needs an ancilla context");
        if ((s = lgt_reset(c, LGT_INIT_PLUS, 0))) return s;
        return ground_circuit(c);
    }
    double amp = 0;
    if (init == LGT_INIT_PLUS) {
        amp = std::ldexp(1.0, -n / 2) * ((n & 1) ? std::sqrt(0.5) : 1.0);
    } else if (init == LGT_INIT_BASIS) {
        if (basis_index >> n) return fail(c, LGT_E_INVALID, "basis index >= 2^N");
    } else if (init == LGT_INIT_ZGROUND) {
        // uniform superposition of the 2^(N - rank) basis states with every U_p = +1
        std::vector<uint64_t> rows(c->lat.plaq_mask);
        int rank = 0;
        for (int bit = 0; bit < n; ++bit) {
            auto it = std::find_if(rows.begin(), rows.end(), [&](uint64_t r) { return (r >> bit) & 1; });
            if (it == rows.end()) continue;
            uint64_t piv = *it;
            rows.erase(it);
            for (auto &r : rows)
                if ((r >> bit) & 1) r ^= piv;
            ++rank;
        }
        const int k = n - rank;
        amp = std::ldexp(1.0, -k / 2) * ((k & 1) ? std::sqrt(0.5) : 1.0);
    } else {
        return fail(c, LGT_E_INVALID, "bad init kind");
    }
    // an ancilla context: the lattice state on the ancilla-|0> half, the other half cleared
    if (c->n_anc)
        HIPCHK(c, timed(c, KF_PROJECT, [&] {
            return launch_project_scale(c->dtype, c->state, nq(c), 1ull << n, 1.0, c->stream);
        }));
    HIPCHK(c, timed(c, KF_INIT, [&] {
        return launch_init(c->dtype, c->state, n, init, basis_index, amp, c->ptab_dev, c->stream);
    }));
    return LGT_OK;
}

static lgt_status evolve_fused(lgt_ctx *c, double dt, const std::vector<double> &cx,
                               const std::vector<double> &cz, lgt_order order);

lgt_status lgt_evolve(lgt_ctx *c, const lgt_schedule *sched, lgt_order order, lgt_form form,
                      int64_t first_step, int64_t count)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    if (order != LGT_ORDER_TROTTER && order != LGT_ORDER_SYMMETRIC)
        return fail(c, LGT_E_INVALID, "bad order");
    if (form != LGT_FORM_FUSED && form != LGT_FORM_CIRCUIT && form != LGT_FORM_ANCILLA &&
        form != LGT_FORM_CONTROLLED)
        return fail(c, LGT_E_UNSUPPORTED, "unknown form");
    const bool anc_form = form == LGT_FORM_ANCILLA || form == LGT_FORM_CONTROLLED;
    if (anc_form != (c->n_anc == 1))
        return fail(c, LGT_E_UNSUPPORTED, anc_form ? "this form needs an ancilla context"
                                                   : "an ancilla context runs the ancilla forms only");
    double dt = 0;
    std::vector<double> cx, cz;
    std::string why = schedule_coeffs(sched, first_step, count, dt, cx, cz);
    if (!why.empty()) return fail(c, LGT_E_INVALID, why);
    if (count == 0) return LGT_OK;
    const Lattice &lat = c->lat;
    const int n = lat.n_links;
    StepTables st;
    if (anc_form) {
        // eq. (ara) for every plaquette with the ancilla (bit n) as the CNOT target; the
        // symmetric order merges neighbouring half steps like the other forms
        build_step_tables(n, lat.n_plaq, dt, cx.data(), cz.data(), (int)count, order, st);
        const int nt = nq(c), a = n;
        const bool ctl = form == LGT_FORM_CONTROLLED;
        std::vector<double> theta(st.n_phase);
        if (order == LGT_ORDER_TROTTER) {
            for (int64_t j = 0; j < count; ++j) theta[j] = dt * cz[j];
        } else {
            theta[0] = 0.5 * dt * cz[0];
            for (int64_t j = 0; j < count; ++j)
                theta[j + 1] = (j + 1 < count) ? 0.5 * dt * (cz[j] + cz[j + 1]) : 0.5 * dt * cz[j];
        }
        auto gadgets = [&](double th) -> hipError_t {
            for (int p = 0; p < lat.n_plaq; ++p) {
                const int32_t *l = &lat.plaq_links[4 * p];
                for (int k = 0; k < 4; ++k) {
                    hipError_t e = timed(c, KF_GATE_CNOT, [&] { return launch_gate_cnot(c->dtype, c->state, nt, l[k], a, c->stream); });
                    if (e != hipSuccess) return e;
                }
                hipError_t e = timed(c, KF_GATE_RZ, [&] { return launch_gate_rz(c->dtype, c->state, nt, a, -2.0 * th, c->stream); });
                if (e != hipSuccess) return e;
                for (int k = 3; k >= 0; --k) {
                    e = timed(c, KF_GATE_CNOT, [&] { return launch_gate_cnot(c->dtype, c->state, nt, l[k], a, c->stream); });
                    if (e != hipSuccess) return e;
                }
            }
            return hipSuccess;
        };
        // R_x on every link; controlled: between two CZ(ancilla, link), which reverses the
        // rotation on the ancilla-|1> half
        auto links = [&](double alpha) -> hipError_t {
            for (int q = 0; q < n; ++q) {
                hipError_t e = hipSuccess;
                if (ctl) e = timed(c, KF_GATE_CZ, [&] { return launch_gate_cz(c->dtype, c->state, nt, a, q, c->stream); });
                if (e == hipSuccess)
                    e = timed(c, KF_GATE_RX, [&] { return launch_gate_rx(c->dtype, c->state, nt, q, -2.0 * alpha, c->stream); });
                if (e == hipSuccess && ctl)
                    e = timed(c, KF_GATE_CZ, [&] { return launch_gate_cz(c->dtype, c->state, nt, a, q, c->stream); });
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        };
        const int pre = st.pre_phase;
        if (pre) HIPCHK(c, gadgets(theta[0]));
        for (int64_t j = 0; j < count; ++j) {
            HIPCHK(c, links(dt * cx[j]));
            HIPCHK(c, gadgets(theta[j + pre]));
        }
        return LGT_OK;
    }
    if (form == LGT_FORM_CIRCUIT) {
        // one pass per gate; the symmetric order merges neighbouring half steps
        // like the fused path (rewritten product after eq. (s))
        build_step_tables(n, lat.n_plaq, dt, cx.data(), cz.data(), (int)count, order, st);
        std::vector<double> theta(st.n_phase);
        if (order == LGT_ORDER_TROTTER) {
            for (int64_t j = 0; j < count; ++j) theta[j] = dt * cz[j];
        } else {
            theta[0] = 0.5 * dt * cz[0];
            for (int64_t j = 0; j < count; ++j)
                theta[j + 1] = (j + 1 < count) ? 0.5 * dt * (cz[j] + cz[j + 1]) : 0.5 * dt * cz[j];
        }
        auto gadgets = [&](double th) -> hipError_t {
            for (int p = 0; p < lat.n_plaq; ++p) {
                const int32_t *l = &lat.plaq_links[4 * p];
                const int tq = l[3];
                for (int k = 0; k < 3; ++k) {
                    hipError_t e = timed(c, KF_GATE_CNOT, [&] { return launch_gate_cnot(c->dtype, c->state, n, l[k], tq, c->stream); });
                    if (e != hipSuccess) return e;
                }
                hipError_t e = timed(c, KF_GATE_RZ, [&] { return launch_gate_rz(c->dtype, c->state, n, tq, -2.0 * th, c->stream); });
                if (e != hipSuccess) return e;
                for (int k = 2; k >= 0; --k) {
                    e = timed(c, KF_GATE_CNOT, [&] { return launch_gate_cnot(c->dtype, c->state, n, l[k], tq, c->stream); });
                    if (e != hipSuccess) return e;
                }
            }
            return hipSuccess;
        };
        const int pre = st.pre_phase;
        if (pre) HIPCHK(c, gadgets(theta[0]));
        for (int64_t j = 0; j < count; ++j) {
            const double alpha = dt * cx[j];
            for (int q = 0; q < n; ++q)
                HIPCHK(c, timed(c, KF_GATE_RX, [&] { return launch_gate_rx(c->dtype, c->state, n, q, -2.0 * alpha, c->stream); }));
            HIPCHK(c, gadgets(theta[j + pre]));
        }
        return LGT_OK;
    }
    return evolve_fused(c, dt, cx, cz, order);
}

// fused form: the whole call as one chain of pass launches.  The FP32 phase rows are
// rounded and uploaded in chunks of doubling size, each chunk's launches enqueued as soon as
// its rows are staged, so the device starts on the first steps while the host rounds the rest.
static lgt_status evolve_fused(lgt_ctx *c, double dt, const std::vector<double> &cx,
                               const std::vector<double> &cz, lgt_order order)
{
    const Lattice &lat = c->lat;
    const int64_t count = (int64_t)cx.size();
    if (count > (1 << 24)) return fail(c, LGT_E_INVALID, "too many steps in one call");
    const bool f32 = c->dtype == LGT_C64;
    StepTables st;
    build_step_tables(lat.n_links, lat.n_plaq, dt, cx.data(), cz.data(), (int)count, order, st);
    Tables tb;
    std::vector<long double> gain;
    if (f32) {
        round_rot_f32(st, lat.n_links, tb.rf, gain);
        tb.pf.assign((size_t)st.n_phase * (lat.n_plaq + 1), Cplx<float>{});
    } else {
        round_tables_f64(st, lat.n_plaq, tb.rd, tb.pd);
    }
    const size_t rot_row = f32 ? sizeof(RotParam<float>) : sizeof(RotParam<double>);
    const size_t ph_row = (f32 ? sizeof(Cplx<float>) : sizeof(Cplx<double>)) * (lat.n_plaq + 1);
    tb.rot_bytes = rot_row * (size_t)count;
    tb.ph_bytes = ph_row * (size_t)st.n_phase;
    const size_t rb = align256(tb.rot_bytes), pb = align256(tb.ph_bytes);
    HIPCHK(c, ensure_stage(c, rb + pb + 256));
    HIPCHK(c, ensure_dev(c, &c->rot_dev, &c->rot_cap, rb));
    HIPCHK(c, ensure_dev(c, &c->ph_dev, &c->ph_cap, pb));
    if (c->inst_cap < 1) {
        void *p = c->inst_dev;
        size_t cap = 0;
        HIPCHK(c, ensure_dev(c, &p, &cap, sizeof(DevInst)));
        c->inst_dev = (DevInst *)p;
        c->inst_cap = 1;
    }
    char *stg = (char *)c->stage;
    DevInst di{};
    di.psi = c->state;
    di.rot = c->rot_dev;
    di.phase = c->ph_dev;
    di.ptab = c->ptab_dev;
    di.step0 = 0;
    di.ph0 = 0;
    di.n_total = (int)count;
    std::memcpy(stg + rb + pb, &di, sizeof(di));
    HIPCHK(c, hipMemcpyAsync(c->inst_dev, stg + rb + pb, sizeof(DevInst), hipMemcpyHostToDevice, c->stream));
    std::vector<uint8_t> forms;
    or_forms(st, forms);
    const int n = lat.n_links, total = (int)count, pre = st.pre_phase;
    // the single on-chip kernel runs every step at once
    const bool chunked = !small_supported(c->dtype, n);
    FusedCursor cur;
    PhaseRounding prnd;   // phase-row rounding state carried from chunk to chunk
    for (int j0 = 0, len = kFirstChunk; j0 < total; j0 += len, len *= 2) {
        const int j1 = chunked ? (int)std::min<int64_t>(total, (int64_t)j0 + len) : total;
        // rows read by the launches of steps [j0, j1): link layers j0 .. j1 (a merged launch
        // ending the chunk also rotates step j1) and phase rows up to j1 - 1 + pre; the
        // previous chunk already sent link layer j0
        const int r0 = j0 == 0 ? 0 : j0 + 1, r1 = std::min(total, j1 + 1);
        const int k0 = j0 == 0 ? 0 : j0 + pre, k1 = j1 + pre;
        if (f32) round_phase_f32(st, lat.n_plaq, gain, k0, k1, tb.pf, prnd);
        const char *rsrc = (const char *)rot_ptr(tb, c->dtype), *psrc = (const char *)ph_ptr(tb, c->dtype);
        if (r1 > r0) {
            const size_t off = rot_row * r0, len_b = rot_row * (size_t)(r1 - r0);
            std::memcpy(stg + off, rsrc + off, len_b);
            HIPCHK(c, hipMemcpyAsync((char *)c->rot_dev + off, stg + off, len_b, hipMemcpyHostToDevice, c->stream));
        }
        if (k1 > k0) {
            const size_t off = ph_row * k0, len_b = ph_row * (size_t)(k1 - k0);
            std::memcpy(stg + rb + off, psrc + off, len_b);
            HIPCHK(c, hipMemcpyAsync((char *)c->ph_dev + off, stg + rb + off, len_b, hipMemcpyHostToDevice, c->stream));
        }
        HIPCHK(c, enqueue_fused_range(c->dtype, n, lat.n_plaq, c->inst_dev, 1, total, j0, j1,
                                      pre ? 0 : -1, pre, forms.data(), c->plan, c->stream, c, cur));
        if (!chunked) break;
    }
    HIPCHK(c, hipEventRecord(c->stage_free, c->stream));
    return LGT_OK;
}

static lgt_status reduce_masks(lgt_ctx *c, bool flip, const uint64_t *masks, int n_masks,
                               std::vector<long double> &out)
{
    const int n = nq(c);
    const int chunk = flip ? kFlipChunk : kMaskChunk;
    const int g = flip ? reduce_blocks(n) : reduce_diag_blocks(n);
    out.assign(n_masks, 0.0L);
    for (int k0 = 0; k0 < n_masks; k0 += chunk) {
        const int m = std::min(chunk, n_masks - k0);
        HIPCHK(c, hipMemcpyAsync(c->masks_dev, masks + k0, sizeof(uint64_t) * m,
                                 hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, timed(c, flip ? KF_RED_FLIP : KF_RED_DIAG, [&] {
            return flip ? launch_reduce_flip(c->dtype, c->state, n, c->masks_dev, m, c->partials, c->stream)
                        : launch_reduce_diag(c->dtype, c->state, n, c->masks_dev, m, c->partials, c->stream);
        }));
        HIPCHK(c, hipMemcpyAsync(c->partials_host.data(), c->partials, sizeof(double) * g * chunk,
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int i = 0; i < m; ++i) {
            long double acc = 0;
            for (int b = 0; b < g; ++b) acc += c->partials_host[(size_t)b * chunk + i];
            out[k0 + i] = acc;
        }
    }
    return LGT_OK;
}

static lgt_status norm_of(lgt_ctx *c, long double &nrm)
{
    uint64_t zero = 0;
    std::vector<long double> v;
    lgt_status s = reduce_masks(c, false, &zero, 1, v);
    if (s) return s;
    nrm = v[0];
    return LGT_OK;
}

// Sec. 2.3 with the ancilla (bit N): for every plaquette, CNOTs from its links onto the
// ancilla, a measurement that keeps ancilla |0> (even parity, U_p = +1), CNOTs back; the
// product of the projections is normalised at the end.
static lgt_status ground_circuit(lgt_ctx *c)
{
    const Lattice &lat = c->lat;
    const int nt = nq(c), a = lat.n_links;
    for (int p = 0; p < lat.n_plaq; ++p) {
        const int32_t *l = &lat.plaq_links[4 * p];
        for (int k = 0; k < 4; ++k)
            HIPCHK(c, timed(c, KF_GATE_CNOT, [&] { return launch_gate_cnot(c->dtype, c->state, nt, l[k], a, c->stream); }));
        HIPCHK(c, timed(c, KF_PROJECT, [&] { return launch_project_scale(c->dtype, c->state, nt, 1ull << a, 1.0, c->stream); }));
        for (int k = 3; k >= 0; --k)
            HIPCHK(c, timed(c, KF_GATE_CNOT, [&] { return launch_gate_cnot(c->dtype, c->state, nt, l[k], a, c->stream); }));
    }
    long double nrm = 0;
    lgt_status s = norm_of(c, nrm);
    if (s) return s;
    if (!(nrm > 0)) return fail(c, LGT_E_STATE, "projection left a zero state");
    const double scale = (double)(1.0L / std::sqrt(nrm));
    HIPCHK(c, timed(c, KF_PROJECT, [&] { return launch_project_scale(c->dtype, c->state, nt, 0, scale, c->stream); }));
    return LGT_OK;
}

// The sigma^x basis of Sec. 3.3 for the X density of states: the Hadamard layer H on every
// link, written H = S R_x(pi/2) S with S = diag(1, i).  Only |<c|H^N psi>|^2 is needed, so
// the last S (a phase) is dropped and the transform is one fused step of the tile passes on
// a copy of the state: the phase i^popcount(b) (the plaquette-phase slot, fed syndrome
// tables that return b itself, so the phase index is the number of |1> links), the link
// layer exp(-i pi/4 sigma^x) on every link (tan form t = -1, scale 2^(-N/2) in the closing
// phase row).  The copy and its tables belong to the context from the first call on.
static lgt_status xdos_transform(lgt_ctx *c)
{
    const int n = c->lat.n_links, np1 = n + 1;
    const size_t eb = elem_bytes(c->dtype);
    // table block: identity syndrome tables | rotation | 2 phase rows | instance
    const size_t o_rot = sizeof(uint32_t) * kParityBytes * 256, o_ph = o_rot + 256,
                 o_inst = align256(o_ph + 2 * np1 * eb), tab_bytes = o_inst + sizeof(DevInst);
    if (!c->xdos_buf) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && c->state_bytes + (64u << 20) > free_b)
            return fail(c, LGT_E_OOM, "X-DOS buffer does not fit in free device memory");
        if (hipMalloc(&c->xdos_buf, c->state_bytes) != hipSuccess) {
            c->xdos_buf = nullptr;
            return fail(c, LGT_E_OOM, "X-DOS buffer");
        }
    }
    if (!c->xdos_tab) {
        std::vector<char> h(tab_bytes, 0);
        uint32_t *id = (uint32_t *)h.data();
        for (int k = 0; k < 4; ++k)
            for (int v = 0; v < 256; ++v) id[k * 256 + v] = (uint32_t)v << (8 * k);
        const double scale = std::pow(2.0, -0.5 * n);
        static const int re4[4] = {1, 0, -1, 0}, im4[4] = {0, 1, 0, -1};
        auto put = [&](size_t off, int i, double re, double im) {
            if (c->dtype == LGT_C64) {
                ((float *)(h.data() + off))[2 * i] = (float)re;
                ((float *)(h.data() + off))[2 * i + 1] = (float)im;
            } else {
                ((double *)(h.data() + off))[2 * i] = re;
                ((double *)(h.data() + off))[2 * i + 1] = im;
            }
        };
        put(o_rot, 0, 1.0, -1.0);                    // (u, v) = (1, tan(-pi/4))
        for (int m = 0; m <= n; ++m) {
            put(o_ph, m, re4[m & 3], im4[m & 3]);     // i^m
            put(o_ph, np1 + m, scale, 0.0);           // cos(-pi/4)^N
        }
        if (hipMalloc(&c->xdos_tab, tab_bytes) != hipSuccess) {
            c->xdos_tab = nullptr;
            return fail(c, LGT_E_OOM, "X-DOS tables");
        }
        DevInst di{};
        di.psi = c->xdos_buf;
        di.rot = (char *)c->xdos_tab + o_rot;
        di.phase = (char *)c->xdos_tab + o_ph;
        di.ptab = (const uint32_t *)c->xdos_tab;
        di.n_total = 1;
        std::memcpy(h.data() + o_inst, &di, sizeof di);
        // written once, before any kernel reads it
        HIPCHK(c, hipMemcpy(c->xdos_tab, h.data(), tab_bytes, hipMemcpyHostToDevice));
    }
    HIPCHK(c, hipMemcpyAsync(c->xdos_buf, c->state, c->state_bytes, hipMemcpyDeviceToDevice, c->stream));
    const uint8_t form = kFormTan;
    HIPCHK(c, enqueue_fused_steps(c->dtype, n, n, (const DevInst *)((char *)c->xdos_tab + o_inst), 1, 1,
                                  0, 1, &form, c->plan, c->stream, nullptr));
    return LGT_OK;
}

lgt_status lgt_measure(lgt_ctx *c, const lgt_observable *obs, double *out, size_t out_len)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    if (!obs || !out) return fail(c, LGT_E_INVALID, "null argument");
    const Lattice &lat = c->lat;
    std::vector<uint64_t> masks;
    bool flip = false;
    size_t need = 0;
    switch (obs->kind) {
    case LGT_OBS_NORM: need = 1; break;
    case LGT_OBS_Z:
    case LGT_OBS_X:
        if (obs->n_masks < 1 || !obs->masks) return fail(c, LGT_E_INVALID, "need masks");
        for (int i = 0; i < obs->n_masks; ++i)
            if (obs->masks[i] >> nq(c)) return fail(c, LGT_E_INVALID, "mask has bits beyond the qubits");
        masks.assign(obs->masks, obs->masks + obs->n_masks);
        flip = obs->kind == LGT_OBS_X;
        need = masks.size();
        break;
    case LGT_OBS_PLAQ: masks = lat.plaq_mask; need = masks.size(); break;
    case LGT_OBS_STAR: masks = lat.star_mask; flip = true; need = masks.size(); break;
    case LGT_OBS_SIGMAX:
    case LGT_OBS_SIGMAZ:
        for (int q = 0; q < lat.n_links; ++q) masks.push_back(1ull << q);
        flip = obs->kind == LGT_OBS_SIGMAX;
        need = masks.size();
        break;
    case LGT_OBS_ENERGY: need = 1; break;
    case LGT_OBS_ZDOS: need = lat.n_plaq + 1; break;
    case LGT_OBS_XDOS: need = lat.n_links + 1; break;
    default: return fail(c, LGT_E_INVALID, "unknown observable");
    }
    if (out_len < need) return fail(c, LGT_E_INVALID, "output array too short");
    long double nrm = 0;
    if ((s = norm_of(c, nrm))) return s;
    if (obs->kind == LGT_OBS_NORM) {
        out[0] = (double)nrm;
        return LGT_OK;
    }
    if (!(nrm > 0)) return fail(c, LGT_E_STATE, "state has zero norm");
    if (obs->kind == LGT_OBS_ZDOS) {
        const int g = reduce_blocks(nq(c));
        HIPCHK(c, timed(c, KF_RED_DOS, [&] {
            return launch_reduce_dos(c->dtype, c->state, nq(c), c->ptab_dev, lat.n_plaq, c->partials, c->stream);
        }));
        HIPCHK(c, hipMemcpyAsync(c->partials_host.data(), c->partials, sizeof(double) * g * kPartialWidth,
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int m = 0; m <= lat.n_plaq; ++m) {
            long double acc = 0;
            for (int b = 0; b < g; ++b) acc += c->partials_host[(size_t)b * kPartialWidth + m];
            out[m] = (double)(acc / nrm);
        }
        return LGT_OK;
    }
    if (obs->kind == LGT_OBS_XDOS) {
        if (lat.n_links > kMaxPlaq) return fail(c, LGT_E_UNSUPPORTED, "X-DOS supports <= 32 links");
        if (c->n_anc) return fail(c, LGT_E_UNSUPPORTED, "X-DOS of an ancilla context");
        if ((s = xdos_transform(c))) return s;
        const int g = reduce_blocks(lat.n_links);
        HIPCHK(c, timed(c, KF_RED_DOS, [&] {
            return launch_reduce_popcount(c->dtype, c->xdos_buf, lat.n_links, c->ptab_dev, c->partials, c->stream);
        }));
        HIPCHK(c, hipMemcpyAsync(c->partials_host.data(), c->partials, sizeof(double) * g * kPartialWidth,
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int k = 0; k <= lat.n_links; ++k) {
            long double acc = 0;
            for (int b = 0; b < g; ++b) acc += c->partials_host[(size_t)b * kPartialWidth + k];
            out[k] = (double)(acc / nrm);
        }
        return LGT_OK;
    }
    if (obs->kind == LGT_OBS_ENERGY) {
        std::vector<uint64_t> sx;
        for (int q = 0; q < lat.n_links; ++q) sx.push_back(1ull << q);
        std::vector<long double> vx, vz;
        if ((s = reduce_masks(c, true, sx.data(), (int)sx.size(), vx))) return s;
        if ((s = reduce_masks(c, false, lat.plaq_mask.data(), lat.n_plaq, vz))) return s;
        long double ex = 0, ez = 0;
        for (auto v : vx) ex += v;
        for (auto v : vz) ez += v;
        out[0] = (double)((-(long double)obs->cx * ex - (long double)obs->cz * ez) / nrm);
        return LGT_OK;
    }
    std::vector<long double> v;
    if ((s = reduce_masks(c, flip, masks.data(), (int)masks.size(), v))) return s;
    for (size_t i = 0; i < masks.size(); ++i) out[i] = (double)(v[i] / nrm);
    return LGT_OK;
}

lgt_status lgt_scan(lgt_ctx *c, const lgt_schedule *sched, lgt_order order, int64_t first_step,
                    int64_t substeps, int64_t n_points, const uint64_t *masks, int n_masks,
                    double *out, size_t out_len)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    if (!sched || !out) return fail(c, LGT_E_INVALID, "null argument");
    if (order != LGT_ORDER_TROTTER && order != LGT_ORDER_SYMMETRIC)
        return fail(c, LGT_E_INVALID, "bad order");
    if (substeps < 1 || n_points < 1 || n_masks < 0 || n_masks > 32 || (n_masks > 0 && !masks))
        return fail(c, LGT_E_INVALID, "bad scan sizes");
    if (c->n_anc) return fail(c, LGT_E_UNSUPPORTED, "scans run the fused form: not on an ancilla context");
    const Lattice &lat = c->lat;
    const int n = lat.n_links;
    for (int i = 0; i < n_masks; ++i)
        if (masks[i] >> n) return fail(c, LGT_E_INVALID, "mask has bits beyond N");
    const int width = 5 + n_masks;
    if (out_len < (size_t)n_points * width) return fail(c, LGT_E_INVALID, "output array too short");
    // the whole range must lie inside the schedule
    {
        double dt0;
        std::vector<double> a, b;
        std::string why = schedule_coeffs(sched, first_step + substeps * (n_points - 1), substeps, dt0, a, b);
        if (!why.empty()) return fail(c, LGT_E_INVALID, why);
    }
    // diagonal masks: the norm, the plaquettes, the loops; off-diagonal: single links
    std::vector<uint64_t> mk(1, 0);
    mk.insert(mk.end(), lat.plaq_mask.begin(), lat.plaq_mask.end());
    mk.insert(mk.end(), masks, masks + n_masks);
    const int nd = (int)mk.size();
    for (int q = 0; q < n; ++q) mk.push_back(1ull << q);
    const int ncol = (int)mk.size();
    void *mdev = nullptr;
    double *sums = nullptr;
    auto cleanup = [&] {
        if (mdev) (void)hipFree(mdev);
        if (sums) (void)hipFree(sums);
    };
    auto bail = [&](lgt_status st, const std::string &m) {
        (void)hipStreamSynchronize(c->stream);
        cleanup();
        return fail(c, st, m);
    };
    if (hipMalloc(&mdev, sizeof(uint64_t) * ncol) != hipSuccess ||
        hipMalloc((void **)&sums, sizeof(double) * ncol * (size_t)n_points) != hipSuccess)
        return bail(LGT_E_OOM, "scan buffers");
    if (hipMemcpy(mdev, mk.data(), sizeof(uint64_t) * ncol, hipMemcpyHostToDevice) != hipSuccess)
        return bail(LGT_E_DEVICE, "scan mask upload");
    const uint64_t *md = (const uint64_t *)mdev;
    const int g = reduce_blocks(n), gd = reduce_diag_blocks(n);
    std::vector<double> cxs(n_points), czs(n_points);
    for (int64_t k = 0; k < n_points; ++k) {
        double dt = 0;
        std::vector<double> cx, cz;
        std::string why = schedule_coeffs(sched, first_step + k * substeps, substeps, dt, cx, cz);
        if (!why.empty()) return bail(LGT_E_INVALID, why);
        cxs[k] = cx.back();
        czs[k] = cz.back();
        if ((s = evolve_fused(c, dt, cx, cz, order))) {
            std::string m = c->err;
            return bail(s, m);
        }
        double *row = sums + (size_t)k * ncol;
        hipError_t e = hipSuccess;
        for (int off = 0; off < nd && e == hipSuccess; off += kMaskChunk) {
            const int m = std::min(kMaskChunk, nd - off);
            e = timed(c, KF_RED_DIAG, [&] {
                return launch_reduce_diag(c->dtype, c->state, n, md + off, m, c->partials, c->stream);
            });
            if (e == hipSuccess) e = launch_sum_cols(c->partials, gd, kMaskChunk, m, row + off, c->stream);
        }
        for (int off = nd; off < ncol && e == hipSuccess; off += kFlipChunk) {
            const int m = std::min(kFlipChunk, ncol - off);
            e = timed(c, KF_RED_FLIP, [&] {
                return launch_reduce_flip(c->dtype, c->state, n, md + off, m, c->partials, c->stream);
            });
            if (e == hipSuccess) e = launch_sum_cols(c->partials, g, kFlipChunk, m, row + off, c->stream);
        }
        if (e != hipSuccess) return bail(LGT_E_DEVICE, std::string("scan readout: ") + hipGetErrorString(e));
    }
    std::vector<double> host((size_t)ncol * n_points);
    if (hipMemcpyAsync(host.data(), sums, sizeof(double) * host.size(), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return bail(LGT_E_DEVICE, "scan download");
    cleanup();
    for (int64_t k = 0; k < n_points; ++k) {
        const double *h = &host[(size_t)k * ncol];
        double *o = out + (size_t)k * width;
        const long double nrm = h[0];
        long double zs = 0, xs = 0;
        for (int p = 0; p < lat.n_plaq; ++p) zs += h[1 + p];
        for (int q = 0; q < n; ++q) xs += h[nd + q];
        o[0] = cxs[k];
        o[1] = czs[k];
        o[2] = nrm > 0 ? (double)(-zs / nrm) : 0.0;
        o[3] = nrm > 0 ? (double)(-xs / nrm) : 0.0;
        o[4] = (double)nrm;
        for (int i = 0; i < n_masks; ++i) o[5 + i] = nrm > 0 ? (double)(h[1 + lat.n_plaq + i] / nrm) : 0.0;
    }
    return LGT_OK;
}

lgt_status lgt_critical_point(const double *g, const double *h, int n, int stride,
                              double *g_c, double *d2_min)
{
    if (!g || !h || !g_c || !d2_min || stride < 1 || n < 2 * stride + 3)
        return fail(nullptr, LGT_E_INVALID, "critical point: bad arguments");
    for (int i = 1; i < n; ++i)
        if (!(g[i] > g[i - 1])) return fail(nullptr, LGT_E_INVALID, "couplings must increase");
    std::vector<double> d2(n, 0.0);
    int best = -1;
    for (int i = stride; i + stride < n; ++i) {
        const double gl = g[i - stride], gm = g[i], gr = g[i + stride];
        d2[i] = 2.0 * ((h[i + stride] - h[i]) / (gr - gm) - (h[i] - h[i - stride]) / (gm - gl)) / (gr - gl);
        if (best < 0 || d2[i] < d2[best]) best = i;
    }
    double x = g[best], y = d2[best];
    if (best - 1 >= stride && best + 1 + stride < n) {
        // vertex of the parabola through the lowest point and its neighbours
        const double x0 = g[best - 1], x1 = g[best], x2 = g[best + 1];
        const double y0 = d2[best - 1], y1 = d2[best], y2 = d2[best + 1];
        const double den = (x0 - x1) * (x0 - x2) * (x1 - x2);
        const double A = (x2 * (y1 - y0) + x1 * (y0 - y2) + x0 * (y2 - y1)) / den;
        const double B = (x2 * x2 * (y0 - y1) + x1 * x1 * (y2 - y0) + x0 * x0 * (y1 - y2)) / den;
        const double C = (x1 * x2 * (x1 - x2) * y0 + x2 * x0 * (x2 - x0) * y1 + x0 * x1 * (x0 - x1) * y2) / den;
        if (A > 0) {
            const double xv = -B / (2 * A);
            if (xv >= x0 && xv <= x2) {
                x = xv;
                y = C - B * B / (4 * A);
            }
        }
    }
    *g_c = x;
    *d2_min = y;
    return LGT_OK;
}

lgt_status lgt_crossing(const double *g, const double *a, const double *b, int n, double *g_x)
{
    if (!g || !a || !b || !g_x || n < 2) return fail(nullptr, LGT_E_INVALID, "crossing: bad arguments");
    for (int i = 1; i < n; ++i) {
        const double d0 = a[i - 1] - b[i - 1], d1 = a[i] - b[i];
        if (d0 == 0) {
            *g_x = g[i - 1];
            return LGT_OK;
        }
        if ((d0 < 0) != (d1 < 0) || d1 == 0) {
            *g_x = g[i - 1] + (g[i] - g[i - 1]) * d0 / (d0 - d1);
            return LGT_OK;
        }
    }
    return fail(nullptr, LGT_E_INVALID, "no crossing");
}

lgt_status lgt_sample(lgt_ctx *c, uint64_t n_shots, uint64_t seed, uint64_t *out)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    if (!out) return fail(c, LGT_E_INVALID, "null output");
    if (n_shots < 1 || n_shots > (1ull << 26)) return fail(c, LGT_E_INVALID, "n_shots out of range");
    const int n = nq(c);
    const size_t nb = (size_t)1 << (n - sample_block_bits(n));
    double *sums = nullptr, *prefix = nullptr;
    uint64_t *dev_out = nullptr;
    auto cleanup = [&] {
        if (sums) (void)hipFree(sums);
        if (prefix) (void)hipFree(prefix);
        if (dev_out) (void)hipFree(dev_out);
    };
    if (hipMalloc((void **)&sums, nb * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&prefix, nb * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&dev_out, n_shots * sizeof(uint64_t)) != hipSuccess) {
        cleanup();
        return fail(c, LGT_E_OOM, "sampling buffers");
    }
    hipError_t e = timed(c, KF_SAMPLE, [&] {
        return launch_sample(c->dtype, c->state, n, n_shots, seed, sums, prefix, dev_out, c->stream);
    });
    if (e == hipSuccess) e = hipMemcpyAsync(out, dev_out, n_shots * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    cleanup();
    if (e != hipSuccess) return fail(c, LGT_E_DEVICE, std::string("sample: ") + hipGetErrorString(e));
    return LGT_OK;
}

lgt_status lgt_sample_noalloc(lgt_ctx *c, uint64_t n_shots, uint64_t seed, uint64_t *out)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    if (!out) return fail(c, LGT_E_INVALID, "null output");
    if (n_shots < 1 || n_shots > (uint64_t)kScratchShots)
        return fail(c, LGT_E_INVALID, "n_shots must be in [1, 2^20] for the allocation-free sampler");
    const int n = nq(c);
    if (((uint64_t)1 << (n - sample_block_bits(n))) > (uint64_t)kScratchSums)
        return fail(c, LGT_E_INVALID, "the allocation-free sampler takes states of at most 30 qubits");
    void *scr = nullptr;
    HIPCHK(c, scratch_address(c->device, &scr));
    // launched untimed: the profiling events come from a pool the library may need to grow
    HIPCHK(c, launch_sample_scratch(c->dtype, c->state, n, n_shots, seed, scr, c->stream));
    HIPCHK(c, hipMemcpyAsync(out, (uint64_t *)scr + kScratchSums, n_shots * sizeof(uint64_t),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LGT_OK;
}

lgt_status lgt_get_state(lgt_ctx *c, void *host, size_t bytes)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    if (!host || bytes != c->state_bytes) return fail(c, LGT_E_INVALID, "host buffer must be state_bytes");
    HIPCHK(c, hipMemcpyAsync(host, c->state, bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LGT_OK;
}

lgt_status lgt_set_state(lgt_ctx *c, const void *host, size_t bytes)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    if (!host || bytes != c->state_bytes) return fail(c, LGT_E_INVALID, "host buffer must be state_bytes");
    HIPCHK(c, hipMemcpyAsync(c->state, host, bytes, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LGT_OK;
}

lgt_status lgt_copy_state(lgt_ctx *dst, lgt_ctx *src)
{
    lgt_status s = check_ctx(dst);
    if (s) return s;
    if (!src || src->dtype != dst->dtype || src->lat.d != dst->lat.d || src->n_anc != dst->n_anc ||
        std::memcmp(src->lat.L, dst->lat.L, sizeof src->lat.L) != 0 || src->device != dst->device)
        return fail(dst, LGT_E_INVALID, "copy needs contexts of one lattice, dtype and device");
    if (src == dst) return LGT_OK;
    HIPCHK(dst, hipStreamSynchronize(src->stream));
    HIPCHK(dst, hipMemcpyAsync(dst->state, src->state, dst->state_bytes, hipMemcpyDeviceToDevice,
                               dst->stream));
    return LGT_OK;
}

lgt_status lgt_sync(lgt_ctx *c)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LGT_OK;
}

lgt_status lgt_set_graphs(lgt_ctx *c, int on)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    if (!on) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second);
        c->graphs.clear();
    }
    c->use_graphs = on != 0;
    return LGT_OK;
}

lgt_status lgt_set_profiling(lgt_ctx *c, int on)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    HIPCHK(c, prof_harvest(c));
    c->profiling = on > 0;
    c->prof_stride = on > 1 ? on : 1;
    for (int k = 0; k < KF_COUNT; ++k) {
        c->prof_launches[k] = 0;
        c->prof_ms[k] = 0;
        c->prof_seen[k] = 0;
    }
    return LGT_OK;
}

lgt_status lgt_kernel_stats(lgt_ctx *c, const char **names, int64_t *launches, double *total_ms,
                            int cap, int *n)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    if (!n) return fail(c, LGT_E_INVALID, "null count");
    HIPCHK(c, prof_harvest(c));
    int k = 0;
    for (int f = 0; f < KF_COUNT && k < cap; ++f) {
        if (!c->prof_launches[f]) continue;
        if (names) names[k] = kernel_family_name(f);
        if (launches) launches[k] = c->prof_launches[f];
        if (total_ms) total_ms[k] = c->prof_ms[f];
        ++k;
    }
    *n = k;
    return LGT_OK;
}

const char *lgt_last_error(const lgt_ctx *c)
{
    return c ? c->err.c_str() : g_err.c_str();
}

lgt_status lgt_plan_describe(const lgt_ctx *c, char *out, size_t len)
{
    if (!c || !out || len == 0) return fail(nullptr, LGT_E_INVALID, "null argument");
    const std::string d = describe_plan(plan_passes(c->lat.n_links, c->dtype, c->plan, 1), c->lat.n_links);
    std::snprintf(out, len, "%s", d.c_str());
    return d.size() < len ? LGT_OK : fail(const_cast<lgt_ctx *>(c), LGT_E_INVALID, "buffer too short");
}

lgt_status lgt_plan_query(int n_links, lgt_dtype dtype, int plan, char *out, size_t len)
{
    if (!out || len == 0) return fail(nullptr, LGT_E_INVALID, "null argument");
    if (n_links < 1 || n_links > kMaxLinks) return fail(nullptr, LGT_E_INVALID, "n_links out of range");
    if (dtype != LGT_C64 && dtype != LGT_C128) return fail(nullptr, LGT_E_INVALID, "unknown dtype");
    if (plan < 0 || (plan & ~kPlanNoMerge) > 5) return fail(nullptr, LGT_E_INVALID, "unknown plan code");
    const std::string d = describe_plan(plan_passes(n_links, dtype, plan, 1), n_links);
    std::snprintf(out, len, "%s", d.c_str());
    return d.size() < len ? LGT_OK : fail(nullptr, LGT_E_INVALID, "buffer too short");
}

lgt_status lgt_set_plan(lgt_ctx *c, int plan)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    if (plan < 0 || (plan & ~kPlanNoMerge) > 5) return fail(c, LGT_E_INVALID, "unknown plan code");
    c->plan = plan;
    return LGT_OK;
}

lgt_status lgt_get_plan(const lgt_ctx *c, int *plan)
{
    if (!c || !plan) return fail(nullptr, LGT_E_INVALID, "null argument");
    *plan = c->plan;
    return LGT_OK;
}

lgt_status lgt_tune(lgt_ctx *c, int steps)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    if (steps < 1 || steps > 1024) return fail(c, LGT_E_INVALID, "steps must be in [1, 1024]");
    if (c->n_anc) return fail(c, LGT_E_UNSUPPORTED, "the ancilla forms have no pass plan to tune");
    const Lattice &lat = c->lat;
    const int n = lat.n_links;
    if (small_supported(c->dtype, n)) return LGT_OK;   // one on-chip kernel: nothing to choose
    // identity tables: u = 1, v = 0 and unit phases leave every amplitude bit for bit unchanged
    const int np1 = lat.n_plaq + 1, total = steps + 2;
    const size_t eb = elem_bytes(c->dtype);
    std::vector<char> rot((size_t)total * eb, 0), ph((size_t)total * np1 * eb, 0);
    for (int j = 0; j < total; ++j) {
        if (c->dtype == LGT_C64) ((float *)rot.data())[2 * j] = 1.0f;
        else ((double *)rot.data())[2 * j] = 1.0;
    }
    for (int k = 0; k < total * np1; ++k) {
        if (c->dtype == LGT_C64) ((float *)ph.data())[2 * k] = 1.0f;
        else ((double *)ph.data())[2 * k] = 1.0;
    }
    void *drot = nullptr, *dph = nullptr;
    DevInst *dinst = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&] {
        if (drot) (void)hipFree(drot);
        if (dph) (void)hipFree(dph);
        if (dinst) (void)hipFree(dinst);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    DevInst di{};
    hipError_t e = hipMalloc(&drot, rot.size());
    if (e == hipSuccess) e = hipMalloc(&dph, ph.size());
    if (e == hipSuccess) e = hipMalloc((void **)&dinst, sizeof(DevInst));
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMemcpyAsync(drot, rot.data(), rot.size(), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dph, ph.data(), ph.size(), hipMemcpyHostToDevice, c->stream);
    di.psi = c->state;
    di.rot = drot;
    di.phase = dph;
    di.ptab = c->ptab_dev;
    di.n_total = total;
    if (e == hipSuccess) e = hipMemcpyAsync(dinst, &di, sizeof di, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    std::vector<uint8_t> forms(total, 1);
    int best = c->plan;
    float best_ms = 1e30f;
    std::vector<std::string> seen;
    for (int cand : {1, 2, 3, 4, 5}) {
        if (e != hipSuccess) break;
        const std::string d = describe_plan(plan_passes(n, c->dtype, cand, 1), n);
        if (std::find(seen.begin(), seen.end(), d) != seen.end()) continue;
        seen.push_back(d);
        e = enqueue_fused_steps(c->dtype, n, lat.n_plaq, dinst, 1, 2, -1, 0, forms.data(), cand, c->stream, nullptr);
        if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
        if (e == hipSuccess)
            e = enqueue_fused_steps(c->dtype, n, lat.n_plaq, dinst, 1, steps, -1, 0, forms.data(), cand, c->stream, nullptr);
        if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms < best_ms) {
            best_ms = ms;
            best = cand;
        }
    }
    cleanup();
    if (e != hipSuccess) return fail(c, LGT_E_DEVICE, std::string("tune: ") + hipGetErrorString(e));
    c->plan = best;
    return LGT_OK;
}

static lgt_status batch_group_evolve(int n_inst, lgt_ctx *const *ctxs, const lgt_schedule *scheds,
                                     const lgt_order *orders, int64_t first_step, int64_t count);

lgt_status lgt_batch_evolve(int n_inst, lgt_ctx *const *ctxs, const lgt_schedule *scheds,
                            const lgt_order *orders, int64_t first_step, int64_t count)
{
    if (n_inst < 1 || !ctxs || !scheds || !orders) return fail(nullptr, LGT_E_INVALID, "bad batch arguments");
    lgt_ctx *c0 = ctxs[0];
    if (!c0) return fail(nullptr, LGT_E_INVALID, "null context in batch");
    if (n_inst > 65535) return fail(nullptr, LGT_E_INVALID, "too many instances");
    for (int i = 0; i < n_inst; ++i) {
        lgt_ctx *c = ctxs[i];
        if (!c || c->dtype != c0->dtype || c->lat.d != c0->lat.d ||
            std::memcmp(c->lat.L, c0->lat.L, sizeof c->lat.L) != 0 || c->device != c0->device)
            return fail(nullptr, LGT_E_INVALID, "batch contexts must share lattice, dtype and device");
        if (c->n_anc) return fail(nullptr, LGT_E_UNSUPPORTED, "batches run the fused form: no ancilla contexts");
        if (orders[i] != LGT_ORDER_TROTTER && orders[i] != LGT_ORDER_SYMMETRIC)
            return fail(nullptr, LGT_E_INVALID, "bad order");
        if (orders[i] != orders[0])
            return fail(nullptr, LGT_E_UNSUPPORTED, "batched instances must share the order");
    }
    lgt_status s = check_ctx(c0);
    if (s) return fail(nullptr, s, c0->err);
    if (count == 0) return LGT_OK;
    // Instances per launch: the tuned group size of the first context (lgt_batch_tune), else
    // states that each fit the 256 MB Infinity Cache but together do not run in groups that
    // do, one group after the other (four 24-link complex64 states, 128 MiB each, in one
    // launch took 61 us per instance-step, one at a time 57 us).  Each instance's arithmetic
    // is the same either way.
    const size_t per_group = c0->batch_group > 0 ? (size_t)c0->batch_group
                                                 : kCacheStateBytes / c0->state_bytes;
    if (per_group >= 1 && (size_t)n_inst > per_group) {
        for (int i0 = 0; i0 < n_inst; i0 += (int)per_group) {
            const int m = (int)std::min<size_t>(per_group, (size_t)(n_inst - i0));
            if ((s = batch_group_evolve(m, ctxs + i0, scheds + i0, orders + i0, first_step, count)))
                return s;
            // the next group starts once this one has left the cache
            if (hipStreamSynchronize(ctxs[i0]->stream) != hipSuccess)
                return fail(nullptr, LGT_E_DEVICE, "batch group sync");
        }
        return LGT_OK;
    }
    return batch_group_evolve(n_inst, ctxs, scheds, orders, first_step, count);
}

}  // extern "C"

// one launch group of a batch: every pass one launch over the n_inst instances
static lgt_status batch_group_evolve(int n_inst, lgt_ctx *const *ctxs, const lgt_schedule *scheds,
                                     const lgt_order *orders, int64_t first_step, int64_t count)
{
    lgt_ctx *c0 = ctxs[0];
    lgt_status s = LGT_OK;
    // every instance's tables in one staging block, built on several host threads (the
    // FP32 rounding of a 2000-step table takes milliseconds per instance).  Complex64 runs of
    // tile passes round and upload their phase rows in chunks of 32, 64, 128, ... steps,
    // each chunk's launches enqueued as soon as its rows are staged, as a single run does;
    // a batch replayed from a graph, or run by the one-kernel small-state path, rounds its
    // tables whole first.
    const Lattice &lat = c0->lat;
    const bool graph = c0->use_graphs && !c0->profiling && c0->stream;
    const bool piped = c0->dtype == LGT_C64 && !graph && !small_supported(c0->dtype, lat.n_links);
    std::vector<Tables> tbs(n_inst);
    std::vector<StepTables> sts(n_inst);
    std::vector<std::string> whys(n_inst);
    std::vector<std::vector<long double>> gains(n_inst);
    parallel_for(n_inst, [&](int i) {
        double dt;
        std::vector<double> cx, cz;
        whys[i] = schedule_coeffs(&scheds[i], first_step, count, dt, cx, cz);
        if (!whys[i].empty()) return;
        if (!piped) {
            make_tables(lat, c0->dtype, dt, cx, cz, orders[i], sts[i], tbs[i]);
            return;
        }
        build_step_tables(lat.n_links, lat.n_plaq, dt, cx.data(), cz.data(), (int)count, orders[i], sts[i]);
        round_rot_f32(sts[i], lat.n_links, tbs[i].rf, gains[i]);
        tbs[i].pf.assign((size_t)sts[i].n_phase * (lat.n_plaq + 1), Cplx<float>{});
        tbs[i].rot_bytes = tbs[i].rf.size() * sizeof(RotParam<float>);
        tbs[i].ph_bytes = tbs[i].pf.size() * sizeof(Cplx<float>);
    });
    std::vector<uint8_t> forms;
    for (int i = 0; i < n_inst; ++i) {
        if (!whys[i].empty()) return fail(nullptr, LGT_E_INVALID, whys[i]);
        or_forms(sts[i], forms);
    }
    const StepTables &st = sts[0];
    const size_t rb = align256(tbs[0].rot_bytes), pb = align256(tbs[0].ph_bytes);
    const size_t ib = align256(sizeof(DevInst) * n_inst);
    const size_t total = (rb + pb) * n_inst + ib;
    for (int i = 1; i < n_inst; ++i)
        if (ctxs[i]->stream != c0->stream && hipStreamSynchronize(ctxs[i]->stream) != hipSuccess)
            return fail(nullptr, LGT_E_DEVICE, "sync of a batch member failed");
    if (ensure_stage(c0, total) != hipSuccess) return fail(nullptr, LGT_E_OOM, "staging buffer");
    if (ensure_dev(c0, &c0->rot_dev, &c0->rot_cap, total) != hipSuccess)
        return fail(nullptr, LGT_E_OOM, "batch tables");
    char *stg = (char *)c0->stage;
    char *dev = (char *)c0->rot_dev;
    std::vector<DevInst> di(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        std::memcpy(stg + i * (rb + pb), rot_ptr(tbs[i], c0->dtype), tbs[i].rot_bytes);
        if (!piped) std::memcpy(stg + i * (rb + pb) + rb, ph_ptr(tbs[i], c0->dtype), tbs[i].ph_bytes);
        di[i].psi = ctxs[i]->state;
        di[i].rot = dev + i * (rb + pb);
        di[i].phase = dev + i * (rb + pb) + rb;
        di[i].ptab = c0->ptab_dev;
        di[i].step0 = 0;
        di[i].ph0 = 0;
        di[i].n_total = (int)count;
    }
    std::memcpy(stg + (rb + pb) * n_inst, di.data(), sizeof(DevInst) * n_inst);
    const DevInst *dinst = (const DevInst *)(dev + (rb + pb) * n_inst);
    hipError_t e = hipSuccess;
    if (piped) {
        // link rows and the instance array first, then the phase rows chunk by chunk
        for (int i = 0; i < n_inst && e == hipSuccess; ++i)
            e = hipMemcpyAsync(dev + i * (rb + pb), stg + i * (rb + pb), tbs[i].rot_bytes,
                               hipMemcpyHostToDevice, c0->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync((void *)dinst, stg + (rb + pb) * n_inst, sizeof(DevInst) * n_inst,
                               hipMemcpyHostToDevice, c0->stream);
        const int pre = st.pre_phase, steps = (int)count;
        const size_t ph_row = sizeof(Cplx<float>) * (lat.n_plaq + 1);
        std::vector<PhaseRounding> prs(n_inst);
        FusedCursor cur;
        for (int j0 = 0, len = kFirstChunk; j0 < steps && e == hipSuccess; j0 += len, len *= 2) {
            const int j1 = (int)std::min<int64_t>(steps, (int64_t)j0 + len);
            // phase rows read by the launches of steps [j0, j1) (as in a single run)
            const int k0 = j0 == 0 ? 0 : j0 + pre, k1 = j1 + pre;
            parallel_for(n_inst, [&](int i) {
                round_phase_f32(sts[i], lat.n_plaq, gains[i], k0, k1, tbs[i].pf, prs[i]);
                std::memcpy(stg + i * (rb + pb) + rb + ph_row * k0,
                            (const char *)tbs[i].pf.data() + ph_row * k0, ph_row * (k1 - k0));
            });
            for (int i = 0; i < n_inst && e == hipSuccess; ++i)
                e = hipMemcpyAsync(dev + i * (rb + pb) + rb + ph_row * k0,
                                   stg + i * (rb + pb) + rb + ph_row * k0, ph_row * (k1 - k0),
                                   hipMemcpyHostToDevice, c0->stream);
            if (e == hipSuccess)
                e = enqueue_fused_range(c0->dtype, lat.n_links, lat.n_plaq, dinst, n_inst, steps, j0,
                                        j1, pre ? 0 : -1, pre, forms.data(), c0->plan, c0->stream,
                                        c0, cur);
        }
        if (e == hipSuccess) e = hipEventRecord(c0->stage_free, c0->stream);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(c0->stream);
            return fail(nullptr, LGT_E_DEVICE, std::string("batch launch: ") + hipGetErrorString(e));
        }
    } else {
        if (hipMemcpyAsync(dev, stg, total, hipMemcpyHostToDevice, c0->stream) != hipSuccess ||
            hipEventRecord(c0->stage_free, c0->stream) != hipSuccess)
            return fail(nullptr, LGT_E_DEVICE, "batch upload");
        if (graph) {
            // the launches depend only on this key (the tables and state pointers are read
            // from the instance array on the device): the same key replays the same graph
            std::string key = std::to_string(n_inst) + ":" + std::to_string(count) + ":" +
                              std::to_string(c0->plan) + ":" + std::to_string(st.pre_phase) + ":" +
                              std::to_string((uintptr_t)dinst) + ":";
            key.append((const char *)forms.data(), forms.size());
            auto it = c0->graphs.find(key);
            if (it == c0->graphs.end() && c0->graphs.size() >= kMaxGraphs) {
                // a bounded cache: drop every graph once the last launch of one has ended
                if ((e = hipStreamSynchronize(c0->stream)) != hipSuccess)
                    return fail(nullptr, LGT_E_DEVICE, std::string("batch sync: ") + hipGetErrorString(e));
                for (auto &g : c0->graphs) (void)hipGraphExecDestroy(g.second);
                c0->graphs.clear();
            }
            if (it == c0->graphs.end()) {
                hipGraph_t hg = nullptr;
                hipGraphExec_t exec = nullptr;
                e = hipStreamBeginCapture(c0->stream, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    const hipError_t el = enqueue_fused(c0, dinst, n_inst, (int)count, st.pre_phase, forms.data());
                    e = hipStreamEndCapture(c0->stream, &hg);
                    if (el != hipSuccess) e = el;
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&exec, hg, nullptr, nullptr, 0);
                if (hg) (void)hipGraphDestroy(hg);
                if (e == hipSuccess) it = c0->graphs.emplace(key, exec).first;
            }
            if (e == hipSuccess) e = hipGraphLaunch(it->second, c0->stream);
        } else {
            e = enqueue_fused(c0, dinst, n_inst, (int)count, st.pre_phase, forms.data());
        }
        if (e != hipSuccess) return fail(nullptr, LGT_E_DEVICE, std::string("batch launch: ") + hipGetErrorString(e));
    }
    // the other contexts must not race ahead of the shared launches
    for (int i = 1; i < n_inst; ++i)
        if (ctxs[i]->stream != c0->stream && hipStreamSynchronize(c0->stream) != hipSuccess)
            return fail(nullptr, LGT_E_DEVICE, "batch sync");
    return LGT_OK;
}

extern "C" {

lgt_status lgt_batch_set_group(lgt_ctx *c, int group)
{
    lgt_status s = check_ctx(c);
    if (s) return s;
    if (group < 0 || group > 65535) return fail(c, LGT_E_INVALID, "group size must be in [0, 65535]");
    c->batch_group = group;
    return LGT_OK;
}

lgt_status lgt_batch_tune(int n, lgt_ctx *const *ctxs, int steps, int *group_out)
{
    if (n < 1 || n > 65535 || !ctxs || !ctxs[0] || !group_out)
        return fail(nullptr, LGT_E_INVALID, "bad batch tune arguments");
    if (steps < 1 || steps > 1024) return fail(nullptr, LGT_E_INVALID, "steps must be in [1, 1024]");
    lgt_ctx *c0 = ctxs[0];
    for (int i = 0; i < n; ++i) {
        lgt_ctx *c = ctxs[i];
        if (!c || c->dtype != c0->dtype || c->lat.d != c0->lat.d ||
            std::memcmp(c->lat.L, c0->lat.L, sizeof c->lat.L) != 0 || c->device != c0->device)
            return fail(nullptr, LGT_E_INVALID, "batch contexts must share lattice, dtype and device");
        if (c->n_anc) return fail(nullptr, LGT_E_UNSUPPORTED, "batches run the fused form: no ancilla contexts");
    }
    lgt_status s = check_ctx(c0);
    if (s) return fail(nullptr, s, c0->err);
    const Lattice &lat = c0->lat;
    const int N = lat.n_links;
    if (small_supported(c0->dtype, N)) {
        // one on-chip kernel runs every instance and step of a batch: one launch group
        c0->batch_group = n;
        *group_out = n;
        return LGT_OK;
    }
    for (int i = 0; i < n; ++i)
        if (hipStreamSynchronize(ctxs[i]->stream) != hipSuccess)
            return fail(nullptr, LGT_E_DEVICE, "sync of a batch member failed");
    // identity tables, as in lgt_tune: u = 1, v = 0 and unit phases leave every state bit for
    // bit unchanged
    const int np1 = lat.n_plaq + 1, total = steps + 2;
    const size_t eb = elem_bytes(c0->dtype);
    std::vector<char> rot((size_t)total * eb, 0), ph((size_t)total * np1 * eb, 0);
    for (int j = 0; j < total; ++j) {
        if (c0->dtype == LGT_C64) ((float *)rot.data())[2 * j] = 1.0f;
        else ((double *)rot.data())[2 * j] = 1.0;
    }
    for (int k = 0; k < total * np1; ++k) {
        if (c0->dtype == LGT_C64) ((float *)ph.data())[2 * k] = 1.0f;
        else ((double *)ph.data())[2 * k] = 1.0;
    }
    void *drot = nullptr, *dph = nullptr;
    DevInst *dinst = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&] {
        (void)hipStreamSynchronize(c0->stream);
        if (drot) (void)hipFree(drot);
        if (dph) (void)hipFree(dph);
        if (dinst) (void)hipFree(dinst);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    std::vector<DevInst> di(n);
    hipError_t e = hipMalloc(&drot, rot.size());
    if (e == hipSuccess) e = hipMalloc(&dph, ph.size());
    if (e == hipSuccess) e = hipMalloc((void **)&dinst, sizeof(DevInst) * n);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int i = 0; i < n; ++i) {
        di[i] = DevInst{};
        di[i].psi = ctxs[i]->state;
        di[i].rot = drot;
        di[i].phase = dph;
        di[i].ptab = c0->ptab_dev;
        di[i].n_total = total;
    }
    if (e == hipSuccess) e = hipMemcpy(drot, rot.data(), rot.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dph, ph.data(), ph.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dinst, di.data(), sizeof(DevInst) * n, hipMemcpyHostToDevice);
    // candidates: every instance in one launch, the Infinity-Cache-sized group, halves, ..., one
    std::vector<int> cands{n};
    const size_t cache_group = kCacheStateBytes / c0->state_bytes;
    if (cache_group >= 1 && cache_group < (size_t)n) cands.push_back((int)cache_group);
    for (int g = (n + 1) / 2; g >= 1; g = (g == 1) ? 0 : (g + 1) / 2)
        if (std::find(cands.begin(), cands.end(), g) == cands.end()) cands.push_back(g);
    std::vector<uint8_t> forms(total, kFormTan);
    int best = n;
    float best_ms = 1e30f;
    for (int g : cands) {
        if (e != hipSuccess) break;
        auto run = [&](int count) -> hipError_t {
            for (int i0 = 0; i0 < n; i0 += g) {
                const int m = std::min(g, n - i0);
                hipError_t r = enqueue_fused_steps(c0->dtype, N, lat.n_plaq, dinst + i0, m, count, -1,
                                                   0, forms.data(), c0->plan, c0->stream, nullptr);
                if (r != hipSuccess) return r;
            }
            return hipSuccess;
        };
        e = run(2);
        if (e == hipSuccess) e = hipEventRecord(e0, c0->stream);
        if (e == hipSuccess) e = run(steps);
        if (e == hipSuccess) e = hipEventRecord(e1, c0->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms < best_ms) {
            best_ms = ms;
            best = g;
        }
    }
    cleanup();
    if (e != hipSuccess) return fail(nullptr, LGT_E_DEVICE, std::string("batch tune: ") + hipGetErrorString(e));
    c0->batch_group = best;
    *group_out = best;
    return LGT_OK;
}

}  // extern "C"
