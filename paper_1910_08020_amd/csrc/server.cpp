// Continuous-batching server for adiabatic runs of mixed lattice sizes.
//
// Requests are admitted first-in first-out while their state and tables fit
// the HBM budget and a slot is free.  A worker thread advances every admitted
// run by up to chunk_steps substeps per round; runs of the same lattice and
// precision share one launch per pass (each instance at its own step offset),
// so a run that arrives while others are on the GPU joins at the next round.
// A finished run is read out on the GPU (energy, plaquettes, Gauss law) and its
// memory goes back to the budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "lgt_internal.hpp"

using namespace lgt;

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Shape {
    int d, L[3], dtype;
    bool operator<(const Shape &o) const
    {
        if (d != o.d) return d < o.d;
        if (dtype != o.dtype) return dtype < o.dtype;
        return std::memcmp(L, o.L, sizeof L) < 0;
    }
};

struct ShapeRes {
    Lattice lat;
    uint32_t *ptab_dev = nullptr;
    size_t state_bytes = 0;
};

struct Run {
    uint64_t ticket = 0;
    Shape shape{};
    const ShapeRes *sr = nullptr;  // stable pointer into the server's shape map
    bool admitted = false;         // footprint counted against the budget
    lgt_schedule sched{};
    std::vector<double> cx_copy, cz_copy;
    int order = LGT_ORDER_TROTTER;
    size_t footprint = 0;
    Clock::time_point t_submit, t_admit;
    // resident state (valid while admitted)
    void *psi = nullptr;
    void *tables = nullptr;        // rot | phase
    size_t rot_bytes = 0;
    int n_total = 0, pre = 0, step = 0;
    int adv = 0;                   // steps the run advances in the current round
    std::vector<uint8_t> forms;   // per step: 1 tan-form, 2 cot-form link rotation
    double cx_last = 0, cz_last = 0;
    std::vector<char> blob;        // host copy of the tables, built on the submitting thread
    std::atomic<bool> cancel{false};        // stop at the next round boundary (lgt_server_cancel)
    std::atomic<bool> inject_fault{false};  // test hook: the run's next launch group fails
};

// the run's rot | phase tables (rounded for its dtype), built when it is submitted so that
// the worker thread only uploads them
void build_tables(const Lattice &lat, int dtype, Run *r, const std::vector<double> &cx,
                  const std::vector<double> &cz, double dt)
{
    const int n = lat.n_links;
    r->cx_last = cx.back();
    r->cz_last = cz.back();
    StepTables st;
    build_step_tables(n, lat.n_plaq, dt, cx.data(), cz.data(), (int)cx.size(), r->order, st);
    auto pack = [&](const auto &rot, const auto &ph) {
        r->rot_bytes = (rot.size() * sizeof(rot[0]) + 255) & ~(size_t)255;
        r->blob.resize(r->rot_bytes + ph.size() * sizeof(ph[0]));
        std::memcpy(r->blob.data(), rot.data(), rot.size() * sizeof(rot[0]));
        std::memcpy(r->blob.data() + r->rot_bytes, ph.data(), ph.size() * sizeof(ph[0]));
    };
    if (dtype == LGT_C64) {
        std::vector<RotParam<float>> rot;
        std::vector<Cplx<float>> ph;
        round_tables_f32(st, n, lat.n_plaq, rot, ph);
        pack(rot, ph);
    } else {
        std::vector<RotParam<double>> rot;
        std::vector<Cplx<double>> ph;
        round_tables_f64(st, lat.n_plaq, rot, ph);
        pack(rot, ph);
    }
    r->n_total = st.n_steps;
    r->pre = st.pre_phase;
    r->forms.resize(st.n_steps);
    for (int j = 0; j < st.n_steps; ++j) r->forms[j] = (st.rot_u[j] == 1.0) ? 1 : 2;
}

}  // namespace

struct lgt_server {
    size_t budget = 0, used = 0;
    int max_slots = 0, chunk = 0, device = 0;
    hipStream_t stream = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Run *> pending;
    std::vector<Run *> active;
    std::map<uint64_t, lgt_result> results;
    std::map<uint64_t, Run *> live;   // queued and admitted runs by ticket
    std::map<Shape, ShapeRes> shapes;
    uint64_t next_ticket = 1;
    bool stop = false;
    uint64_t n_ok = 0, n_failed = 0, n_cancelled = 0;   // finished runs by outcome
    std::thread worker;
    // device scratch owned by the worker
    DevInst *inst_dev = nullptr;
    size_t inst_cap = 0;
    double *partials = nullptr;
    std::vector<double> partials_host;
    uint64_t *masks_dev = nullptr;
    void *stage = nullptr;
    size_t stage_cap = 0;
};

namespace {

constexpr int kParts = 2048 * (kMaxPlaq + 1);
// longest run (and round) the server takes, the step limit of one lgt_evolve call
constexpr int64_t kMaxRunSteps = (int64_t)1 << 24;
// state bytes of one launch group that stay in the 256 MB Infinity Cache between passes
constexpr size_t kCacheStateBytes = (size_t)160 << 20;

// Steps a run of this state size advances per round: chunk_steps for the states whose
// steps stream the state (24-link complex64, 128 MiB, about 54 us a step, and larger),
// up to 4x more for small states, whose steps cost about one launch each (7 us), so that
// small runs are not held to the pace of large ones.  (Up to 8x, a round's device time
// per shape about even, halved the median latency of the served mix again but raised
// its 99th percentile by a fifth.)  The count depends on the run's shape alone, so a run takes the same
// steps in every round whether it runs alone or in a mix.
int round_steps(int chunk, size_t state_bytes)
{
    const double t_step = std::max(7e-6, 2.0 * (double)state_bytes / 5e12);
    const double ref = 2.0 * (double)((size_t)128 << 20) / 5e12;
    const int64_t k = std::lround(std::min(4.0, std::max(1.0, ref / t_step)));
    return (int)std::min<int64_t>((int64_t)chunk * k, kMaxRunSteps);
}

size_t elem_bytes(int dtype) { return dtype == LGT_C64 ? 8 : 16; }

hipError_t stage_to_device(lgt_server *s, void *dst, const void *src, size_t n)
{
    if (s->stage_cap < n) {
        if (s->stage) (void)hipHostFree(s->stage);
        s->stage = nullptr;
        s->stage_cap = 0;
        hipError_t e = hipHostMalloc(&s->stage, n, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        s->stage_cap = n;
    }
    std::memcpy(s->stage, src, n);
    hipError_t e = hipMemcpyAsync(dst, s->stage, n, hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s->stream);   // staging buffer reused right after
}

// sum of per-block partials over the masks of one reduction launch
hipError_t reduce(lgt_server *s, int dtype, const void *psi, int n, bool flip,
                  const uint64_t *masks, int n_masks, std::vector<long double> &out)
{
    const int chunk = flip ? 8 : 32;
    const int g = flip ? reduce_blocks(n) : reduce_diag_blocks(n);
    out.assign(n_masks, 0.0L);
    for (int k0 = 0; k0 < n_masks; k0 += chunk) {
        const int m = std::min(chunk, n_masks - k0);
        hipError_t e = hipMemcpyAsync(s->masks_dev, masks + k0, sizeof(uint64_t) * m,
                                      hipMemcpyHostToDevice, s->stream);
        if (e != hipSuccess) return e;
        e = flip ? launch_reduce_flip(dtype, psi, n, s->masks_dev, m, s->partials, s->stream)
                 : launch_reduce_diag(dtype, psi, n, s->masks_dev, m, s->partials, s->stream);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(s->partials_host.data(), s->partials, sizeof(double) * g * chunk,
                           hipMemcpyDeviceToHost, s->stream);
        if (e != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s->stream)) != hipSuccess) return e;
        for (int i = 0; i < m; ++i) {
            long double acc = 0;
            for (int b = 0; b < g; ++b) acc += s->partials_host[(size_t)b * chunk + i];
            out[k0 + i] = acc;
        }
    }
    return hipSuccess;
}

hipError_t readout(lgt_server *s, Run *r, lgt_result &res)
{
    const Lattice &lat = r->sr->lat;
    const int n = lat.n_links;
    std::vector<uint64_t> diag(1, 0ull);
    diag.insert(diag.end(), lat.plaq_mask.begin(), lat.plaq_mask.end());
    std::vector<uint64_t> flip;
    for (int q = 0; q < n; ++q) flip.push_back(1ull << q);
    flip.insert(flip.end(), lat.star_mask.begin(), lat.star_mask.end());
    std::vector<long double> vd, vf;
    hipError_t e = reduce(s, r->shape.dtype, r->psi, n, false, diag.data(), (int)diag.size(), vd);
    if (e != hipSuccess) return e;
    e = reduce(s, r->shape.dtype, r->psi, n, true, flip.data(), (int)flip.size(), vf);
    if (e != hipSuccess) return e;
    const long double nrm = vd[0];
    long double plaq = 0, sx = 0, gv = 0;
    for (int p = 0; p < lat.n_plaq; ++p) plaq += vd[1 + p];
    for (int q = 0; q < n; ++q) sx += vf[q];
    for (int i = 0; i < lat.n_sites; ++i)
        gv = std::max(gv, std::fabs(1.0L - vf[n + i] / nrm));
    res.norm = (double)nrm;
    res.plaq_mean = (double)(plaq / nrm / lat.n_plaq);
    res.energy = (double)((-(long double)r->cx_last * sx - (long double)r->cz_last * plaq) / nrm);
    res.gauss_violation = (double)gv;
    return hipSuccess;
}

void finish(lgt_server *s, Run *r, lgt_status st, const lgt_result *res_in)
{
    lgt_result res{};
    if (res_in) res = *res_in;
    res.done = 1;
    res.status = st;
    const auto now = Clock::now();
    res.latency_ms = ms_between(r->t_submit, now);
    res.queue_ms = (r->t_admit.time_since_epoch().count() ? ms_between(r->t_submit, r->t_admit)
                                                           : res.latency_ms);
    if (r->psi) (void)hipFreeAsync(r->psi, s->stream);
    if (r->tables) (void)hipFreeAsync(r->tables, s->stream);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (r->admitted) s->used -= r->footprint;
        s->results[r->ticket] = res;
        s->live.erase(r->ticket);
        if (st == LGT_OK) ++s->n_ok;
        else if (st == LGT_E_STATE) ++s->n_cancelled;
        else ++s->n_failed;
    }
    s->cv_done.notify_all();
    delete r;
}

// allocate, upload tables and prepare |+>^N (plus the leading half phase)
lgt_status admit(lgt_server *s, Run *r)
{
    const ShapeRes &sr = *r->sr;
    const Lattice &lat = sr.lat;
    const int n = lat.n_links, dtype = r->shape.dtype;
    const std::vector<char> &blob = r->blob;
    r->step = 0;
    if (hipMallocAsync(&r->psi, sr.state_bytes, s->stream) != hipSuccess) return LGT_E_OOM;
    if (hipMallocAsync(&r->tables, blob.size() + 256, s->stream) != hipSuccess) return LGT_E_OOM;
    if (stage_to_device(s, r->tables, blob.data(), blob.size()) != hipSuccess) return LGT_E_DEVICE;
    const double amp = std::ldexp(1.0, -n / 2) * ((n & 1) ? std::sqrt(0.5) : 1.0);
    if (launch_init(dtype, r->psi, n, LGT_INIT_PLUS, 0, amp, sr.ptab_dev, s->stream) != hipSuccess)
        return LGT_E_DEVICE;
    if (r->pre) {
        DevInst di{};
        di.psi = r->psi;
        di.rot = r->tables;
        di.phase = (char *)r->tables + r->rot_bytes;
        di.ptab = sr.ptab_dev;
        di.n_total = r->n_total;
        if (stage_to_device(s, s->inst_dev, &di, sizeof di) != hipSuccess) return LGT_E_DEVICE;
        if (launch_phase(dtype, s->inst_dev, 1, n, 0, lat.n_plaq, s->stream) != hipSuccess)
            return LGT_E_DEVICE;
        if (hipStreamSynchronize(s->stream) != hipSuccess) return LGT_E_DEVICE;
    }
    r->t_admit = Clock::now();
    return LGT_OK;
}

// finish every run of `runs` with `st`, under no lock; the server's lists are updated by
// the caller
void finish_all(lgt_server *s, const std::vector<Run *> &runs, lgt_status st)
{
    for (Run *r : runs) finish(s, r, st, nullptr);
}

void worker_loop(lgt_server *s)
{
    (void)hipSetDevice(s->device);
    for (;;) {
        std::vector<Run *> newly, cancelled;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty() || !s->active.empty(); });
            if (s->stop && s->active.empty()) {
                // cancel what was never admitted
                while (!s->pending.empty()) {
                    Run *r = s->pending.front();
                    s->pending.pop_front();
                    lgt_result res{};
                    res.done = 1;
                    res.status = LGT_E_STATE;
                    res.latency_ms = ms_between(r->t_submit, Clock::now());
                    s->results[r->ticket] = res;
                    s->live.erase(r->ticket);
                    ++s->n_cancelled;
                    delete r;
                }
                s->cv_done.notify_all();
                return;
            }
            // runs cancelled while admitted stop at this round boundary
            std::vector<Run *> keep;
            for (Run *r : s->active) (r->cancel ? cancelled : keep).push_back(r);
            s->active.swap(keep);
            // FIFO admission by slot and HBM footprint
            while (!s->stop && !s->pending.empty() &&
                   (int)(s->active.size() + newly.size()) < s->max_slots &&
                   s->used + s->pending.front()->footprint <= s->budget) {
                Run *r = s->pending.front();
                s->pending.pop_front();
                s->used += r->footprint;
                r->admitted = true;
                newly.push_back(r);
            }
        }
        finish_all(s, cancelled, LGT_E_STATE);
        for (Run *r : newly) {
            lgt_status st = admit(s, r);
            if (st != LGT_OK) {
                finish(s, r, st, nullptr);
                continue;
            }
            std::lock_guard<std::mutex> lk(s->mu);
            s->active.push_back(r);
        }
        std::vector<Run *> act;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            act = s->active;
        }
        if (act.empty()) continue;
        // one batched launch sequence per lattice shape, split into groups whose states
        // fit the Infinity Cache together when each state does (the groups run one after
        // the other on the server's stream)
        std::map<Shape, std::vector<Run *>> groups;
        for (Run *r : act) groups[r->shape].push_back(r);
        std::vector<std::vector<Run *>> lgroups;
        for (auto &g : groups) {
            const size_t sb = g.second[0]->sr->state_bytes;
            const size_t per = sb <= kCacheStateBytes ? std::max<size_t>(1, kCacheStateBytes / sb)
                                                      : g.second.size();
            for (size_t i = 0; i < g.second.size(); i += per)
                lgroups.emplace_back(g.second.begin() + i,
                                     g.second.begin() + std::min(g.second.size(), i + per));
        }
        size_t need = 0;
        for (auto &g : lgroups) need += ((g.size() * sizeof(DevInst)) + 255) & ~(size_t)255;
        if (s->inst_cap < need) {
            (void)hipStreamSynchronize(s->stream);
            if (s->inst_dev) (void)hipFree(s->inst_dev);
            s->inst_dev = nullptr;
            s->inst_cap = 0;
            if (hipMalloc((void **)&s->inst_dev, need * 2) != hipSuccess) {
                finish_all(s, act, LGT_E_OOM);
                std::lock_guard<std::mutex> lk(s->mu);
                s->active.clear();
                continue;
            }
            s->inst_cap = need * 2;
        }
        std::vector<char> host(need);
        size_t off = 0;
        std::vector<size_t> offs;
        for (auto &g : lgroups) {
            const ShapeRes &sr = *g[0]->sr;
            DevInst *di = (DevInst *)(host.data() + off);
            for (size_t i = 0; i < g.size(); ++i) {
                Run *r = g[i];
                di[i] = DevInst{};
                di[i].psi = r->psi;
                di[i].rot = r->tables;
                di[i].phase = (char *)r->tables + r->rot_bytes;
                di[i].ptab = sr.ptab_dev;
                di[i].step0 = r->step;
                di[i].ph0 = r->step + r->pre;
                di[i].n_total = r->n_total;
            }
            offs.push_back(off);
            off += ((g.size() * sizeof(DevInst)) + 255) & ~(size_t)255;
        }
        // a group whose launches fail ends its own runs; the others go on.  A failed upload
        // or stream synchronisation ends every run of the round.
        bool round_fail = stage_to_device(s, s->inst_dev, host.data(), need) != hipSuccess;
        std::vector<char> group_fail(lgroups.size(), 0);
        for (size_t gi = 0; gi < lgroups.size() && !round_fail; ++gi) {
            const std::vector<Run *> &g = lgroups[gi];
            const ShapeRes &sr = *g[0]->sr;
            int steps = 0;
            for (Run *r : g) steps = std::max(steps, r->n_total - r->step);
            steps = std::min(steps, round_steps(s->chunk, sr.state_bytes));
            for (Run *r : g) r->adv = steps;
            bool inject = false;
            for (Run *r : g) inject = inject || r->inject_fault;
            if (inject) {
                // test hook: the group's launch reports a failure; nothing is launched
                group_fail[gi] = 1;
                continue;
            }
            std::vector<uint8_t> forms(steps, 0);
            for (Run *r : g)
                for (int j = 0; j < steps && r->step + j < r->n_total; ++j) forms[j] |= r->forms[r->step + j];
            if (enqueue_fused_steps(g[0]->shape.dtype, sr.lat.n_links, sr.lat.n_plaq,
                                    (const DevInst *)((char *)s->inst_dev + offs[gi]), (int)g.size(),
                                    steps, -1, 0, forms.data(), 0, s->stream, nullptr) != hipSuccess)
                group_fail[gi] = 1;
        }
        if (!round_fail && hipStreamSynchronize(s->stream) != hipSuccess) round_fail = true;
        std::vector<Run *> still;
        for (size_t gi = 0; gi < lgroups.size(); ++gi) {
            for (Run *r : lgroups[gi]) {
                if (round_fail || group_fail[gi]) {
                    finish(s, r, LGT_E_DEVICE, nullptr);
                    continue;
                }
                r->step = std::min(r->n_total, r->step + r->adv);
                if (r->step >= r->n_total) {
                    lgt_result res{};
                    const bool ok = readout(s, r, res) == hipSuccess;
                    finish(s, r, ok ? LGT_OK : LGT_E_DEVICE, &res);
                } else {
                    still.push_back(r);
                }
            }
        }
        std::lock_guard<std::mutex> lk(s->mu);
        // runs cancelled during the round stay listed until the next round boundary
        s->active = still;
    }
}

// queue a run: validate and copy the request, build its tables on the caller's thread
lgt_status submit_run(lgt_server *s, const lgt_request *req, uint64_t *ticket)
{
    Shape sh{};
    sh.d = req->d;
    sh.dtype = req->dtype;
    for (int i = 0; i < 3; ++i) sh.L[i] = (i < req->d) ? req->L[i] : 1;
    std::unique_ptr<Run> r(new Run());
    r->t_submit = Clock::now();
    r->shape = sh;
    r->sched = req->sched;
    r->order = req->order;
    if (req->sched.ramp == LGT_RAMP_EXPLICIT) {
        if (!req->sched.cx || !req->sched.cz) return LGT_E_INVALID;
        r->cx_copy.assign(req->sched.cx, req->sched.cx + req->sched.n_steps);
        r->cz_copy.assign(req->sched.cz, req->sched.cz + req->sched.n_steps);
        r->sched.cx = r->cx_copy.data();
        r->sched.cz = r->cz_copy.data();
    }
    double dt;
    std::vector<double> cx, cz;
    if (!schedule_coeffs(&r->sched, 0, r->sched.n_steps, dt, cx, cz).empty()) return LGT_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->shapes.find(sh);
    if (it == s->shapes.end()) {
        ShapeRes sr;
        std::string why = build_lattice(req->d, req->L, sr.lat);
        if (!why.empty())
            return why.find("too many") != std::string::npos ? LGT_E_UNSUPPORTED : LGT_E_INVALID;
        uint32_t tab[kParityBytes][256];
        build_parity_tables(sr.lat, tab);
        if (hipSetDevice(s->device) != hipSuccess || hipMalloc((void **)&sr.ptab_dev, sizeof tab) != hipSuccess)
            return LGT_E_DEVICE;
        if (hipMemcpy(sr.ptab_dev, tab, sizeof tab, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(sr.ptab_dev);
            return LGT_E_DEVICE;
        }
        sr.state_bytes = ((size_t)1 << sr.lat.n_links) * elem_bytes(sh.dtype);
        it = s->shapes.emplace(sh, std::move(sr)).first;
    }
    const ShapeRes &sr = it->second;
    r->sr = &it->second;
    const size_t steps = (size_t)r->sched.n_steps;
    r->footprint = sr.state_bytes + steps * 2 * 8 * (sh.dtype == LGT_C64 ? 1 : 2) +
                   (steps + 1) * (sr.lat.n_plaq + 1) * elem_bytes(sh.dtype) + 1024;
    if (r->footprint > s->budget) return LGT_E_OOM;
    // the tables are built here, on the caller's thread, outside the lock (the shape's
    // lattice stays put in the map)
    lk.unlock();
    build_tables(sr.lat, sh.dtype, r.get(), cx, cz, dt);
    lk.lock();
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->results[r->ticket] = lgt_result{};
    s->live[r->ticket] = r.get();
    s->pending.push_back(r.release());
    lk.unlock();
    s->cv_work.notify_one();
    return LGT_OK;
}

// the queued or admitted run holding `ticket`, or null (call with the lock held)
Run *find_run(lgt_server *s, uint64_t ticket)
{
    auto it = s->live.find(ticket);
    return it == s->live.end() ? nullptr : it->second;
}

}  // namespace

extern "C" {

lgt_status lgt_server_create(size_t hbm_budget, int max_slots, int chunk_steps, lgt_server **out)
{
    if (!out || max_slots < 1 || max_slots > 65535 || chunk_steps < 1 || hbm_budget == 0)
        return LGT_E_INVALID;
    *out = nullptr;
    lgt_server *s = new (std::nothrow) lgt_server();
    if (!s) return LGT_E_OOM;
    s->budget = hbm_budget;
    s->max_slots = max_slots;
    // a round never needs more steps than the longest run takes
    s->chunk = (int)std::min<int64_t>(chunk_steps, kMaxRunSteps);
    if (hipGetDevice(&s->device) != hipSuccess ||
        hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc((void **)&s->partials, sizeof(double) * kParts) != hipSuccess ||
        hipMalloc((void **)&s->masks_dev, sizeof(uint64_t) * 64) != hipSuccess ||
        hipMalloc((void **)&s->inst_dev, 4096) != hipSuccess) {
        if (s->stream) (void)hipStreamDestroy(s->stream);
        if (s->partials) (void)hipFree(s->partials);
        if (s->masks_dev) (void)hipFree(s->masks_dev);
        delete s;
        return LGT_E_DEVICE;
    }
    s->inst_cap = 4096;
    s->partials_host.resize(kParts);
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return LGT_OK;
}

lgt_status lgt_server_submit(lgt_server *s, const lgt_request *req, uint64_t *ticket)
{
    if (!s || !req || !ticket) return LGT_E_INVALID;
    if (req->dtype != LGT_C64 && req->dtype != LGT_C128) return LGT_E_INVALID;
    if (req->order != LGT_ORDER_TROTTER && req->order != LGT_ORDER_SYMMETRIC) return LGT_E_INVALID;
    // the step count is checked before anything is copied or built from it
    if (req->sched.n_steps < 1 || req->sched.n_steps > kMaxRunSteps) return LGT_E_INVALID;
    if (req->d < 2 || req->d > 3) return LGT_E_INVALID;
    try {
        return submit_run(s, req, ticket);
    } catch (const std::bad_alloc &) {
        return LGT_E_OOM;
    } catch (...) {
        return LGT_E_INVALID;
    }
}

// a finished result is handed out once: the call that returns it also releases the ticket
lgt_status lgt_server_poll(lgt_server *s, uint64_t ticket, lgt_result *out)
{
    if (!s || !out) return LGT_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->results.find(ticket);
    if (it == s->results.end()) return LGT_E_INVALID;
    *out = it->second;
    if (out->done) s->results.erase(it);
    return LGT_OK;
}

lgt_status lgt_server_wait(lgt_server *s, uint64_t ticket, double timeout_ms, lgt_result *out)
{
    if (!s || !out) return LGT_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto ready = [&] {
        auto it = s->results.find(ticket);
        return it == s->results.end() || it->second.done;
    };
    if (timeout_ms < 0) s->cv_done.wait(lk, ready);
    else s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready);
    auto it = s->results.find(ticket);
    if (it == s->results.end()) return LGT_E_INVALID;
    *out = it->second;
    if (!out->done) return LGT_E_BUSY;
    s->results.erase(it);
    return LGT_OK;
}

lgt_status lgt_server_cancel(lgt_server *s, uint64_t ticket)
{
    if (!s) return LGT_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->results.find(ticket);
    if (it == s->results.end()) return LGT_E_INVALID;
    if (it->second.done) return LGT_E_STATE;
    for (auto q = s->pending.begin(); q != s->pending.end(); ++q) {
        if ((*q)->ticket != ticket) continue;
        Run *r = *q;
        s->pending.erase(q);
        lgt_result res{};
        res.done = 1;
        res.status = LGT_E_STATE;
        res.latency_ms = ms_between(r->t_submit, Clock::now());
        res.queue_ms = res.latency_ms;
        it->second = res;
        s->live.erase(ticket);
        ++s->n_cancelled;
        delete r;
        lk.unlock();
        s->cv_done.notify_all();
        return LGT_OK;
    }
    Run *r = find_run(s, ticket);
    if (!r) return LGT_E_STATE;   // finishing: its result is about to arrive
    r->cancel = true;              // admitted: stops at the next round boundary
    lk.unlock();
    s->cv_work.notify_one();
    return LGT_OK;
}

lgt_status lgt_server_inject_fault(lgt_server *s, uint64_t ticket)
{
    if (!s) return LGT_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    Run *r = find_run(s, ticket);
    if (!r) return LGT_E_INVALID;
    r->inject_fault = true;
    return LGT_OK;
}

lgt_status lgt_server_stats(lgt_server *s, lgt_server_stats_t *out)
{
    if (!s || !out) return LGT_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    out->budget_bytes = s->budget;
    out->used_bytes = s->used;
    out->pending = (int)s->pending.size();
    out->active = (int)s->active.size();
    out->completed = s->n_ok;
    out->failed = s->n_failed;
    out->cancelled = s->n_cancelled;
    uint64_t undelivered = 0;
    for (auto &kv : s->results) undelivered += kv.second.done ? 1 : 0;
    out->undelivered = undelivered;
    return LGT_OK;
}

lgt_status lgt_server_destroy(lgt_server *s)
{
    if (!s) return LGT_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    for (auto &kv : s->shapes)
        if (kv.second.ptab_dev) (void)hipFree(kv.second.ptab_dev);
    if (s->inst_dev) (void)hipFree(s->inst_dev);
    if (s->partials) (void)hipFree(s->partials);
    if (s->masks_dev) (void)hipFree(s->masks_dev);
    if (s->stage) (void)hipHostFree(s->stage);
    (void)hipStreamDestroy(s->stream);
    for (Run *r : s->pending) delete r;   // none left: the worker cancels the queue on exit
    delete s;
    return LGT_OK;
}

}  // extern "C"
