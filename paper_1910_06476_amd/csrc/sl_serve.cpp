// Request loop behind the C ABI of include/sl.h (sl_server_*): continuous
// batching of independent transport problems on one GPU.
//
// A request is one whole problem: mesh, velocity, optional ghost rows, dt,
// step count and options.  Requests wait in arrival order and are admitted
// while a slot is free and the device memory they need fits the budget.
//
// The loop runs on host threads of the server's own, started by the first
// sl_server_progress or sl_server_drain:
// * the worker sets requests up (mesh, velocity, ghost rows) and retires
//   finished ones (field and statistics to host memory, mesh freed).  All
//   requests admissible at one moment are set up (on up to four threads at
//   once) and then published together, so that requests of one kernel
//   variant submitted together start in the same tick.
// * the feeder notices finished requests and keeps every group's steps
//   queued on the device.
// The caller's own thread only submits and collects, so the device stays fed
// while the caller builds its next inputs.
//
// Memory: one device allocation (the arena, sized by the budget) made with
// the first admission; each admitted request takes one contiguous block of
// it (first fit) and its mesh carves its buffers from that block.  Streams:
// one per slot, kept for the server's life.  Admission and retirement thus
// allocate and free no device memory (freeing would wait for the device).
//
// Batched requests: admitted requests small enough that their own advect
// launch leaves the device partly idle (fewer than kBatchBlocks blocks) and
// whose steps share a kernel variant (dimension, nodes per direction, advect
// variant) form a group, and the
// feeder steps each group in ticks: one tick is one launch of each step
// kernel over the elements of all members with steps left, every block
// working for one member on that member's own buffers (the kernels' batched
// forms; a tick of one member launches the single-mesh kernels).  Members
// join at the next tick after they are published and leave after their last
// one.  Each group has its own stream, on which it keeps about two
// milliseconds of ticks queued ahead (by the measured tick time).  The
// launch arguments of a batched tick travel to the device through a ring of
// pinned host slots.
//
// Other requests (larger ones, steps that cannot join a batch, or a server
// created with SL_SERVER_NO_BATCH) queue all their steps at admission on
// their own stream, with an event after each, so they overlap with
// everything else.
//
// Locking: the device hold (sl::ApiHold) is always taken before the
// server's mutex, never after.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "sl_internal.h"

namespace {

enum { REQ_WAITING = 0, REQ_SETUP = 1, REQ_ACTIVE = 2, REQ_FINISHED = 3, REQ_DONE = 4 };

constexpr int kAheadMin = 2, kAheadMax = 64;  // ticks a group keeps queued and not finished
constexpr double kAheadMs = 2.0;              // ... enough for about this much device time
constexpr int kStages = 32;                   // pinned argument slots
constexpr size_t kBlockSlack = 8192;          // per request: the 256-byte alignment of its buffers
constexpr auto kFeedPoll = std::chrono::microseconds(100);
constexpr int kSetupThreads = 4;              // threads setting up one admission batch
constexpr int kBatchBlocks = 2048;            // batched: advect launches below this many blocks

double now_us()
{
    using namespace std::chrono;
    return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

struct Request {
    int64_t id = 0;
    int state = REQ_WAITING;
    sl_mesh_desc desc{};
    std::vector<double> u0, a, div, ghost;
    int32_t ghost_rows = 0;
    double dt = 0.0;
    int32_t nsteps = 0;
    sl_step_opts opts{};
    size_t bytes = 0;
    // while admitted
    size_t block_off = 0, block_len = 0;  // its block of the arena
    sl::BumpBlock bump;                   // the mesh's buffers, carved from the block
    hipStream_t stream = nullptr;         // the slot's stream
    sl_mesh* mesh = nullptr;
    sl_status setup_rc = SL_OK;
    sl::StepLaunch L{};
    hipEvent_t ready = nullptr;  // batched: after the set-up, for the group's stream to wait on
    std::vector<hipEvent_t> ev;  // unbatched: ev[0] before the first step, ev[k] after step k
    bool batched = false;
    int32_t launched = 0;        // batched: steps queued so far
    std::vector<int> ticks;      // batched: the ticks that carried its steps
    // when done
    std::vector<double> result;
    sl_stats stats{};
    sl_status status = SL_OK;
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;  // host clock, microseconds
    double device_ms = 0.0;                              // before the first to after the last step
    int64_t admit_seq = -1;
};

// one batched step of a group: events around its launches, and how many
// holders (its members and the group's queue) still have to read them
struct Tick {
    hipEvent_t start = nullptr, end = nullptr;
    int refs = 0;
};

using GroupKey = std::tuple<int, int, int>;  // dim, n, advect variant

struct Group {
    std::vector<Request*> members;  // in admission order
    hipStream_t stream = nullptr;   // the group's ticks
    char* dargs = nullptr;          // device: advect and constrain block offsets, then member arguments
    std::deque<int> queued;         // ticks queued and not yet seen finished
    double tick_ms = 0.05;          // running mean of its finished ticks' device time
};

// first fit over one device allocation, free ranges coalesced
struct Arena {
    char* base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free;  // offset -> length

    bool fits(size_t len) const
    {
        for (const auto& f : free)
            if (f.second >= len) return true;
        return false;
    }
    bool take(size_t len, size_t* off)
    {
        for (auto it = free.begin(); it != free.end(); ++it)
            if (it->second >= len) {
                *off = it->first;
                const size_t rest = it->second - len, at = it->first + len;
                free.erase(it);
                if (rest) free[at] = rest;
                return true;
            }
        return false;
    }
    void give(size_t off, size_t len)
    {
        auto it = free.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != free.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free.erase(nx);
        }
        if (it != free.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free.erase(it);
            }
        }
    }
};

}  // namespace

struct sl_server {
    int32_t max_active = 1;
    bool batch = true;
    size_t budget = 0, used = 0;
    int64_t next_id = 1;
    int64_t admitted = 0;
    std::deque<Request*> waiting;
    std::vector<Request*> active;   // published, stepping
    std::deque<Request*> finished;  // last step done, not yet retired
    int32_t slots = 0;              // requests in set-up, active, finished or being retired
    std::map<int64_t, std::unique_ptr<Request>> all;
    std::vector<float> step_ms;  // per-step device latencies of retired requests
    int64_t dof_updates = 0;     // of retired requests
    // device resources, made on first use and kept
    Arena arena;
    std::vector<hipStream_t> streams, free_streams;
    // batched work
    std::map<GroupKey, Group> groups;
    std::vector<Tick> ticks;
    std::vector<int> free_ticks;
    size_t slot_bytes = 0;
    char* stage = nullptr;  // pinned, kStages slots
    hipEvent_t stage_ev[kStages] = {};
    bool stage_used[kStages] = {};
    int stage_next = 0;
    int64_t batch_launches = 0, batch_member_steps = 0;
    // the loop's threads
    std::mutex mu;
    std::condition_variable cv_work, cv_feed, cv_done;
    std::thread worker, feeder;
    bool started = false, stop = false;
    int device = 0;
    sl_status error = SL_OK;  // first device error of the loop
};

namespace {

size_t args_bytes() { return std::max(sizeof(sl::Step1DArgs), sizeof(sl::Step2DArgs)); }

// bytes of the block offsets at the head of a slot (two tables of
// max_active + 1 ints, rounded to 256)
size_t head_bytes(int max_active) { return round256(2 * sizeof(int) * (size_t)(max_active + 1)); }

size_t block_bytes(const Request* r) { return round256(r->bytes) + kBlockSlack; }

void fail_loop(sl_server* s, sl_status rc)
{
    if (s->error == SL_OK) s->error = rc;
    s->cv_done.notify_all();
}

void free_events(Request* r)
{
    for (hipEvent_t e : r->ev) (void)hipEventDestroy(e);
    r->ev.clear();
    if (r->ready) (void)hipEventDestroy(r->ready);
    r->ready = nullptr;
}

// ticks keep their events when released, for the next tick to reuse
void release_tick(sl_server* s, int k)
{
    if (--s->ticks[(size_t)k].refs > 0) return;
    s->free_ticks.push_back(k);
}

int new_tick(sl_server* s)
{
    if (!s->free_ticks.empty()) {
        const int k = s->free_ticks.back();
        s->free_ticks.pop_back();
        return k;
    }
    Tick t;
    if (hipEventCreate(&t.start) != hipSuccess) return -1;
    if (hipEventCreate(&t.end) != hipSuccess) {
        (void)hipEventDestroy(t.start);
        return -1;
    }
    s->ticks.push_back(t);
    return (int)s->ticks.size() - 1;
}

// ---- admission -------------------------------------------------------------

// the arena, once: the budget plus each slot's rounding and alignment slack
// (so that any set of requests within the budget fits, fragmentation
// aside), within 90% of the device memory free now
sl_status ensure_arena(sl_server* s)
{
    if (s->arena.base) return SL_OK;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return SL_E_DEVICE;
    size_t want = round256(s->budget) + (kBlockSlack + 256) * (size_t)s->max_active;
    want = std::min(want, free_b / 10 * 9) / 256 * 256;
    if (want == 0 || hipMalloc((void**)&s->arena.base, want) != hipSuccess) {
        s->arena.base = nullptr;
        return SL_E_NOMEM;
    }
    s->arena.size = want;
    s->arena.free.clear();
    s->arena.free[0] = want;
    return SL_OK;
}

// the front waiting request can be admitted now (or must be failed: it can
// never fit the arena)
bool front_admissible(const sl_server* s)
{
    if (s->waiting.empty() || s->slots >= s->max_active) return false;
    const Request* r = s->waiting.front();
    if (s->used + r->bytes > s->budget) return false;
    if (!s->arena.base) return true;
    const size_t len = block_bytes(r);
    return len > s->arena.size || s->arena.fits(len);
}

hipStream_t take_stream(sl_server* s)
{
    if (!s->free_streams.empty()) {
        hipStream_t st = s->free_streams.back();
        s->free_streams.pop_back();
        return st;
    }
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return nullptr;
    s->streams.push_back(st);
    return st;
}

void finish_unadmitted(sl_server* s, Request* r, sl_status rc)
{
    r->status = rc;
    r->state = REQ_DONE;
    r->t_done = now_us();
    s->cv_done.notify_all();
}

// reserve a slot, budget, block and stream for a request taken from the
// front of the queue (under the lock); false if it was failed instead
bool reserve(sl_server* s, Request* r)
{
    sl_status rc = ensure_arena(s);
    const size_t len = block_bytes(r);
    if (rc == SL_OK && len > s->arena.size) rc = SL_E_NOMEM;
    size_t off = 0;
    if (rc == SL_OK && !s->arena.take(len, &off)) rc = SL_E_NOMEM;  // front_admissible checked the fit
    hipStream_t st = rc == SL_OK ? take_stream(s) : nullptr;
    if (rc == SL_OK && !st) {
        s->arena.give(off, len);
        rc = SL_E_DEVICE;
    }
    if (rc != SL_OK) {
        finish_unadmitted(s, r, rc);
        return false;
    }
    r->block_off = off;
    r->block_len = len;
    r->bump = sl::BumpBlock{s->arena.base + off, len, 0};
    r->stream = st;
    r->state = REQ_SETUP;
    r->t_admit = now_us();
    r->admit_seq = s->admitted++;
    s->used += r->bytes;
    s->slots += 1;
    return true;
}

// unbatched: every step queued at once on the request's stream
sl_status launch_all(Request* r)
{
    sl_status rc = SL_OK;
    r->ev.resize((size_t)r->nsteps + 1, nullptr);
    for (auto& e : r->ev)
        if (hipEventCreate(&e) != hipSuccess) rc = SL_E_DEVICE;
    if (rc == SL_OK && hipEventRecord(r->ev[0], r->stream) != hipSuccess) rc = SL_E_DEVICE;
    for (int32_t k = 1; rc == SL_OK && k <= r->nsteps; ++k) {
        rc = sl_step(r->mesh, r->dt, 1, &r->opts);
        if (rc == SL_OK && hipEventRecord(r->ev[k], r->stream) != hipSuccess) rc = SL_E_DEVICE;
    }
    return rc;
}

// set-up of one reserved request, outside the lock: the mesh in its block on
// its stream, velocity, ghost rows; then either all its steps queued, or an
// event for its group to start after
void prepare(bool batch, Request* r)
{
    sl_mesh_desc d = r->desc;
    d.u0 = r->u0.data();
    d.stream = r->stream;
    sl::tl_bump = &r->bump;
    sl_status rc = sl_create_mesh(&d, &r->mesh);
    if (rc == SL_OK) rc = sl_set_velocity(r->mesh, r->a.data(), r->div.empty() ? nullptr : r->div.data());
    if (rc == SL_OK && r->ghost_rows > 0) rc = sl_set_ghost(r->mesh, r->ghost.data(), r->ghost_rows);
    sl::tl_bump = nullptr;
    if (rc == SL_OK) rc = sl::step_prepare(r->mesh, r->dt, r->opts, &r->L);  // validates the options
    r->batched = rc == SL_OK && batch && r->nsteps > 0 && r->L.variant >= 0 && r->L.adv_blocks < kBatchBlocks;
    if (rc == SL_OK && r->batched) {
        if (hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(r->ready, r->stream) != hipSuccess)
            rc = SL_E_DEVICE;
    } else if (rc == SL_OK) {
        rc = launch_all(r);
    }
    r->setup_rc = rc;
}

// set up a batch of reserved requests on up to kSetupThreads threads (this
// one included; the helpers take the device hold themselves)
void prepare_all(int device, bool batch, const std::vector<Request*>& rs)
{
    std::atomic<size_t> next{0};
    auto run = [&] {
        for (size_t k; (k = next.fetch_add(1)) < rs.size();) prepare(batch, rs[k]);
    };
    std::vector<std::thread> helpers;
    const size_t nh = std::min(rs.size(), (size_t)kSetupThreads) - 1;
    for (size_t h = 0; h < nh; ++h) {
        try {
            helpers.emplace_back([&, device] {
                (void)hipSetDevice(device);
                const sl::ApiHold hold;
                run();
            });
        } catch (...) {
            break;  // fewer helpers: this thread does the rest
        }
    }
    run();
    for (std::thread& t : helpers) t.join();
}

// give back what an admitted request holds (under the lock)
void unreserve(sl_server* s, Request* r)
{
    s->arena.give(r->block_off, r->block_len);
    s->free_streams.push_back(r->stream);
    r->stream = nullptr;
    s->used -= r->bytes;
    s->slots -= 1;
}

// pinned argument slots and their events of the batched work
sl_status batch_resources(sl_server* s)
{
    if (s->stage) return SL_OK;
    char* stage = nullptr;
    if (hipHostMalloc((void**)&stage, s->slot_bytes * kStages, hipHostMallocDefault) != hipSuccess) return SL_E_NOMEM;
    for (int k = 0; k < kStages; ++k)
        if (hipEventCreateWithFlags(&s->stage_ev[k], hipEventDisableTiming) != hipSuccess) {
            for (int j = 0; j < k; ++j) (void)hipEventDestroy(s->stage_ev[j]);
            (void)hipHostFree(stage);
            return SL_E_DEVICE;
        }
    s->stage = stage;
    return SL_OK;
}

// publish a prepared request (under the lock): into its group, or active
// with its steps already queued; a failed set-up finishes it
void publish(sl_server* s, Request* r)
{
    sl_status rc = r->setup_rc;
    if (rc == SL_OK && r->batched) {
        rc = batch_resources(s);
        Group& g = s->groups[GroupKey(r->L.dim, r->L.n, r->L.variant)];
        if (rc == SL_OK && !g.stream && hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking) != hipSuccess) {
            g.stream = nullptr;
            rc = SL_E_DEVICE;
        }
        if (rc == SL_OK && !g.dargs && hipMalloc((void**)&g.dargs, s->slot_bytes) != hipSuccess) {
            g.dargs = nullptr;
            rc = SL_E_NOMEM;
        }
        if (rc == SL_OK && hipStreamWaitEvent(g.stream, r->ready, 0) != hipSuccess) rc = SL_E_DEVICE;
        if (rc == SL_OK) g.members.push_back(r);
    }
    if (rc != SL_OK) {
        (void)hipStreamSynchronize(r->stream);  // steps queued before the failure
        free_events(r);
        if (r->mesh) sl_destroy_mesh(r->mesh);
        r->mesh = nullptr;
        unreserve(s, r);
        finish_unadmitted(s, r, rc);
        return;
    }
    r->state = REQ_ACTIVE;
    s->active.push_back(r);
}

// ---- ticks -----------------------------------------------------------------

// a pinned argument slot free for the host to fill (its last copy done)
char* take_slot(sl_server* s, int* slot)
{
    const int k = s->stage_next;
    s->stage_next = (k + 1) % kStages;
    if (s->stage_used[k] && hipEventSynchronize(s->stage_ev[k]) != hipSuccess) return nullptr;
    s->stage_used[k] = false;
    *slot = k;
    return s->stage + (size_t)k * s->slot_bytes;
}

// queue one tick of group g: one step of every member with steps left
sl_status queue_tick(sl_server* s, const GroupKey& key, Group& g, bool* queued)
{
    *queued = false;
    std::vector<Request*> mem;
    for (Request* r : g.members)
        if (r->launched < r->nsteps) mem.push_back(r);
    if (mem.empty()) return SL_OK;
    const int nreq = (int)mem.size();
    const int dim = std::get<0>(key), n = std::get<1>(key);
    const int t = new_tick(s);
    if (t < 0) return SL_E_DEVICE;
    Tick& tk = s->ticks[(size_t)t];
    tk.refs = nreq + 1;  // the members and the group's queue
    g.queued.push_back(t);
    int bad = hipEventRecord(tk.start, g.stream) != hipSuccess;
    if (nreq == 1) {
        // one member: the single-mesh kernels, arguments by value
        sl::StepLaunch L;
        const sl_status rc = sl::step_prepare(mem[0]->mesh, mem[0]->dt, mem[0]->opts, &L);
        if (rc != SL_OK) return rc;
        if (dim == 1)
            bad |= sl::launch_advect1d(n, L.a1, g.stream) | sl::launch_constrain1d(n, L.a1, g.stream);
        else
            bad |= sl::launch_advect2d(n, L.a2, g.stream) | sl::launch_constrain2d(n, L.a2, g.stream);
    } else {
        int slot = 0;
        char* host = take_slot(s, &slot);
        if (!host) return SL_E_DEVICE;
        const size_t hb = head_bytes(s->max_active);
        int* adv_start = (int*)host;
        int* con_start = adv_start + s->max_active + 1;
        char* args = host + hb;
        const size_t as = dim == 1 ? sizeof(sl::Step1DArgs) : sizeof(sl::Step2DArgs);
        sl::StepLaunch L0;
        adv_start[0] = con_start[0] = 0;
        for (int k = 0; k < nreq; ++k) {
            sl::StepLaunch L;
            const sl_status rc = sl::step_prepare(mem[(size_t)k]->mesh, mem[(size_t)k]->dt, mem[(size_t)k]->opts, &L);
            if (rc != SL_OK) return rc;
            if (k == 0) L0 = L;
            // packed at the arguments' own size: the kernels index As[r]
            std::memcpy(args + as * (size_t)k, dim == 1 ? (const void*)&L.a1 : (const void*)&L.a2, as);
            adv_start[k + 1] = adv_start[k] + L.adv_blocks;
            con_start[k + 1] = con_start[k] + L.con_blocks;
        }
        // the offsets and the members' arguments, nothing beyond
        if (hipMemcpyAsync(g.dargs, host, hb + as * (size_t)nreq, hipMemcpyHostToDevice, g.stream) != hipSuccess ||
            hipEventRecord(s->stage_ev[slot], g.stream) != hipSuccess)
            return SL_E_DEVICE;
        s->stage_used[slot] = true;
        const int* dadv = (const int*)g.dargs;
        const int* dcon = dadv + s->max_active + 1;
        if (dim == 1) {
            const auto* dA = (const sl::Step1DArgs*)(g.dargs + hb);
            bad |= sl::launch_advect1d_batch(n, L0.a1, dA, dadv, nreq, adv_start[nreq], g.stream);
            bad |= sl::launch_constrain1d_batch(n, dA, dcon, nreq, con_start[nreq], g.stream);
        } else {
            const auto* dA = (const sl::Step2DArgs*)(g.dargs + hb);
            bad |= sl::launch_advect2d_batch(n, L0.a2, dA, dadv, nreq, adv_start[nreq], g.stream);
            bad |= sl::launch_constrain2d_batch(n, dA, dcon, nreq, con_start[nreq], g.stream);
        }
    }
    bad |= hipEventRecord(tk.end, g.stream) != hipSuccess;
    for (Request* r : mem) {
        sl::step_commit(r->mesh, r->dt);
        r->launched += 1;
        r->ticks.push_back(t);
    }
    s->batch_launches += 1;
    s->batch_member_steps += nreq;
    *queued = true;
    return bad ? SL_E_DEVICE : SL_OK;
}

// keep about kAheadMs of every group's ticks queued (kAheadMin..kAheadMax)
sl_status queue_ticks(sl_server* s)
{
    for (auto& kv : s->groups) {
        Group& g = kv.second;
        while (!g.queued.empty()) {  // forget finished ticks, learning their time
            const Tick& t = s->ticks[(size_t)g.queued.front()];
            const hipError_t q = hipEventQuery(t.end);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) return SL_E_DEVICE;
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, t.start, t.end) == hipSuccess) g.tick_ms = 0.8 * g.tick_ms + 0.2 * ms;
            release_tick(s, g.queued.front());
            g.queued.pop_front();
        }
        const int ahead = std::max(kAheadMin, std::min(kAheadMax, (int)(kAheadMs / std::max(g.tick_ms, 1e-3))));
        while ((int)g.queued.size() < ahead) {
            bool queued = false;
            const sl_status rc = queue_tick(s, kv.first, g, &queued);
            if (rc != SL_OK) return rc;
            if (!queued) break;
        }
    }
    return SL_OK;
}

// the event after a request's last step (null while not all are queued)
hipEvent_t last_event(const sl_server* s, const Request* r)
{
    if (!r->batched) return r->ev.empty() ? nullptr : r->ev.back();
    if (r->launched < r->nsteps || r->ticks.empty()) return nullptr;
    return s->ticks[(size_t)r->ticks.back()].end;
}

// active requests whose last step has finished move to the worker
sl_status collect_finished(sl_server* s, bool* moved)
{
    for (size_t i = 0; i < s->active.size();) {
        Request* r = s->active[i];
        const hipEvent_t last = last_event(s, r);
        const hipError_t q = (r->batched && r->nsteps == 0) ? hipSuccess
                             : last                          ? hipEventQuery(last)
                                                             : hipErrorNotReady;
        if (q == hipSuccess) {
            r->state = REQ_FINISHED;
            s->finished.push_back(r);
            s->active.erase(s->active.begin() + (long)i);
            *moved = true;
        } else if (q == hipErrorNotReady) {
            ++i;
        } else {
            return SL_E_DEVICE;
        }
    }
    return SL_OK;
}

// ---- retirement ------------------------------------------------------------

// outside the lock: field and statistics to host, per-step latencies, mesh
// destroyed (its buffers stay in the block until unreserve)
void retire_read(Request* r, const std::vector<std::pair<hipEvent_t, hipEvent_t>>& tick_ev,
                 std::vector<float>* step_ms)
{
    const size_t nd = r->desc.dim == 1 ? (size_t)(r->desc.order + 1) : (size_t)(r->desc.order + 1) * (r->desc.order + 1);
    const size_t nf = (size_t)r->desc.kx * r->desc.ky * nd;
    r->result.resize(nf);
    if (r->batched) {
        // the group's stream may hold later ticks of others: read without
        // waiting on it (this request's last tick has finished)
        r->status = sl::read_settled(r->mesh, r->result.data(), &r->stats);
        for (const auto& e : tick_ev) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) step_ms->push_back(ms);
        }
        float tot = 0.0f;
        if (!tick_ev.empty() && hipEventElapsedTime(&tot, tick_ev.front().first, tick_ev.back().second) == hipSuccess)
            r->device_ms = tot;
    } else {
        r->status = sl_read(r->mesh, r->result.data(), &r->stats);
        for (size_t k = 1; k < r->ev.size(); ++k) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, r->ev[k - 1], r->ev[k]) == hipSuccess) step_ms->push_back(ms);
        }
        float tot = 0.0f;
        if (r->ev.size() > 1 && hipEventElapsedTime(&tot, r->ev.front(), r->ev.back()) == hipSuccess) r->device_ms = tot;
    }
    free_events(r);
    sl_destroy_mesh(r->mesh);
    r->mesh = nullptr;
}

// under the lock: the request's ticks, group place, block, stream and slot
void retire_commit(sl_server* s, Request* r, const std::vector<float>& step_ms)
{
    for (int k : r->ticks) release_tick(s, k);
    r->ticks.clear();
    if (r->batched) {
        auto it = s->groups.find(GroupKey(r->L.dim, r->L.n, r->L.variant));
        if (it != s->groups.end()) {
            auto& m = it->second.members;
            m.erase(std::remove(m.begin(), m.end(), r), m.end());
        }
    }
    s->step_ms.insert(s->step_ms.end(), step_ms.begin(), step_ms.end());
    s->dof_updates += (int64_t)r->result.size() * r->nsteps;
    unreserve(s, r);
    r->t_done = now_us();
    r->state = REQ_DONE;
}

// ---- the loop's threads ----------------------------------------------------

bool worker_has_work(const sl_server* s) { return !s->finished.empty() || front_admissible(s); }

void worker_loop(sl_server* s)
{
    (void)hipSetDevice(s->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stop || worker_has_work(s); });
            if (s->stop) return;
        }
        const sl::ApiHold hold;
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop) return;
        if (!s->finished.empty()) {
            Request* r = s->finished.front();
            s->finished.pop_front();
            std::vector<std::pair<hipEvent_t, hipEvent_t>> tick_ev;
            for (int k : r->ticks) tick_ev.emplace_back(s->ticks[(size_t)k].start, s->ticks[(size_t)k].end);
            lk.unlock();
            std::vector<float> ms;
            retire_read(r, tick_ev, &ms);
            lk.lock();
            retire_commit(s, r, ms);
            s->cv_done.notify_all();
            continue;
        }
        // every request admissible now, in arrival order; set up; published together
        std::vector<Request*> batch;
        while (front_admissible(s)) {
            Request* r = s->waiting.front();
            s->waiting.pop_front();
            if (reserve(s, r)) batch.push_back(r);
        }
        if (batch.empty()) continue;
        const bool batching = s->batch;
        lk.unlock();
        prepare_all(s->device, batching, batch);
        lk.lock();
        for (Request* r : batch) publish(s, r);
        s->cv_feed.notify_one();
    }
}

void feeder_loop(sl_server* s)
{
    (void)hipSetDevice(s->device);
    for (;;) {
        {
            const sl::ApiHold hold;
            std::lock_guard<std::mutex> lk(s->mu);
            if (s->stop) return;
            bool moved = false;
            sl_status rc = collect_finished(s, &moved);
            if (moved) s->cv_work.notify_one();
            if (rc == SL_OK && s->error == SL_OK) rc = queue_ticks(s);
            if (rc != SL_OK) fail_loop(s, rc);
        }
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop) return;
        if (s->active.empty() || s->error != SL_OK)
            s->cv_feed.wait(lk, [&] { return s->stop || (!s->active.empty() && s->error == SL_OK); });
        else
            s->cv_feed.wait_for(lk, kFeedPoll);
    }
}

// start the loop's threads once (under the device hold and the lock); if
// one cannot start, the server is stopped for good
sl_status start_loop(sl_server* s)
{
    if (s->started) return s->stop ? SL_E_NOMEM : SL_OK;
    if (hipGetDevice(&s->device) != hipSuccess) return SL_E_DEVICE;
    s->started = true;
    try {
        s->worker = std::thread(worker_loop, s);
        s->feeder = std::thread(feeder_loop, s);
    } catch (...) {
        s->stop = true;  // the threads started see it and end; destroy joins them
        s->cv_work.notify_all();
        s->cv_feed.notify_all();
        return SL_E_NOMEM;
    }
    return SL_OK;
}

}  // namespace

extern "C" {

sl_status sl_server_create(const sl_server_desc* d, sl_server** out)
{
    if (!out) return SL_E_INVALID;
    *out = nullptr;
    if (!d || d->max_active < 1 || d->max_active > 64 || d->hbm_budget == 0) return SL_E_INVALID;
    if (d->flags & ~SL_SERVER_NO_BATCH) return SL_E_INVALID;
    std::unique_ptr<sl_server> s(new (std::nothrow) sl_server());
    if (!s) return SL_E_NOMEM;
    s->max_active = d->max_active;
    s->budget = d->hbm_budget;
    s->batch = (d->flags & SL_SERVER_NO_BATCH) == 0;
    s->slot_bytes = head_bytes(s->max_active) + args_bytes() * (size_t)s->max_active;
    *out = s.release();  // host only: threads and device resources come later
    return SL_OK;
}

sl_status sl_server_submit(sl_server* s, const sl_request* q, int64_t* id)
{
    if (!s || !q || !id || !q->mesh.u0 || !q->a || q->nsteps < 0 || !(q->dt > 0)) return SL_E_INVALID;
    // requests are uniform meshes: the field, velocity and result are sized
    // from kx, ky and order, and the descriptor keeps no caller pointer
    if (q->mesh.orders) return SL_E_INVALID;
    if (q->mesh.bc != SL_BC_PERIODIC && (!q->ghost || q->ghost_rows < 1)) return SL_E_INVALID;
    std::unique_ptr<Request> r(new (std::nothrow) Request());
    if (!r) return SL_E_NOMEM;
    sl_status rc = sl_mesh_bytes(&q->mesh, q->mesh.bc != SL_BC_PERIODIC ? q->ghost_rows : 0, &r->bytes);
    if (rc != SL_OK) return rc;
    if (r->bytes > s->budget) return SL_E_NOMEM;  // could never be admitted
    const int n = q->mesh.order + 1;
    const size_t nd = q->mesh.dim == 1 ? (size_t)n : (size_t)n * n;
    const size_t nf = (size_t)q->mesh.kx * q->mesh.ky * nd;
    // the copies are made before taking the lock
    try {
        r->u0.assign(q->mesh.u0, q->mesh.u0 + nf);
        r->a.assign(q->a, q->a + nf * q->mesh.dim);
        if (q->div_a) r->div.assign(q->div_a, q->div_a + nf);
        if (q->mesh.bc != SL_BC_PERIODIC) {
            const size_t ng = q->mesh.dim == 1 ? 2 : (size_t)2 * n * (q->mesh.kx + q->mesh.ky);
            r->ghost.assign(q->ghost, q->ghost + ng * (size_t)q->ghost_rows);
            r->ghost_rows = q->ghost_rows;
        }
    } catch (...) {
        return SL_E_NOMEM;
    }
    r->desc = q->mesh;
    r->desc.u0 = nullptr;
    r->dt = q->dt;
    r->nsteps = q->nsteps;
    r->opts = q->opts;
    r->t_submit = now_us();
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    s->waiting.push_back(r.get());
    *id = r->id;
    s->all[r->id] = std::move(r);
    s->cv_work.notify_one();
    return SL_OK;
}

sl_status sl_server_progress(sl_server* s, int32_t* active, int32_t* waiting)
{
    if (!s) return SL_E_INVALID;
    const sl::ApiHold hold;
    std::lock_guard<std::mutex> lk(s->mu);
    const sl_status rc = start_loop(s);
    if (rc != SL_OK) return rc;
    if (active) *active = s->slots;
    if (waiting) *waiting = (int32_t)s->waiting.size();
    return s->error;
}

sl_status sl_server_drain(sl_server* s)
{
    if (!s) return SL_E_INVALID;
    {
        const sl::ApiHold hold;
        std::lock_guard<std::mutex> lk(s->mu);
        const sl_status rc = start_loop(s);
        if (rc != SL_OK) return rc;
    }
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->error != SL_OK || (s->waiting.empty() && s->slots == 0); });
    return s->error;
}

sl_status sl_server_result(sl_server* s, int64_t id, double* u_out, sl_stats* st, sl_request_timing* tm)
{
    if (!s) return SL_E_INVALID;
    std::unique_ptr<Request> r;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(id);
        if (it == s->all.end()) return SL_E_INVALID;
        if (it->second->state != REQ_DONE) return SL_E_STATE;
        r = std::move(it->second);
        s->all.erase(it);
    }
    if (u_out && !r->result.empty()) std::memcpy(u_out, r->result.data(), r->result.size() * sizeof(double));
    if (st) *st = r->stats;
    if (tm) {
        tm->queue_us = r->t_admit > 0 ? r->t_admit - r->t_submit : 0.0;
        tm->total_us = r->t_done - r->t_submit;
        tm->device_ms = r->device_ms;
        tm->bytes = r->bytes;
        tm->admit_seq = r->admit_seq;
    }
    return r->status;
}

sl_status sl_server_latency(sl_server* s, double p50_p99[2], int64_t* samples, int64_t* dof_updates)
{
    if (!s || !p50_p99) return SL_E_INVALID;
    std::vector<float> v;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        v = s->step_ms;
        if (dof_updates) *dof_updates = s->dof_updates;
    }
    p50_p99[0] = p50_p99[1] = 0.0;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        p50_p99[0] = v[std::min(v.size() - 1, (size_t)(0.50 * (double)v.size()))];
        p50_p99[1] = v[std::min(v.size() - 1, (size_t)(0.99 * (double)v.size()))];
    }
    if (samples) *samples = (int64_t)v.size();
    return SL_OK;
}

sl_status sl_server_batching(sl_server* s, int64_t* launches, int64_t* member_steps)
{
    if (!s) return SL_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    if (launches) *launches = s->batch_launches;
    if (member_steps) *member_steps = s->batch_member_steps;
    return SL_OK;
}

sl_status sl_server_destroy(sl_server* s)
{
    if (!s) return SL_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    s->cv_feed.notify_all();
    if (s->worker.joinable()) s->worker.join();
    if (s->feeder.joinable()) s->feeder.join();
    const sl::ApiHold hold;
    for (auto& kv : s->groups)
        if (kv.second.stream) (void)hipStreamSynchronize(kv.second.stream);
    for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
    for (auto& kv : s->all) {
        Request* r = kv.second.get();
        free_events(r);
        if (r->mesh) sl_destroy_mesh(r->mesh);
        r->mesh = nullptr;
    }
    for (auto& kv : s->groups) {
        if (kv.second.dargs) (void)hipFree(kv.second.dargs);
        if (kv.second.stream) (void)hipStreamDestroy(kv.second.stream);
    }
    for (Tick& t : s->ticks) {
        if (t.start) (void)hipEventDestroy(t.start);
        if (t.end) (void)hipEventDestroy(t.end);
    }
    if (s->stage) {
        for (int k = 0; k < kStages; ++k) (void)hipEventDestroy(s->stage_ev[k]);
        (void)hipHostFree(s->stage);
    }
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    if (s->arena.base) (void)hipFree(s->arena.base);
    delete s;
    return SL_OK;
}

}  // extern "C"
