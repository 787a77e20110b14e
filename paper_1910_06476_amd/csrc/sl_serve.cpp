// Request loop behind the C ABI of include/sl.h (sl_server_*): continuous
// batching of independent transport problems on one GPU.
//
// A request is one whole problem: mesh, velocity, optional ghost rows, dt,
// step count and options.  Requests wait in arrival order and are admitted
// while a slot is free and the device memory they need fits the budget.
// An admitted request gets its own mesh (and set-up stream).
//
// Batched requests: admitted requests whose steps share a kernel variant
// (dimension, nodes per direction, advect variant) form a group, and the
// server steps each group in ticks: one tick is one launch of each step
// kernel over the elements of all members with steps left, every block
// working for one member on that member's own buffers (the kernels' batched
// forms).  Members join at the next tick after admission and leave after
// their last one, so the membership changes continuously; a few ticks per
// group are queued ahead on the server's stream.  A step's launch arguments
// travel to the device through a ring of pinned host slots.
//
// Other requests (steps that cannot join a batch, or a server created with
// SL_SERVER_NO_BATCH) queue all their steps at admission on their own
// stream, with an event after each, so they overlap with everything else.
//
// sl_server_progress retires finished requests (copies the field to host
// memory, frees the mesh and the memory it held), admits waiting ones and
// queues ticks, in the same call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <tuple>
#include <vector>

#include "sl_internal.h"

namespace {

enum { REQ_WAITING = 0, REQ_ACTIVE = 1, REQ_DONE = 2 };

constexpr int kAhead = 4;    // ticks a group may have queued and not finished
constexpr int kStages = 32;  // pinned argument slots

double now_us()
{
    using namespace std::chrono;
    return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

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
    sl_mesh* mesh = nullptr;
    std::vector<hipEvent_t> ev;  // unbatched: ev[0] before the first step, ev[k] after step k
    bool batched = false;
    int32_t launched = 0;        // batched: steps queued so far
    std::vector<int> ticks;      // batched: the ticks that carried its steps
    std::vector<double> result;
    sl_stats stats{};
    sl_status status = SL_OK;
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;  // host clock, microseconds
    double device_ms = 0.0;                              // before the first to after the last step
    int64_t admit_seq = -1;
};

// one batched step of a group: events around its two launches, and how many
// members still have to read them
struct Tick {
    hipEvent_t start = nullptr, end = nullptr;
    int refs = 0;
};

using GroupKey = std::tuple<int, int, int>;  // dim, n, advect variant

struct Group {
    std::vector<Request*> members;  // in admission order
    char* dargs = nullptr;          // device: member arguments, then advect and constrain block offsets
    std::deque<int> queued;         // ticks queued and not yet seen finished
};

}  // namespace

struct sl_server {
    int32_t max_active = 1;
    bool batch = true;
    size_t budget = 0, used = 0;
    int64_t next_id = 1;
    int64_t admitted = 0;
    std::deque<Request*> waiting;
    std::vector<Request*> active;
    std::map<int64_t, std::unique_ptr<Request>> all;
    std::vector<float> step_ms;  // per-step device latencies of retired requests
    int64_t dof_updates = 0;     // of retired requests
    // batched work
    hipStream_t stream = nullptr;
    std::map<GroupKey, Group> groups;
    std::vector<Tick> ticks;
    std::vector<int> free_ticks;
    size_t slot_bytes = 0;
    char* stage = nullptr;  // pinned, kStages slots
    hipEvent_t stage_ev[kStages] = {};
    bool stage_used[kStages] = {};
    int stage_next = 0;
    int64_t batch_launches = 0, batch_member_steps = 0;
};

namespace {

size_t args_bytes() { return std::max(sizeof(sl::Step1DArgs), sizeof(sl::Step2DArgs)); }

void free_events(Request* r)
{
    for (hipEvent_t e : r->ev) (void)hipEventDestroy(e);
    r->ev.clear();
}

void release_tick(sl_server* s, int k)
{
    Tick& t = s->ticks[(size_t)k];
    if (--t.refs > 0) return;
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.end);
    t = Tick{};
    s->free_ticks.push_back(k);
}

int new_tick(sl_server* s)
{
    int k;
    if (!s->free_ticks.empty()) {
        k = s->free_ticks.back();
        s->free_ticks.pop_back();
    } else {
        k = (int)s->ticks.size();
        s->ticks.emplace_back();
    }
    Tick& t = s->ticks[(size_t)k];
    if (hipEventCreate(&t.start) != hipSuccess || hipEventCreate(&t.end) != hipSuccess) {
        if (t.start) (void)hipEventDestroy(t.start);
        t = Tick{};
        s->free_ticks.push_back(k);
        return -1;
    }
    return k;
}

// set-up of one request: mesh, velocity, ghost rows on the mesh's stream
sl_status setup(Request* r, void** stream)
{
    sl_mesh_desc d = r->desc;
    d.u0 = r->u0.data();
    d.stream = nullptr;  // the mesh creates its own stream
    sl_status rc = sl_create_mesh(&d, &r->mesh);
    if (rc == SL_OK) rc = sl_set_velocity(r->mesh, r->a.data(), r->div.empty() ? nullptr : r->div.data());
    if (rc == SL_OK && r->ghost_rows > 0) rc = sl_set_ghost(r->mesh, r->ghost.data(), r->ghost_rows);
    double* dphi = nullptr;
    if (rc == SL_OK) rc = sl_device_field(r->mesh, &dphi, stream);
    return rc;
}

// unbatched: every step queued at once on the request's stream
sl_status launch_all(Request* r, hipStream_t stream)
{
    sl_status rc = SL_OK;
    r->ev.resize((size_t)r->nsteps + 1, nullptr);
    for (auto& e : r->ev)
        if (hipEventCreate(&e) != hipSuccess) rc = SL_E_DEVICE;
    if (rc == SL_OK && hipEventRecord(r->ev[0], stream) != hipSuccess) rc = SL_E_DEVICE;
    for (int32_t k = 1; rc == SL_OK && k <= r->nsteps; ++k) {
        rc = sl_step(r->mesh, r->dt, 1, &r->opts);
        if (rc == SL_OK && hipEventRecord(r->ev[k], stream) != hipSuccess) rc = SL_E_DEVICE;
    }
    return rc;
}

// stream, pinned argument slots and their events of the batched work
sl_status batch_resources(sl_server* s)
{
    if (s->stream) return SL_OK;
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return SL_E_DEVICE;
    if (hipHostMalloc((void**)&s->stage, s->slot_bytes * kStages, hipHostMallocDefault) != hipSuccess) {
        s->stage = nullptr;
        (void)hipStreamDestroy(st);
        return SL_E_NOMEM;
    }
    for (int k = 0; k < kStages; ++k)
        if (hipEventCreateWithFlags(&s->stage_ev[k], hipEventDisableTiming) != hipSuccess) {
            for (int j = 0; j < k; ++j) (void)hipEventDestroy(s->stage_ev[j]);
            (void)hipHostFree(s->stage);
            s->stage = nullptr;
            (void)hipStreamDestroy(st);
            return SL_E_DEVICE;
        }
    s->stream = st;
    return SL_OK;
}

// admit one request: set-up, then either every step on its own stream or a
// place in its group (the server's stream first waits for the set-up)
sl_status admit(sl_server* s, Request* r)
{
    void* stream = nullptr;
    sl_status rc = setup(r, &stream);
    sl::StepLaunch L;
    if (rc == SL_OK) rc = sl::step_prepare(r->mesh, r->dt, r->opts, &L);  // validates the options
    bool batched = false;
    if (rc == SL_OK && s->batch && r->nsteps > 0 && L.variant >= 0) rc = batch_resources(s);
    if (rc == SL_OK && s->batch && r->nsteps > 0 && L.variant >= 0) {
        hipEvent_t ready = nullptr;
        if (hipEventCreate(&ready) != hipSuccess || hipEventRecord(ready, (hipStream_t)stream) != hipSuccess ||
            hipStreamWaitEvent(s->stream, ready, 0) != hipSuccess)
            rc = SL_E_DEVICE;
        if (ready) (void)hipEventDestroy(ready);
        if (rc == SL_OK) {
            Group& g = s->groups[GroupKey(L.dim, L.n, L.variant)];
            if (!g.dargs) {
                const size_t need = s->slot_bytes;
                if (hipMalloc((void**)&g.dargs, need) != hipSuccess) {
                    g.dargs = nullptr;
                    rc = SL_E_NOMEM;
                }
            }
            if (rc == SL_OK) {
                g.members.push_back(r);
                batched = true;
            }
        }
    } else if (rc == SL_OK) {
        rc = launch_all(r, (hipStream_t)stream);
    }
    if (rc != SL_OK) {
        free_events(r);
        if (r->mesh) sl_destroy_mesh(r->mesh);
        r->mesh = nullptr;
        return rc;
    }
    r->batched = batched;
    r->state = REQ_ACTIVE;
    r->t_admit = now_us();
    r->admit_seq = s->admitted++;
    s->used += r->bytes;
    s->active.push_back(r);
    return SL_OK;
}

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
    int slot = 0;
    char* host = take_slot(s, &slot);
    if (!host) return SL_E_DEVICE;
    const size_t ab = args_bytes();
    int* adv_start = (int*)(host + ab * (size_t)s->max_active);
    int* con_start = adv_start + s->max_active + 1;
    sl::StepLaunch L0;
    adv_start[0] = con_start[0] = 0;
    for (int k = 0; k < nreq; ++k) {
        sl::StepLaunch L;
        const sl_status rc = sl::step_prepare(mem[(size_t)k]->mesh, mem[(size_t)k]->dt, mem[(size_t)k]->opts, &L);
        if (rc != SL_OK) return rc;
        if (k == 0) L0 = L;
        // packed at the arguments' own size: the kernels index As[r]
        if (L.dim == 1)
            std::memcpy(host + sizeof(L.a1) * (size_t)k, &L.a1, sizeof(L.a1));
        else
            std::memcpy(host + sizeof(L.a2) * (size_t)k, &L.a2, sizeof(L.a2));
        adv_start[k + 1] = adv_start[k] + L.adv_blocks;
        con_start[k + 1] = con_start[k] + L.con_blocks;
    }
    // the offsets follow room for max_active arguments of the larger kind
    if (hipMemcpyAsync(g.dargs, host, s->slot_bytes, hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipEventRecord(s->stage_ev[slot], s->stream) != hipSuccess)
        return SL_E_DEVICE;
    s->stage_used[slot] = true;
    const int t = new_tick(s);
    if (t < 0) return SL_E_DEVICE;
    Tick& tk = s->ticks[(size_t)t];
    const int* dadv = (const int*)(g.dargs + ab * (size_t)s->max_active);
    const int* dcon = dadv + s->max_active + 1;
    const int dim = std::get<0>(key), n = std::get<1>(key);
    int bad = hipEventRecord(tk.start, s->stream) != hipSuccess;
    if (dim == 1) {
        const auto* dA = (const sl::Step1DArgs*)g.dargs;
        bad |= sl::launch_advect1d_batch(n, L0.a1, dA, dadv, nreq, adv_start[nreq], s->stream);
        bad |= sl::launch_constrain1d_batch(n, dA, dcon, nreq, con_start[nreq], s->stream);
    } else {
        const auto* dA = (const sl::Step2DArgs*)g.dargs;
        bad |= sl::launch_advect2d_batch(n, L0.a2, dA, dadv, nreq, adv_start[nreq], s->stream);
        bad |= sl::launch_constrain2d_batch(n, dA, dcon, nreq, con_start[nreq], s->stream);
    }
    bad |= hipEventRecord(tk.end, s->stream) != hipSuccess;
    tk.refs = nreq + 1;  // the members and the group's queue
    for (Request* r : mem) {
        sl::step_commit(r->mesh, r->dt);
        r->launched += 1;
        r->ticks.push_back(t);
    }
    g.queued.push_back(t);
    s->batch_launches += 1;
    s->batch_member_steps += nreq;
    *queued = true;
    return bad ? SL_E_DEVICE : SL_OK;
}

// keep up to kAhead ticks of every group queued
sl_status queue_ticks(sl_server* s)
{
    for (auto& kv : s->groups) {
        Group& g = kv.second;
        while (!g.queued.empty()) {  // forget finished ticks
            const hipError_t q = hipEventQuery(s->ticks[(size_t)g.queued.front()].end);
            if (q == hipErrorNotReady) break;
            if (q != hipSuccess) return SL_E_DEVICE;
            release_tick(s, g.queued.front());
            g.queued.pop_front();
        }
        while ((int)g.queued.size() < kAhead) {
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

// a finished request: field and statistics to host, latencies, free the mesh
void retire(sl_server* s, Request* r)
{
    const size_t nd = r->desc.dim == 1 ? (size_t)(r->desc.order + 1) : (size_t)(r->desc.order + 1) * (r->desc.order + 1);
    const size_t nf = (size_t)r->desc.kx * r->desc.ky * nd;
    r->result.resize(nf);
    if (r->batched) {
        // the server's stream may hold later ticks of others: read without
        // waiting on it (this request's last tick has finished)
        r->status = sl::read_settled(r->mesh, r->result.data(), &r->stats);
        for (int k : r->ticks) {
            const Tick& t = s->ticks[(size_t)k];
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, t.start, t.end) == hipSuccess) s->step_ms.push_back(ms);
        }
        float tot = 0.0f;
        if (!r->ticks.empty() && hipEventElapsedTime(&tot, s->ticks[(size_t)r->ticks.front()].start,
                                                     s->ticks[(size_t)r->ticks.back()].end) == hipSuccess)
            r->device_ms = tot;
        for (int k : r->ticks) release_tick(s, k);
        r->ticks.clear();
        for (auto& kv : s->groups) {
            auto& m = kv.second.members;
            m.erase(std::remove(m.begin(), m.end(), r), m.end());
        }
    } else {
        r->status = sl_read(r->mesh, r->result.data(), &r->stats);
        for (size_t k = 1; k < r->ev.size(); ++k) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, r->ev[k - 1], r->ev[k]) == hipSuccess) s->step_ms.push_back(ms);
        }
        float tot = 0.0f;
        if (r->ev.size() > 1 && hipEventElapsedTime(&tot, r->ev.front(), r->ev.back()) == hipSuccess) r->device_ms = tot;
        free_events(r);
    }
    sl_destroy_mesh(r->mesh);
    r->mesh = nullptr;
    s->used -= r->bytes;
    s->dof_updates += (int64_t)nf * r->nsteps;
    r->t_done = now_us();
    r->state = REQ_DONE;
}

}  // namespace

extern "C" {

sl_status sl_server_create(const sl_server_desc* d, sl_server** out)
{
    const sl::ApiHold hold;
    if (!out) return SL_E_INVALID;
    *out = nullptr;
    if (!d || d->max_active < 1 || d->max_active > 64 || d->hbm_budget == 0) return SL_E_INVALID;
    if (d->flags & ~SL_SERVER_NO_BATCH) return SL_E_INVALID;
    std::unique_ptr<sl_server> s(new (std::nothrow) sl_server());
    if (!s) return SL_E_NOMEM;
    s->max_active = d->max_active;
    s->budget = d->hbm_budget;
    s->batch = (d->flags & SL_SERVER_NO_BATCH) == 0;
    s->slot_bytes =
        (args_bytes() * (size_t)s->max_active + 2 * sizeof(int) * (size_t)(s->max_active + 1) + 255) / 256 * 256;
    *out = s.release();  // host only: the batching resources come with the first batched request
    return SL_OK;
}

sl_status sl_server_submit(sl_server* s, const sl_request* q, int64_t* id)
{
    const sl::ApiHold hold;
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
    r->id = s->next_id++;
    r->t_submit = now_us();
    s->waiting.push_back(r.get());
    *id = r->id;
    s->all[r->id] = std::move(r);
    return SL_OK;
}

sl_status sl_server_progress(sl_server* s, int32_t* active, int32_t* waiting)
{
    const sl::ApiHold hold;
    if (!s) return SL_E_INVALID;
    // retire finished requests (in admission order among those done)
    for (size_t i = 0; i < s->active.size();) {
        Request* r = s->active[i];
        const hipEvent_t last = last_event(s, r);
        const hipError_t q = (r->batched && r->nsteps == 0) ? hipSuccess
                             : last                          ? hipEventQuery(last)
                                                             : hipErrorNotReady;
        if (q == hipSuccess) {
            retire(s, r);
            s->active.erase(s->active.begin() + (long)i);
        } else if (q == hipErrorNotReady) {
            ++i;
        } else {
            return SL_E_DEVICE;
        }
    }
    // admit in arrival order while a slot and the memory budget allow
    while (!s->waiting.empty() && (int32_t)s->active.size() < s->max_active &&
           s->used + s->waiting.front()->bytes <= s->budget) {
        Request* r = s->waiting.front();
        s->waiting.pop_front();
        const sl_status rc = admit(s, r);
        if (rc != SL_OK) {  // the request fails alone; the loop goes on
            r->status = rc;
            r->state = REQ_DONE;
            r->t_done = now_us();
        }
    }
    // the next ticks of every group, the newly admitted members included
    if (s->stream) {
        const sl_status rc = queue_ticks(s);
        if (rc != SL_OK) return rc;
    }
    if (active) *active = (int32_t)s->active.size();
    if (waiting) *waiting = (int32_t)s->waiting.size();
    return SL_OK;
}

sl_status sl_server_drain(sl_server* s)
{
    const sl::ApiHold hold;
    if (!s) return SL_E_INVALID;
    int32_t a = 1, w = 1;
    while (a > 0 || w > 0) {
        const sl_status rc = sl_server_progress(s, &a, &w);
        if (rc != SL_OK) return rc;
        if (a > 0) {
            // wait for the oldest active request's last step, or, while its
            // steps are still being queued, for its group's oldest tick
            const Request* r = s->active.front();
            hipEvent_t e = last_event(s, r);
            if (!e && r->batched)
                for (const auto& kv : s->groups)
                    if (!kv.second.queued.empty() &&
                        std::find(kv.second.members.begin(), kv.second.members.end(), r) != kv.second.members.end())
                        e = s->ticks[(size_t)kv.second.queued.front()].end;
            if (e && hipEventSynchronize(e) != hipSuccess) return SL_E_DEVICE;
        }
    }
    return SL_OK;
}

sl_status sl_server_result(sl_server* s, int64_t id, double* u_out, sl_stats* st, sl_request_timing* tm)
{
    const sl::ApiHold hold;
    if (!s) return SL_E_INVALID;
    auto it = s->all.find(id);
    if (it == s->all.end()) return SL_E_INVALID;
    Request* r = it->second.get();
    if (r->state != REQ_DONE) return SL_E_STATE;
    if (u_out && !r->result.empty()) std::memcpy(u_out, r->result.data(), r->result.size() * sizeof(double));
    if (st) *st = r->stats;
    if (tm) {
        tm->queue_us = r->t_admit > 0 ? r->t_admit - r->t_submit : 0.0;
        tm->total_us = r->t_done - r->t_submit;
        tm->device_ms = r->device_ms;
        tm->bytes = r->bytes;
        tm->admit_seq = r->admit_seq;
    }
    const sl_status rc = r->status;
    s->all.erase(it);
    return rc;
}

sl_status sl_server_latency(sl_server* s, double p50_p99[2], int64_t* samples, int64_t* dof_updates)
{
    const sl::ApiHold hold;
    if (!s || !p50_p99) return SL_E_INVALID;
    std::vector<float> v = s->step_ms;
    p50_p99[0] = p50_p99[1] = 0.0;
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        p50_p99[0] = v[std::min(v.size() - 1, (size_t)(0.50 * (double)v.size()))];
        p50_p99[1] = v[std::min(v.size() - 1, (size_t)(0.99 * (double)v.size()))];
    }
    if (samples) *samples = (int64_t)v.size();
    if (dof_updates) *dof_updates = s->dof_updates;
    return SL_OK;
}

sl_status sl_server_batching(sl_server* s, int64_t* launches, int64_t* member_steps)
{
    const sl::ApiHold hold;
    if (!s) return SL_E_INVALID;
    if (launches) *launches = s->batch_launches;
    if (member_steps) *member_steps = s->batch_member_steps;
    return SL_OK;
}

sl_status sl_server_destroy(sl_server* s)
{
    const sl::ApiHold hold;
    if (!s) return SL_E_INVALID;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (Request* r : s->active) {
        if (!r->batched && r->ev.size()) (void)hipEventSynchronize(r->ev.back());
        free_events(r);
        if (r->mesh) sl_destroy_mesh(r->mesh);
        r->mesh = nullptr;
    }
    for (auto& kv : s->groups)
        if (kv.second.dargs) (void)hipFree(kv.second.dargs);
    for (Tick& t : s->ticks) {
        if (t.start) (void)hipEventDestroy(t.start);
        if (t.end) (void)hipEventDestroy(t.end);
    }
    if (s->stage) {
        for (int k = 0; k < kStages; ++k) (void)hipEventDestroy(s->stage_ev[k]);
        (void)hipHostFree(s->stage);
    }
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return SL_OK;
}

}  // extern "C"
