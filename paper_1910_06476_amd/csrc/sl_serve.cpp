// Request loop behind the C ABI of include/sl.h (sl_server_*): continuous
// batching of independent transport problems on one GPU.
//
// A request is one whole problem: mesh, velocity, optional ghost rows, dt,
// step count and options.  Requests wait in arrival order and are admitted
// while a slot is free and the device memory they need fits the budget.
// An admitted request gets its own mesh on its own stream; all its steps are
// queued at once, with an event after each, so the steps of all admitted
// requests overlap on the device.  sl_server_progress retires finished
// requests (copies the field to host memory, frees the mesh and the memory
// it held) and admits waiting ones in the same call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <vector>

#include "sl_internal.h"

namespace {

enum { REQ_WAITING = 0, REQ_ACTIVE = 1, REQ_DONE = 2 };

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
    std::vector<hipEvent_t> ev;  // ev[0] before the first step, ev[k] after step k
    std::vector<double> result;
    sl_stats stats{};
    sl_status status = SL_OK;
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;  // host clock, microseconds
    double device_ms = 0.0;                              // ev[0] to ev[nsteps]
    int64_t admit_seq = -1;
};

}  // namespace

struct sl_server {
    int32_t max_active = 1;
    size_t budget = 0, used = 0;
    int64_t next_id = 1;
    int64_t admitted = 0;
    std::deque<Request*> waiting;
    std::vector<Request*> active;
    std::map<int64_t, std::unique_ptr<Request>> all;
    std::vector<float> step_ms;  // per-step device latencies of retired requests
    int64_t dof_updates = 0;     // of retired requests
};

namespace {

void free_events(Request* r)
{
    for (hipEvent_t e : r->ev) (void)hipEventDestroy(e);
    r->ev.clear();
}

// admit one request: mesh, velocity, ghost rows, then every step on its stream
sl_status launch(sl_server* s, Request* r)
{
    sl_mesh_desc d = r->desc;
    d.u0 = r->u0.data();
    d.stream = nullptr;  // the mesh creates its own stream
    sl_status rc = sl_create_mesh(&d, &r->mesh);
    if (rc == SL_OK) rc = sl_set_velocity(r->mesh, r->a.data(), r->div.empty() ? nullptr : r->div.data());
    if (rc == SL_OK && r->ghost_rows > 0) rc = sl_set_ghost(r->mesh, r->ghost.data(), r->ghost_rows);
    void* stream = nullptr;
    double* dphi = nullptr;
    if (rc == SL_OK) rc = sl_device_field(r->mesh, &dphi, &stream);
    if (rc == SL_OK) {
        r->ev.resize((size_t)r->nsteps + 1, nullptr);
        for (auto& e : r->ev)
            if (hipEventCreate(&e) != hipSuccess) rc = SL_E_DEVICE;
    }
    if (rc == SL_OK && hipEventRecord(r->ev[0], (hipStream_t)stream) != hipSuccess) rc = SL_E_DEVICE;
    for (int32_t k = 1; rc == SL_OK && k <= r->nsteps; ++k) {
        rc = sl_step(r->mesh, r->dt, 1, &r->opts);
        if (rc == SL_OK && hipEventRecord(r->ev[k], (hipStream_t)stream) != hipSuccess) rc = SL_E_DEVICE;
    }
    if (rc != SL_OK) {
        free_events(r);
        if (r->mesh) sl_destroy_mesh(r->mesh);
        r->mesh = nullptr;
        return rc;
    }
    r->state = REQ_ACTIVE;
    r->t_admit = now_us();
    r->admit_seq = s->admitted++;
    s->used += r->bytes;
    s->active.push_back(r);
    return SL_OK;
}

// a finished request: field and statistics to host, latencies, free the mesh
void retire(sl_server* s, Request* r)
{
    const size_t nd = r->desc.dim == 1 ? (size_t)(r->desc.order + 1) : (size_t)(r->desc.order + 1) * (r->desc.order + 1);
    const size_t nf = (size_t)r->desc.kx * r->desc.ky * nd;
    r->result.resize(nf);
    r->status = sl_read(r->mesh, r->result.data(), &r->stats);
    for (size_t k = 1; k < r->ev.size(); ++k) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r->ev[k - 1], r->ev[k]) == hipSuccess) s->step_ms.push_back(ms);
    }
    float tot = 0.0f;
    if (r->ev.size() > 1 && hipEventElapsedTime(&tot, r->ev.front(), r->ev.back()) == hipSuccess) r->device_ms = tot;
    free_events(r);
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
    sl_server* s = new (std::nothrow) sl_server();
    if (!s) return SL_E_NOMEM;
    s->max_active = d->max_active;
    s->budget = d->hbm_budget;
    *out = s;
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
        const hipError_t q = hipEventQuery(r->ev.back());
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
        const sl_status rc = launch(s, r);
        if (rc != SL_OK) {  // the request fails alone; the loop goes on
            r->status = rc;
            r->state = REQ_DONE;
            r->t_done = now_us();
        }
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
            // wait for the oldest active request rather than spin
            if (hipEventSynchronize(s->active.front()->ev.back()) != hipSuccess) return SL_E_DEVICE;
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

sl_status sl_server_destroy(sl_server* s)
{
    const sl::ApiHold hold;
    if (!s) return SL_E_INVALID;
    for (Request* r : s->active) {
        if (r->ev.size()) (void)hipEventSynchronize(r->ev.back());
        free_events(r);
        if (r->mesh) sl_destroy_mesh(r->mesh);
        r->mesh = nullptr;
    }
    delete s;
    return SL_OK;
}

}  // extern "C"
