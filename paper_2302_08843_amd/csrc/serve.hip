// serve.hip -- the request server of include/mm.h (mm_serve_*): continuous
// batching of relaxations and time integrations of different grids on one GPU.
//
// Every admitted request owns a plan (spectra, Runge-Kutta vectors, device
// step controller; in FP32 the Runge-Kutta state itself in double) and a
// stream slot.  Its Dormand-Prince steps are decided on
// the device, so a fixed sequence of steps is captured once into a HIP graph
// and replayed until the controller reports completion; each launch is
// followed by an 80-byte copy of the controller state to pinned host memory
// and an event, and two launches are kept in flight per request.  The host
// never waits for a step: mm_serve_poll only queries events.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <limits>
#include <list>
#include <map>
#include <tuple>
#include <vector>

#include "engine.h"

namespace mmx {
namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Plans of one class share the spectral kernel: same grid, precision,
// near-field order and cell proportions.
struct ClassKey {
    int g0, g1, g2, prec, p;
    double ry, rz;
    bool operator<(const ClassKey& o) const
    {
        return std::tie(g0, g1, g2, prec, p, ry, rz) <
               std::tie(o.g0, o.g1, o.g2, o.prec, o.p, o.ry, o.rz);
    }
    bool operator==(const ClassKey& o) const { return !(*this < o) && !(o < *this); }
};

struct Req {
    mm_request r;
    double t_submit = 0.0;
    bool waited_mem = false, waited_slot = false;
    hipEvent_t ready = nullptr;  // recorded on the caller's stream at submission
};

struct Active {
    Req q;
    ClassKey key;
    Plan* plan = nullptr;
    size_t plan_bytes = 0;
    int slot = -1;
    hipGraphExec_t exec = nullptr;
    double t_admit = 0.0;
    bool finishing = false;
    int head = 0, inflight = 0;  // ring of two launches
    DevCtl last{};
};

struct Idle {
    ClassKey key;
    Plan* plan;
    size_t bytes;
};

}  // namespace

struct Server {
    mm_serve_opts o{};
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;  // 3 per slot: two launches, the result copy
    DevCtl* pinned = nullptr;        // 2 per slot
    std::vector<int> free_slots;
    std::deque<Req> queue;
    std::vector<Active*> active;
    std::map<ClassKey, SharedTensor*> tensors;
    std::list<Idle> idle;  // least recently used first
    std::deque<mm_completion> done;
    size_t bytes = 0;
    mm_serve_stats st{};
};

namespace {

ClassKey class_of(const mm_request& r, const mm_serve_opts& o)
{
    return ClassKey{r.grid[0], r.grid[1], r.grid[2], (int)o.prec, o.demag_p,
                    r.cell[1] / r.cell[0], r.cell[2] / r.cell[0]};
}

size_t tensor_bytes(const mm_request& r, int prec)
{
    return plan_footprint(r.grid, prec, true) - plan_footprint(r.grid, prec, false);
}

void finish(Server* s, const Req& q, int status, const DevCtl* c, double t_admit)
{
    if (q.ready) (void)hipEventDestroy(q.ready);
    mm_completion m{};
    m.tag = q.r.tag;
    m.status = status;
    if (c) {
        m.accepted = c->accepted;
        m.rejected = c->rejected;
        m.rhs_evals = c->rhs_evals;
        m.t = c->t;
        m.torque = c->torque;
    }
    m.t_submit = q.t_submit;
    m.t_admit = t_admit;
    m.t_done = now_s();
    s->done.push_back(m);
    s->st.completed++;
}

// Drop an idle plan (least recently used first), or a resident spectral
// kernel that no plan uses; false when nothing can be released.
bool release_one(Server* s, const ClassKey* keep)
{
    for (auto it = s->idle.begin(); it != s->idle.end(); ++it) {
        s->bytes -= it->bytes;
        free_plan(it->plan);
        s->idle.erase(it);
        return true;
    }
    for (auto it = s->tensors.begin(); it != s->tensors.end(); ++it) {
        if (it->second->refs == 1 && !(keep && it->first == *keep)) {
            s->bytes -= it->second->bytes;
            release_tensor(it->second);
            s->tensors.erase(it);
            return true;
        }
    }
    return false;
}

void retire_plan(Server* s, Active* a, bool keep)
{
    if (a->exec) (void)hipGraphExecDestroy(a->exec);
    a->exec = nullptr;
    if (keep) {
        s->idle.push_back(Idle{a->key, a->plan, a->plan_bytes});
    } else {
        s->bytes -= a->plan_bytes;
        free_plan(a->plan);
    }
    a->plan = nullptr;
    s->free_slots.push_back(a->slot);
}

template <typename T>
mm_status capture(Server* s, Active* a)
{
    const mm_request& r = a->q.r;
    hipStream_t stream = s->streams[a->slot];
    const bool relax = r.kind == MM_SERVE_RELAX;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    mm_status st = MM_OK;
    for (int i = 0; i < s->o.steps_per_launch && st == MM_OK; ++i)
        st = dev_step<T>(a->plan, r.h_ext, r.terms, r.rtol, r.atol, relax, relax);
    e = hipStreamEndCapture(stream, &g);
    if (st != MM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    e = hipGraphInstantiate(&a->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "graph instantiation");
    return MM_OK;
}

mm_status launch(Server* s, Active* a)
{
    hipStream_t stream = s->streams[a->slot];
    const int idx = (a->head + a->inflight) & 1;
    hipError_t e = hipGraphLaunch(a->exec, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&s->pinned[2 * a->slot + idx], a->plan->ctl, sizeof(DevCtl),
                           hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipEventRecord(s->events[3 * a->slot + idx], stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    a->inflight++;
    s->st.graph_launches++;
    return MM_OK;
}

// Admit the head of the queue if a slot and memory allow.  Returns true if
// the queue may be looked at again.
bool try_admit(Server* s)
{
    if (s->queue.empty()) return false;
    Req& head = s->queue.front();
    if (s->free_slots.empty()) {
        if (!head.waited_slot) s->st.waited_slot++;
        head.waited_slot = true;
        return false;
    }
    const ClassKey key = class_of(head.r, s->o);
    // an idle plan of the same class needs no new memory
    auto reuse = s->idle.end();
    for (auto it = s->idle.begin(); it != s->idle.end(); ++it)
        if (it->key == key) reuse = it;
    if (reuse == s->idle.end()) {
        size_t need = plan_footprint(head.r.grid, s->o.prec, false) +
                      (s->o.prec == MM_FP32 ? state64_bytes(head.r.grid) : 0);
        if (!s->tensors.count(key)) need += tensor_bytes(head.r, s->o.prec);
        while (s->bytes + need > s->o.hbm_budget && release_one(s, &key)) {
        }
        if (s->bytes + need > s->o.hbm_budget) {
            if (s->active.empty()) {
                const Req dead = head;
                s->queue.pop_front();
                set_error("request larger than the server's memory budget");
                finish(s, dead, MM_ENOMEM, nullptr, 0.0);
                return true;
            }
            if (!head.waited_mem) s->st.waited_memory++;
            head.waited_mem = true;
            return false;
        }
    }
    Active* a = new Active();
    a->q = head;
    s->queue.pop_front();  // `head` is gone from here on
    const mm_request& r = a->q.r;
    a->key = key;
    a->slot = s->free_slots.back();
    s->free_slots.pop_back();
    a->t_admit = now_s();
    hipStream_t stream = s->streams[a->slot];
    mm_status st = MM_OK;
    const double nrm = std::sqrt(r.ku_axis[0] * r.ku_axis[0] + r.ku_axis[1] * r.ku_axis[1] +
                                 r.ku_axis[2] * r.ku_axis[2]);
    if (reuse != s->idle.end()) {
        a->plan = reuse->plan;
        a->plan_bytes = reuse->bytes;
        s->idle.erase(reuse);
        Plan* p = a->plan;
        for (int d = 0; d < 3; ++d) {
            p->d[d] = r.cell[d];
            p->eu[d] = r.ku_axis[d] / nrm;
        }
        p->Ms = r.Ms;
        p->A = r.A;
        p->Ku = r.Ku;
        p->alpha = r.alpha;
        p->n_magnetic = r.Ms > 0.0 ? p->N : 0;
        p->stream = stream;
        s->st.plans_reused++;
    } else {
        mm_opts po;
        mm_opts_default(&po);
        po.prec = s->o.prec;
        po.demag_p = s->o.demag_p;
        for (int d = 0; d < 3; ++d) po.ku_axis[d] = r.ku_axis[d];
        po.stream = stream;
        auto ti = s->tensors.find(key);
        SharedTensor* share = ti == s->tensors.end() ? nullptr : ti->second;
        // The class kernel is built at a canonical cell of the class's shape
        // (x edge 1 nm), so it does not depend on which request came first.
        const double canon[3] = {1e-9, 1e-9 * key.ry, 1e-9 * key.rz};
        st = plan_build(r.grid, share ? r.cell : canon, r.Ms, r.A, r.Ku, r.alpha, po, share,
                        &a->plan);
        if (st == MM_OK)
            for (int d = 0; d < 3; ++d) a->plan->d[d] = r.cell[d];
        if (st == MM_OK && !share) {
            SharedTensor* t = new SharedTensor();
            t->Khat = a->plan->Khat;
            t->tw = a->plan->tw;
            t->bytes = tensor_bytes(r, s->o.prec);
            t->refs = 2;  // the server's and the plan's
            a->plan->shared = t;
            s->tensors[key] = t;
            s->bytes += t->bytes;
            s->st.tensors_built++;
        }
        if (st == MM_OK) {
            a->plan_bytes = plan_footprint(r.grid, s->o.prec, false) +
                            (s->o.prec == MM_FP32 ? state64_bytes(r.grid) : 0);
            a->plan->state64 = s->o.prec == MM_FP32;
            s->bytes += a->plan_bytes;
            s->st.plans_created++;
        }
    }
    if (st == MM_OK && a->q.ready) {
        hipError_t e = hipStreamWaitEvent(stream, a->q.ready, 0);
        if (e != hipSuccess) st = hip_fail(e, "waiting for the start state");
    }
    if (st == MM_OK) {
        DevCtl c{};
        const bool relax = r.kind == MM_SERVE_RELAX;
        c.t = 0.0;
        c.dt = -1.0;
        c.t_end = relax ? std::numeric_limits<double>::infinity() : r.t_end;
        c.dt_min = 1e-20;
        c.torque_tol = relax ? r.tol : 0.0;
        c.max_steps = r.max_steps;
        c.relax = relax ? 1 : 0;
        c.renorm = relax ? 1 : 0;
        st = s->o.prec == MM_FP32
                 ? dev_prepare<float>(a->plan, r.m, r.h_ext, r.terms, c, r.rtol, r.atol)
                 : dev_prepare<double>(a->plan, r.m, r.h_ext, r.terms, c, r.rtol, r.atol);
    }
    if (st == MM_OK) st = s->o.prec == MM_FP32 ? capture<float>(s, a) : capture<double>(s, a);
    if (st == MM_OK) st = launch(s, a);
    if (st == MM_OK) st = launch(s, a);
    if (st != MM_OK) {
        finish(s, a->q, st, nullptr, a->t_admit);
        if (a->plan) {
            (void)hipStreamSynchronize(stream);
            retire_plan(s, a, false);
        } else {
            s->free_slots.push_back(a->slot);
        }
        delete a;
        return true;
    }
    s->active.push_back(a);
    s->st.admitted++;
    s->st.bytes_peak = std::max(s->st.bytes_peak, s->bytes);
    return true;
}

// Advance one active request; true when it has completed.
bool progress(Server* s, Active* a)
{
    const int sl = a->slot;
    hipStream_t stream = s->streams[sl];
    if (a->finishing) {
        hipError_t e = hipEventQuery(s->events[3 * sl + 2]);
        if (e == hipErrorNotReady) return false;
        if (e != hipSuccess) {
            finish(s, a->q, hip_fail(e, "request result"), &a->last, a->t_admit);
            retire_plan(s, a, false);
            return true;
        }
        finish(s, a->q, a->last.result, &a->last, a->t_admit);
        retire_plan(s, a, true);
        return true;
    }
    while (a->inflight > 0) {
        const int idx = a->head;
        hipError_t e = hipEventQuery(s->events[3 * sl + idx]);
        if (e == hipErrorNotReady) return false;
        if (e != hipSuccess) {
            finish(s, a->q, hip_fail(e, "graph launch"), &a->last, a->t_admit);
            (void)hipStreamSynchronize(stream);
            retire_plan(s, a, false);
            return true;
        }
        a->last = s->pinned[2 * sl + idx];
        a->inflight--;
        a->head ^= 1;
        if (a->last.done) {
            // any launch still in flight is a no-op; the copy follows it
            hipError_t e2 = dev_result(a->plan, a->q.r.m);
            if (e2 == hipSuccess) e2 = hipEventRecord(s->events[3 * sl + 2], stream);
            if (e2 != hipSuccess) {
                finish(s, a->q, hip_fail(e2, "request result"), &a->last, a->t_admit);
                (void)hipStreamSynchronize(stream);
                retire_plan(s, a, false);
                return true;
            }
            a->finishing = true;
            return false;
        }
        mm_status st = launch(s, a);
        if (st != MM_OK) {
            finish(s, a->q, st, &a->last, a->t_admit);
            (void)hipStreamSynchronize(stream);
            retire_plan(s, a, false);
            return true;
        }
    }
    return false;
}

bool valid_request(const mm_request& r)
{
    for (int d = 0; d < 3; ++d) {
        if (r.grid[d] < 1 || r.grid[d] > 512) return false;
        if (!(r.cell[d] > 0.0) || !std::isfinite(r.cell[d])) return false;
        if (!std::isfinite(r.h_ext[d]) || !std::isfinite(r.ku_axis[d])) return false;
    }
    const double nrm = std::sqrt(r.ku_axis[0] * r.ku_axis[0] + r.ku_axis[1] * r.ku_axis[1] +
                                 r.ku_axis[2] * r.ku_axis[2]);
    if (!(nrm > 0.0)) return false;
    if (!(r.Ms >= 0.0) || !(r.A >= 0.0) || !(r.alpha >= 0.0) || !std::isfinite(r.Ms) ||
        !std::isfinite(r.A) || !std::isfinite(r.Ku) || !std::isfinite(r.alpha))
        return false;
    if (r.kind != MM_SERVE_RELAX && r.kind != MM_SERVE_INTEGRATE) return false;
    if (!(r.rtol > 0.0) || !(r.atol > 0.0) || r.max_steps < 0 || !r.m) return false;
    if (r.kind == MM_SERVE_RELAX && !(r.tol > 0.0)) return false;
    if (r.kind == MM_SERVE_INTEGRATE && !(r.t_end >= 0.0)) return false;
    return true;
}

}  // namespace
}  // namespace mmx

using namespace mmx;

extern "C" {

void mm_serve_opts_default(mm_serve_opts* o)
{
    if (!o) return;
    o->hbm_budget = 0;
    o->max_active = 16;
    o->steps_per_launch = 8;
    o->prec = MM_FP32;
    o->demag_p = 20;
}

double mm_serve_clock(void) { return now_s(); }

mm_status mm_serve_create(mm_server** out, const mm_serve_opts* opt)
{
    if (!out) {
        set_error("null argument");
        return MM_EINVAL;
    }
    *out = nullptr;
    mm_serve_opts o;
    mm_serve_opts_default(&o);
    if (opt) o = *opt;
    if (o.max_active < 1 || o.max_active > 64 || o.steps_per_launch < 1 ||
        o.steps_per_launch > 64 || (o.prec != MM_FP32 && o.prec != MM_FP64)) {
        set_error("max_active and steps_per_launch must lie in [1, 64], prec FP32 or FP64");
        return MM_EINVAL;
    }
    if (o.hbm_budget == 0) {
        size_t fr = 0, tot = 0;
        hipError_t e = hipMemGetInfo(&fr, &tot);
        if (e != hipSuccess) return hip_fail(e, "device memory query");
        o.hbm_budget = fr / 10 * 8;
    }
    Server* s = new Server();
    s->o = o;
    s->st.budget = o.hbm_budget;
    hipError_t e = hipHostMalloc((void**)&s->pinned, 2 * o.max_active * sizeof(DevCtl),
                                 hipHostMallocDefault);
    for (int i = 0; i < o.max_active && e == hipSuccess; ++i) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) s->streams.push_back(st);
        for (int k = 0; k < 3 && e == hipSuccess; ++k) {
            hipEvent_t ev = nullptr;
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) s->events.push_back(ev);
        }
        s->free_slots.push_back(o.max_active - 1 - i);
    }
    if (e != hipSuccess) {
        mm_status st = hip_fail(e, "server streams");
        mm_serve_destroy(reinterpret_cast<mm_server*>(s));
        return st;
    }
    *out = reinterpret_cast<mm_server*>(s);
    return MM_OK;
}

mm_status mm_serve_submit(mm_server* sv, const mm_request* r)
{
    Server* s = reinterpret_cast<Server*>(sv);
    if (!s || !r || !valid_request(*r)) {
        set_error("invalid request");
        return MM_EINVAL;
    }
    Req q;
    q.r = *r;
    q.t_submit = now_s();
    {
        hipError_t e = hipEventCreateWithFlags(&q.ready, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(q.ready, (hipStream_t)r->stream);
        if (e != hipSuccess) {
            if (q.ready) (void)hipEventDestroy(q.ready);
            return hip_fail(e, "recording the start state's stream");
        }
    }
    s->queue.push_back(q);
    s->st.submitted++;
    return MM_OK;
}

mm_status mm_serve_poll(mm_server* sv, mm_completion* out, int max_out, int* n_out)
{
    Server* s = reinterpret_cast<Server*>(sv);
    if (!s || max_out < 0 || (max_out > 0 && !out)) {
        set_error("invalid argument");
        return MM_EINVAL;
    }
    for (size_t i = 0; i < s->active.size();) {
        Active* a = s->active[i];
        if (progress(s, a)) {
            delete a;
            s->active.erase(s->active.begin() + i);
        } else {
            ++i;
        }
    }
    while (try_admit(s)) {
    }
    int n = 0;
    while (n < max_out && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    if (n_out) *n_out = n;
    return MM_OK;
}

mm_status mm_serve_get_stats(const mm_server* sv, mm_serve_stats* st)
{
    const Server* s = reinterpret_cast<const Server*>(sv);
    if (!s || !st) {
        set_error("null argument");
        return MM_EINVAL;
    }
    *st = s->st;
    st->queued = (long)s->queue.size();
    st->active = (long)s->active.size();
    st->bytes_in_use = s->bytes;
    return MM_OK;
}

void mm_serve_destroy(mm_server* sv)
{
    Server* s = reinterpret_cast<Server*>(sv);
    if (!s) return;
    for (Active* a : s->active) {
        (void)hipStreamSynchronize(s->streams[a->slot]);
        if (a->exec) (void)hipGraphExecDestroy(a->exec);
        if (a->q.ready) (void)hipEventDestroy(a->q.ready);
        free_plan(a->plan);
        delete a;
    }
    for (auto& q : s->queue)
        if (q.ready) (void)hipEventDestroy(q.ready);
    for (auto& i : s->idle) free_plan(i.plan);
    for (auto& t : s->tensors) release_tensor(t.second);
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    if (s->pinned) (void)hipHostFree(s->pinned);
    delete s;
}

}  // extern "C"
