// serve.hip -- the request server of include/mm.h (mm_serve_*): continuous
// batching of relaxations and time integrations of different grids on one GPU.
//
// Requests are grouped by grid class (grid, precision, near-field order, cell
// proportions), kind, terms and tolerances.  A group is one batch plan of B
// request slots: spectra, Runge-Kutta space (in FP32 the state itself in
// double), device step controllers and per-request constants for every slot,
// and the class's resident spectral kernel.  Every kernel of a step covers
// all B slots with the request index in its grid, so B requests share each
// launch.  The slots' Dormand-Prince steps are decided on the device, one
// controller per slot, so a fixed sequence of steps is captured once per
// group into HIP graphs covering its first 1, 2, 4, ... B slots, and each
// launch replays the smallest one that covers every stepping request (a new
// request takes the lowest free slot); each launch is followed by a copy of
// the B controller records to pinned host memory and an event, and two
// launches are kept in flight.  A slot whose request finished is refilled with the
// next request of the same group key -- its constants and start state are
// written between launches, in stream order -- so requests join and leave a
// running batch continuously; a slot without a request has a finished
// controller and its steps change nothing.  The host never waits for a step:
// mm_serve_poll only queries events (an admission synchronises on the
// group's stream once, for the new request's starting step).
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

// Requests that can share a group's launches: one class, and the same kind,
// terms and tolerances (those are compiled into the captured steps).
struct GroupKey {
    ClassKey c;
    int kind;
    unsigned terms;
    double rtol, atol;
    bool operator<(const GroupKey& o) const
    {
        return std::tie(c, kind, terms, rtol, atol) <
               std::tie(o.c, o.kind, o.terms, o.rtol, o.atol);
    }
    bool operator==(const GroupKey& o) const { return !(*this < o) && !(o < *this); }
};

struct Req {
    mm_request r;
    double t_submit = 0.0;
    bool waited_mem = false, waited_slot = false;
    hipEvent_t ready = nullptr;  // recorded on the caller's stream at submission
};

struct Slot {
    bool busy = false;       // holds a request
    bool finishing = false;  // its result copy is in flight
    Req q;
    double t_admit = 0.0;
    long first_seq = 0;  // the first launch whose controller copy describes q
    DevCtl last{};
};

// Graphs of a group's steps, one per number of leading slots covered.
struct Graphs {
    std::vector<int> sizes;  // ascending: 1, 2, 4, ..., B
    std::vector<hipGraphExec_t> execs;
    bool empty() const { return execs.empty(); }
    void clear()
    {
        for (hipGraphExec_t e : execs)
            if (e) (void)hipGraphExecDestroy(e);
        execs.clear();
        sizes.clear();
    }
};

struct Group {
    GroupKey key;
    Plan* plan = nullptr;
    size_t bytes = 0;
    int B = 1;    // slots
    int sl = -1;  // stream slot
    Graphs graphs;
    std::vector<Slot> slots;
    int head = 0, inflight = 0;  // ring of two launches
    long seq[2] = {0, 0};        // launch numbers of the ring entries
    long next_seq = 1;
};

struct Idle {
    GroupKey key;
    Plan* plan;
    Graphs graphs;  // kept for batch plans (request-independent)
    size_t bytes;
    int B;
};

}  // namespace

struct Server {
    mm_serve_opts o{};
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;  // per stream slot: 2 launches, then one result copy per slot
    DevCtl* pinned = nullptr;        // per stream slot: 2 x batch controller records
    std::vector<int> free_slots;
    std::deque<Req> queue;
    std::vector<Group*> groups;
    std::map<ClassKey, SharedTensor*> tensors;
    std::list<Idle> idle;  // least recently used first
    std::deque<mm_completion> done;
    size_t bytes = 0;
    mm_serve_stats st{};
};

namespace {

// Requests of a group hold at most this many cells together.
constexpr long kBatchCells = 1L << 17;

int ev_per_stream(const Server* s) { return 2 + s->o.batch; }
hipEvent_t launch_event(Server* s, int sl, int idx) { return s->events[sl * ev_per_stream(s) + idx]; }
hipEvent_t result_event(Server* s, int sl, int b)
{
    return s->events[sl * ev_per_stream(s) + 2 + b];
}
DevCtl* pinned_of(Server* s, int sl, int idx)
{
    return s->pinned + ((size_t)sl * 2 + idx) * s->o.batch;
}

ClassKey class_of(const mm_request& r, const mm_serve_opts& o)
{
    return ClassKey{r.grid[0], r.grid[1], r.grid[2], (int)o.prec, o.demag_p,
                    r.cell[1] / r.cell[0], r.cell[2] / r.cell[0]};
}

GroupKey group_of(const mm_request& r, const mm_serve_opts& o)
{
    return GroupKey{class_of(r, o), r.kind, r.terms, r.rtol, r.atol};
}

size_t tensor_bytes(const mm_request& r, int prec)
{
    return plan_footprint(r.grid, prec, true) - plan_footprint(r.grid, prec, false);
}

// Slots of a group for requests of this grid: up to o.batch, at most
// kBatchCells cells together and within the memory budget; 1 where the
// batched kernels do not cover the grid.
int group_size(const Server* s, const mm_request& r)
{
    if (s->o.batch <= 1 || !batch_supported(r.grid, s->o.prec)) return 1;
    const long N = (long)r.grid[0] * r.grid[1] * r.grid[2];
    int B = (int)std::min<long>(s->o.batch, std::max<long>(1, kBatchCells / N));
    const bool s64 = s->o.prec == MM_FP32;
    const size_t tb = tensor_bytes(r, s->o.prec);
    while (B > 1 && batch_footprint(r.grid, s->o.prec, B, s64) + tb > s->o.hbm_budget) --B;
    return B;
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

void drop_group_plan(Server* s, Plan* p, Graphs& gr, size_t bytes)
{
    gr.clear();
    s->bytes -= bytes;
    free_plan(p);
}

// Drop an idle group (least recently used first), or a resident spectral
// kernel that no plan uses; false when nothing can be released.
bool release_one(Server* s, const ClassKey* keep)
{
    for (auto it = s->idle.begin(); it != s->idle.end(); ++it) {
        drop_group_plan(s, it->plan, it->graphs, it->bytes);
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

// Give a group's stream slot back; keep its plan (and graph, for batch
// plans) for later requests of the key, or free it.
void retire_group(Server* s, Group* g, bool keep)
{
    if (keep) {
        if (g->B == 1) g->graphs.clear();  // a single plan's graph holds its request
        s->idle.push_back(Idle{g->key, g->plan, g->graphs, g->bytes, g->B});
        g->graphs = Graphs{};
    } else {
        (void)hipStreamSynchronize(s->streams[g->sl]);
        drop_group_plan(s, g->plan, g->graphs, g->bytes);
    }
    g->plan = nullptr;
    s->free_slots.push_back(g->sl);
}

// Every request of a group ends with `st` (a failed launch or copy); the
// group's plan is freed.
void fail_group(Server* s, Group* g, mm_status st)
{
    (void)hipStreamSynchronize(s->streams[g->sl]);
    for (Slot& x : g->slots)
        if (x.busy) {
            finish(s, x.q, st, &x.last, x.t_admit);
            x.busy = x.finishing = false;
        }
    g->inflight = 0;
    retire_group(s, g, false);
}

void set_request(Plan* p, const mm_request& r)
{
    const double nrm = std::sqrt(r.ku_axis[0] * r.ku_axis[0] + r.ku_axis[1] * r.ku_axis[1] +
                                 r.ku_axis[2] * r.ku_axis[2]);
    for (int d = 0; d < 3; ++d) {
        p->d[d] = r.cell[d];
        p->eu[d] = r.ku_axis[d] / nrm;
    }
    p->Ms = r.Ms;
    p->A = r.A;
    p->Ku = r.Ku;
    p->alpha = r.alpha;
    p->n_magnetic = r.Ms > 0.0 ? p->N : 0;
}

// One graph of steps_per_launch steps over the plan's first nb slots.
template <typename T>
mm_status capture_one(Server* s, Group* g, const mm_request& r, int nb, hipGraphExec_t* out)
{
    hipStream_t stream = s->streams[g->sl];
    const bool relax = g->key.kind == MM_SERVE_RELAX;
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    mm_status st = MM_OK;
    // a batch plan reads h_ext and the material per slot from device memory;
    // a single plan's field and material are compiled into the graph
    g->plan->batch = nb;
    for (int i = 0; i < s->o.steps_per_launch && st == MM_OK; ++i)
        st = dev_step<T>(g->plan, r.h_ext, r.terms, r.rtol, r.atol, relax, relax);
    g->plan->batch = g->B;
    e = hipStreamEndCapture(stream, &gr);
    if (st != MM_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "graph capture");
    e = hipGraphInstantiate(out, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) {
        *out = nullptr;
        return hip_fail(e, "graph instantiation");
    }
    return MM_OK;
}

// The group's graphs: a single plan one, a batch plan one per covered slot
// count 1, 2, 4, ..., B.
template <typename T>
mm_status capture(Server* s, Group* g, const mm_request& r)
{
    g->graphs.clear();
    for (int nb = 1;; nb = std::min(2 * nb, g->B)) {
        hipGraphExec_t ex = nullptr;
        mm_status st = capture_one<T>(s, g, r, nb, &ex);
        if (st != MM_OK) {
            g->graphs.clear();
            return st;
        }
        g->graphs.sizes.push_back(nb);
        g->graphs.execs.push_back(ex);
        if (nb == g->B) break;
    }
    return MM_OK;
}

// Slots the next launch must cover: up to the highest one still stepping.
int cover(const Group* g)
{
    int hi = 0;
    for (int b = 0; b < g->B; ++b)
        if (g->slots[b].busy && !g->slots[b].finishing) hi = b + 1;
    return hi;
}

mm_status launch(Server* s, Group* g)
{
    if (g->graphs.empty()) {
        set_error("a group without captured steps was launched");
        return MM_EINVAL;
    }
    hipStream_t stream = s->streams[g->sl];
    const int idx = (g->head + g->inflight) & 1;
    const int need = std::max(1, cover(g));
    size_t gi = 0;
    while (gi + 1 < g->graphs.sizes.size() && g->graphs.sizes[gi] < need) ++gi;
    hipError_t e = hipGraphLaunch(g->graphs.execs[gi], stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(pinned_of(s, g->sl, idx), g->plan->ctl, sizeof(DevCtl) * g->B,
                           hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipEventRecord(launch_event(s, g->sl, idx), stream);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    g->seq[idx] = g->next_seq++;
    g->inflight++;
    s->st.graph_launches++;
    return MM_OK;
}

bool any_stepping(const Group* g)
{
    for (const Slot& x : g->slots)
        if (x.busy && !x.finishing) return true;
    return false;
}

// Start the head of the queue in slot b of group g (its stream orders the
// slot's set-up after the launches in flight): constants, start state, first
// right-hand side and step size, then launches if none are in flight.  The
// queue head is consumed whatever the outcome.
template <typename T>
void admit_into(Server* s, Group* g, int b)
{
    Req q = s->queue.front();
    s->queue.pop_front();
    const mm_request& r = q.r;
    hipStream_t stream = s->streams[g->sl];
    const double t0 = now_s();
    mm_status st = MM_OK;
    if (q.ready) {
        hipError_t e = hipStreamWaitEvent(stream, q.ready, 0);
        if (e != hipSuccess) st = hip_fail(e, "waiting for the start state");
    }
    const bool relax = r.kind == MM_SERVE_RELAX;
    DevCtl c{};
    c.t = 0.0;
    c.dt = -1.0;
    c.t_end = relax ? std::numeric_limits<double>::infinity() : r.t_end;
    c.dt_min = 1e-20;
    c.torque_tol = relax ? r.tol : 0.0;
    c.max_steps = r.max_steps;
    c.relax = relax ? 1 : 0;
    c.renorm = relax ? 1 : 0;
    if (g->B > 1) {
        Plan v = batch_view(*g->plan, b);
        set_request(&v, r);
        if (st == MM_OK) {
            hipError_t e = batch_set_slot(*g->plan, b, v, r.h_ext, r.terms, relax ? 1.0 : r.alpha,
                                          !relax);
            if (e != hipSuccess) st = hip_fail(e, "request constants");
        }
        if (st == MM_OK) st = dev_prepare<T>(&v, r.m, r.h_ext, r.terms, c, r.rtol, r.atol);
        if (st == MM_OK && g->graphs.empty()) st = capture<T>(s, g, r);
    } else {
        set_request(g->plan, r);
        if (st == MM_OK) st = dev_prepare<T>(g->plan, r.m, r.h_ext, r.terms, c, r.rtol, r.atol);
        if (st == MM_OK) st = capture<T>(s, g, r);
    }
    if (st != MM_OK) {
        finish(s, q, st, nullptr, t0);
        return;
    }
    Slot& x = g->slots[b];
    x.busy = true;
    x.finishing = false;
    x.q = q;
    x.t_admit = t0;
    x.first_seq = g->next_seq;
    x.last = DevCtl{};
    s->st.admitted++;
    long n = 0;
    for (const Slot& y : g->slots) n += y.busy ? 1 : 0;
    s->st.max_batch = std::max(s->st.max_batch, n);
    while (g->inflight < 2) {
        st = launch(s, g);
        if (st != MM_OK) {
            fail_group(s, g, st);
            return;
        }
    }
}

// A new group for the queue head's key: an idle one or a new batch plan (the
// class kernel built or shared).  nullptr on failure (the head finished).
Group* make_group(Server* s, int B, Idle* reuse)
{
    const Req& head = s->queue.front();
    const mm_request& r = head.r;
    Group* g = new Group();
    g->key = group_of(r, s->o);
    g->sl = s->free_slots.back();
    s->free_slots.pop_back();
    hipStream_t stream = s->streams[g->sl];
    if (reuse) {
        g->plan = reuse->plan;
        g->graphs = reuse->graphs;
        g->bytes = reuse->bytes;
        g->B = reuse->B;
        g->plan->stream = stream;
        s->st.plans_reused++;
    } else {
        g->B = B;
        const ClassKey ck = g->key.c;
        mm_opts po;
        mm_opts_default(&po);
        po.prec = s->o.prec;
        po.demag_p = s->o.demag_p;
        for (int d = 0; d < 3; ++d) po.ku_axis[d] = r.ku_axis[d];
        po.stream = stream;
        auto ti = s->tensors.find(ck);
        SharedTensor* share = ti == s->tensors.end() ? nullptr : ti->second;
        // The class kernel is built at a canonical cell of the class's shape
        // (x edge 1 nm), so it does not depend on which request came first.
        const double canon[3] = {1e-9, 1e-9 * ck.ry, 1e-9 * ck.rz};
        mm_status st = plan_build(r.grid, share ? r.cell : canon, r.Ms, r.A, r.Ku, r.alpha, po,
                                  share, &g->plan, B);
        if (st == MM_OK && !share) {
            SharedTensor* t = new SharedTensor();
            t->Khat = g->plan->Khat;
            t->tw = g->plan->tw;
            t->bytes = tensor_bytes(r, s->o.prec);
            t->refs = 2;  // the server's and the plan's
            g->plan->shared = t;
            s->tensors[ck] = t;
            s->bytes += t->bytes;
            s->st.tensors_built++;
        }
        if (st == MM_OK) {
            Plan* p = g->plan;
            p->state64 = s->o.prec == MM_FP32;
            p->n_magnetic = p->N;
            st = ensure_rk(p);
            // every slot starts empty: a finished controller, zero vectors
            if (st == MM_OK) {
                std::vector<DevCtl> c0(B);
                for (DevCtl& c : c0) c.done = 1;
                const size_t es = s->o.prec == MM_FP32 ? 4 : 8;
                const size_t n3b = 3 * (size_t)p->N * B;
                hipError_t e = hipMemcpyAsync(p->ctl, c0.data(), sizeof(DevCtl) * B,
                                              hipMemcpyHostToDevice, stream);
                if (e == hipSuccess && B > 1) e = batch_init_slots(*p);
                if (e == hipSuccess) e = hipMemsetAsync(p->rk, 0, 10 * n3b * es, stream);
                if (e == hipSuccess && p->st64)
                    e = hipMemsetAsync(p->st64, 0, 2 * n3b * sizeof(double), stream);
                if (e == hipSuccess) e = hipStreamSynchronize(stream);
                if (e != hipSuccess) st = hip_fail(e, "batch set-up");
            }
        }
        if (st != MM_OK) {
            const Req dead = head;
            s->queue.pop_front();
            finish(s, dead, st, nullptr, 0.0);
            if (g->plan) free_plan(g->plan);
            s->free_slots.push_back(g->sl);
            delete g;
            return nullptr;
        }
        g->bytes = batch_footprint(r.grid, s->o.prec, B, s->o.prec == MM_FP32);
        s->bytes += g->bytes;
        s->st.plans_created++;
    }
    g->slots.assign(g->B, Slot{});
    s->groups.push_back(g);
    s->st.bytes_peak = std::max(s->st.bytes_peak, s->bytes);
    return g;
}

// Admit the head of the queue if a slot of its group, or a stream and memory
// for a new group, allow.  Returns true if the queue may be looked at again.
bool try_admit(Server* s)
{
    if (s->queue.empty()) return false;
    Req& head = s->queue.front();
    const GroupKey key = group_of(head.r, s->o);
    // a free slot in a running group of the key (not one that failed and
    // waits for the next poll to be removed: it has no plan)
    for (Group* g : s->groups) {
        if (!(g->key == key) || !g->plan) continue;
        for (int b = 0; b < g->B; ++b)
            if (!g->slots[b].busy) {
                if (s->o.prec == MM_FP32)
                    admit_into<float>(s, g, b);
                else
                    admit_into<double>(s, g, b);
                if (g->plan) s->st.plans_reused++;
                return true;
            }
    }
    if (s->free_slots.empty()) {
        if (!head.waited_slot) s->st.waited_slot++;
        head.waited_slot = true;
        return false;
    }
    // an idle group of the key needs no new memory
    auto reuse = s->idle.end();
    for (auto it = s->idle.begin(); it != s->idle.end(); ++it)
        if (it->key == key) reuse = it;
    int B = 1;
    if (reuse == s->idle.end()) {
        B = group_size(s, head.r);
        size_t need = batch_footprint(head.r.grid, s->o.prec, B, s->o.prec == MM_FP32);
        if (!s->tensors.count(key.c)) need += tensor_bytes(head.r, s->o.prec);
        while (s->bytes + need > s->o.hbm_budget && release_one(s, &key.c)) {
        }
        if (s->bytes + need > s->o.hbm_budget) {
            if (s->groups.empty()) {
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
    Idle held{};
    const bool have = reuse != s->idle.end();
    if (have) {
        held = *reuse;
        s->idle.erase(reuse);
    }
    Group* g = make_group(s, B, have ? &held : nullptr);
    if (!g) return true;
    if (s->o.prec == MM_FP32)
        admit_into<float>(s, g, 0);
    else
        admit_into<double>(s, g, 0);
    return true;
}

// Advance one group: collect finished result copies and launches, start the
// result copies of finished requests, keep two launches in flight while a
// request steps.  True when the group has retired.
bool progress(Server* s, Group* g)
{
    if (!g->plan) return true;  // failed at admission
    const int sl = g->sl;
    hipStream_t stream = s->streams[sl];
    for (int b = 0; b < g->B; ++b) {
        Slot& x = g->slots[b];
        if (!x.finishing) continue;
        hipError_t e = hipEventQuery(result_event(s, sl, b));
        if (e == hipErrorNotReady) continue;
        finish(s, x.q, e == hipSuccess ? x.last.result : hip_fail(e, "request result"), &x.last,
               x.t_admit);
        x.busy = x.finishing = false;
    }
    while (g->inflight > 0) {
        const int idx = g->head;
        hipError_t e = hipEventQuery(launch_event(s, sl, idx));
        if (e == hipErrorNotReady) break;
        if (e != hipSuccess) {
            fail_group(s, g, hip_fail(e, "graph launch"));
            return true;
        }
        const DevCtl* cp = pinned_of(s, sl, idx);
        const long sq = g->seq[idx];
        g->inflight--;
        g->head ^= 1;
        for (int b = 0; b < g->B; ++b) {
            Slot& x = g->slots[b];
            if (!x.busy || x.finishing || sq < x.first_seq) continue;
            x.last = cp[b];
            if (!x.last.done) continue;
            // launches still in flight leave a finished slot unchanged; the
            // copy follows them
            Plan v = g->B > 1 ? batch_view(*g->plan, b) : *g->plan;
            hipError_t e2 = dev_result(&v, x.q.r.m);
            if (e2 == hipSuccess) e2 = hipEventRecord(result_event(s, sl, b), stream);
            if (e2 != hipSuccess) {
                fail_group(s, g, hip_fail(e2, "request result"));
                return true;
            }
            x.finishing = true;
        }
    }
    if (any_stepping(g)) {
        while (g->inflight < 2) {
            mm_status st = launch(s, g);
            if (st != MM_OK) {
                fail_group(s, g, st);
                return true;
            }
        }
        return false;
    }
    for (const Slot& x : g->slots)
        if (x.busy) return false;  // result copies in flight
    if (g->inflight > 0) return false;
    retire_group(s, g, true);
    return true;
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
    o->batch = 8;
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
        o.steps_per_launch > 64 || o.batch < 1 || o.batch > 64 ||
        (o.prec != MM_FP32 && o.prec != MM_FP64)) {
        set_error("max_active, steps_per_launch and batch must lie in [1, 64], prec FP32 or FP64");
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
    hipError_t e = hipHostMalloc((void**)&s->pinned,
                                 (size_t)2 * o.batch * o.max_active * sizeof(DevCtl),
                                 hipHostMallocDefault);
    if (e != hipSuccess) s->pinned = nullptr;
    for (int i = 0; i < o.max_active && e == hipSuccess; ++i) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) s->streams.push_back(st);
        for (int k = 0; k < 2 + o.batch && e == hipSuccess; ++k) {
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
    for (size_t i = 0; i < s->groups.size();) {
        Group* g = s->groups[i];
        if (progress(s, g)) {
            delete g;
            s->groups.erase(s->groups.begin() + i);
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
    long act = 0;
    for (const Group* g : s->groups)
        for (const Slot& x : g->slots) act += x.busy ? 1 : 0;
    st->active = act;
    st->bytes_in_use = s->bytes;
    return MM_OK;
}

void mm_serve_destroy(mm_server* sv)
{
    Server* s = reinterpret_cast<Server*>(sv);
    if (!s) return;
    for (Group* g : s->groups) {
        if (g->plan) {
            (void)hipStreamSynchronize(s->streams[g->sl]);
            g->graphs.clear();
            free_plan(g->plan);
        }
        for (Slot& x : g->slots)
            if (x.busy && x.q.ready) (void)hipEventDestroy(x.q.ready);
        delete g;
    }
    for (auto& q : s->queue)
        if (q.ready) (void)hipEventDestroy(q.ready);
    for (auto& i : s->idle) {
        i.graphs.clear();
        free_plan(i.plan);
    }
    for (auto& t : s->tensors) release_tensor(t.second);
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    if (s->pinned) (void)hipHostFree(s->pinned);
    delete s;
}

}  // extern "C"
