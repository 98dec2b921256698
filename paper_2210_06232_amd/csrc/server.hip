// server.hip -- continuous-batching execution of many independent EI-FP solves.
//
// Requests are grouped by (nx, ny, nz, precision).  A group owns the executor for its
// shape (twiddle tables), one stream, and a device array of member descriptors; one
// chunk of k steps of the whole group is k launches of the five-pass step (or k
// replays of a HIP graph captured for the group's current batch size), so every
// member advances by k steps in the same kernels.  Members join and leave between
// chunks.  k stops at the next output point of any member and is capped so that a
// chunk lasts a few milliseconds, which bounds how long an arrival waits to join.
// Groups of different shapes live on different streams, so their chunks overlap on
// the device.
//
// One host thread (the scheduler) makes every HIP call of the loop: completion checks
// (event queries), admission (allocation and upload), descriptor updates and launches.
// API calls from other threads only touch host queues under the server mutex, except
// eifp_server_fields, which copies on its own stream while the scheduler holds the
// request's group idle.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "engine.h"

using namespace eifp;

namespace {

using Clock = std::chrono::steady_clock;

constexpr double kChunkTargetMs = 4.0;   // wall time one chunk aims at
constexpr double kHeadAgingS = 0.5;      // after this wait the queue head blocks bypass
constexpr double kModelBw = 4.0e12;      // bytes/s, first guess of a step's time

struct Key {
    int nx, ny, nz, prec;
    int anchored;  // members advance by jumps from their anchored spectra
    bool operator<(const Key& o) const {
        return std::tie(nx, ny, nz, prec, anchored) < std::tie(o.nx, o.ny, o.nz, o.prec, o.anchored);
    }
};

Key key_of(const eifp_request& rq) {
    return Key{rq.nx, rq.ny, rq.nz, (int)rq.prec, (rq.flags & EIFP_REQ_ANCHORED) ? 1 : 0};
}

struct Group;

struct Req {
    long long id = 0;
    eifp_request rq{};            // H0/E0 cleared after the copy
    std::vector<double> host64;   // FP64 request: H then E
    std::vector<float> host32;    // FP32 request: H then E, rounded once on the host
    PropParams pp{};
    double t_arrive = 0, t_admit = 0;
    long long state_bytes = 0, bytes = 0;
    void* state = nullptr;
    void* snap = nullptr;
    void* spec = nullptr;  // anchored spectrum (anchored requests)
    void* work = nullptr;  // transform buffer of stepped requests with large states
    bool anchored = false;  // spec holds the spectrum of the initial state
    Group* g = nullptr;
    long long done = 0;    // steps completed and observed
    long long target = 0;  // steps done once the in-flight chunk completes
    bool has_snap = false;
    long long snap_step = 0;  // steps done when the current snapshot was taken
    bool finished = false;
    bool kept = false;
    bool cancel = false;   // eifp_server_cancel asked; ends where no chunk or copy uses it
    int readers = 0;       // eifp_server_fields calls copying from this request
};

struct Group {
    Key key{};
    Engine en;
    hipStream_t st = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    void* desc_dev = nullptr;
    DescImage* desc_host = nullptr;  // pinned
    double* partials = nullptr;
    double* inv_dev = nullptr;
    double* inv_host = nullptr;      // pinned
    long long bytes = 0;
    int nparts = 0;
    std::vector<Req*> members;
    bool dirty = true;
    bool in_flight = false;
    int k = 0;                       // steps in flight
    int nm_flight = 0;
    std::map<std::pair<int, bool>, hipGraphExec_t> graphs;  // (batch size, with invariants)
    double ms_per_member_step = 0;   // running estimate
    int readers = 0;
};

long long state_bytes_of(int nx, int ny, int nz, int prec) {
    return 6LL * nx * ny * nz * (prec == EIFP_FP64 ? 8 : 4);
}

// partial records per member (the capacity the engine's passes need)
int nparts_of(const Key& k) {
    const Grid3 g{k.nx, k.ny, k.nz, k.nx / 2};
    return k.prec == EIFP_FP64 ? partial_capacity<double>(g) : partial_capacity<float>(g);
}

long long group_bytes_of(const Key& k, int max_batch) {
    const long long ts = k.prec == EIFP_FP64 ? 8 : 4;
    const long long np = nparts_of(k);
    // partial and invariant slots, two descriptor regions (jumps and anchoring), tables
    return (long long)max_batch * (np * INV_NPART * 8 + 8 * 8 + 2 * (long long)sizeof(DescImage)) +
           2 * ts * (k.nx + k.ny + k.nz);
}

// Stepped requests whose state is at least this large transform in a work buffer of
// their own, so that a chunk's steps run the x inverse of one step and the x forward of
// the next as one kernel (one read of the state fewer per step); their chunks are
// enqueued kernel by kernel, which costs nothing next to kernels of this size.  Smaller
// requests step in place from captured one-step graphs.
constexpr long long kCombineBytes = 64LL << 20;

bool uses_work(long long state_bytes, int flags) {
    return !(flags & EIFP_REQ_ANCHORED) && state_bytes >= kCombineBytes;
}

long long footprint_of(int nx, int ny, int nz, int prec, int flags) {
    const long long sb = state_bytes_of(nx, ny, nz, prec);
    return sb * (1 + ((flags & EIFP_REQ_NO_SNAPSHOT) ? 0 : 1) + ((flags & EIFP_REQ_ANCHORED) ? 1 : 0) +
                 (uses_work(sb, flags) ? 1 : 0));
}

double pct(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    size_t r = (size_t)std::ceil(q * (double)v.size());
    if (r < 1) r = 1;
    return v[r - 1];
}

}  // namespace

struct eifp_server {
    long long budget = 0;
    int max_batch = 1;
    int flags = 0;
    bool dry = false;
    int device = 0;
    Clock::time_point t0 = Clock::now();

    std::mutex mu;
    std::condition_variable cv_sched, cv_ev;
    std::deque<Req*> pending;
    std::map<long long, std::unique_ptr<Req>> reqs;
    std::map<Key, std::unique_ptr<Group>> groups;
    std::deque<eifp_event> events;
    std::vector<double> lat;
    long long next_id = 1;
    long long submitted = 0, admitted = 0, completed = 0, failed = 0, running = 0, peak_running = 0;
    long long cancelled = 0;
    long long cancel_asks = 0;  // requests asked to cancel that have not ended yet
    long long used = 0, peak = 0;
    long long chunks = 0;
    double batch_sum = 0;
    double point_steps = 0;
    double first_arrive = -1, last_done = 0;
    bool stop = false;
    std::thread th;
    // host-side fault injection for tests of failure isolation: with
    // EIFP_SERVER_FAULT_CHUNK=n in the environment when the server is created, its n-th
    // chunk (counted over all groups from 1) fails as a device error would, before
    // anything is enqueued; its members end with an error event and the server goes on
    long long fault_chunk = 0, chunk_attempts = 0;

    double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

// ------------------------------- device side of a group ------------------------------

void group_free(Group* g) {
    if (!g) return;
    if (g->st) (void)hipStreamSynchronize(g->st);
    for (auto& kv : g->graphs) (void)hipGraphExecDestroy(kv.second);
    g->graphs.clear();
    for (void* p : {g->desc_dev, (void*)g->partials, (void*)g->inv_dev})
        if (p) (void)hipFree(p);
    if (g->desc_host) (void)hipHostFree(g->desc_host);
    if (g->inv_host) (void)hipHostFree(g->inv_host);
    if (g->ev0) (void)hipEventDestroy(g->ev0);
    if (g->ev1) (void)hipEventDestroy(g->ev1);
    if (g->st) (void)hipStreamDestroy(g->st);
    g->en.release();
}

eifp_status group_alloc(Group* g, int max_batch) {
    EIFP_HIP_TRY(hipStreamCreateWithFlags(&g->st, hipStreamNonBlocking));
    EIFP_HIP_TRY(hipEventCreate(&g->ev0));
    EIFP_HIP_TRY(hipEventCreate(&g->ev1));
    eifp_status st = g->en.init(g->key.nx, g->key.ny, g->key.nz, (eifp_precision)g->key.prec, g->st);
    if (st) return st;
    g->nparts = g->en.nrec;
    const size_t pb = (size_t)max_batch * g->nparts * INV_NPART * sizeof(double);
    if (hipMalloc((void**)&g->partials, pb) != hipSuccess || hipMalloc((void**)&g->inv_dev, max_batch * 64) != hipSuccess ||
        hipMalloc(&g->desc_dev, 2 * max_batch * sizeof(DescImage)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(EIFP_ERR_OUT_OF_MEMORY, "batch table allocation failed");
    }
    EIFP_HIP_TRY(hipHostMalloc((void**)&g->desc_host, 2 * max_batch * sizeof(DescImage), hipHostMallocDefault));
    EIFP_HIP_TRY(hipHostMalloc((void**)&g->inv_host, max_batch * 64, hipHostMallocDefault));
    return EIFP_OK;
}

void req_free_buffers(eifp_server* sv, Req* r) {
    if (!sv->dry)
        for (void* p : {r->state, r->snap, r->spec, r->work})
            if (p) (void)hipFree(p);
    r->state = r->snap = r->spec = r->work = nullptr;
}

void req_free_device(eifp_server* sv, Req* r) {
    req_free_buffers(sv, r);
    sv->used -= r->bytes;
    r->bytes = 0;
}

// ------------------------------- events ----------------------------------------------

void push_event(eifp_server* sv, Req* r, int kind, eifp_status st, const double* inv) {
    eifp_event e{};
    e.user_tag = r->rq.user_tag;
    e.req_id = r->id;
    e.kind = kind;
    e.status = st;
    e.step = r->done;
    e.inv.t = r->rq.tau * (double)r->done;
    e.inv.steps_done = r->done;
    if (inv) {
        e.inv.energy = inv[0];
        e.inv.helicity = inv[1];
        e.inv.momentum[0] = inv[2];
        e.inv.momentum[1] = inv[3];
        e.inv.momentum[2] = inv[4];
        e.inv.div_h_l2 = inv[5];
        e.inv.div_e_l2 = inv[6];
    }
    e.t_arrive = r->t_arrive;
    e.t_admit = r->t_admit;
    e.t_event = sv->now();
    sv->events.push_back(e);
    sv->cv_ev.notify_all();
}

enum class End { Done, Failed, Cancelled };

// Retire a member that finished, failed or was cancelled: free or keep its memory,
// record stats.
void retire(eifp_server* sv, Req* r, End how) {
    const bool ok = how == End::Done;
    if (r->cancel) sv->cancel_asks--;
    Group* g = r->g;
    if (g) {
        g->members.erase(std::remove(g->members.begin(), g->members.end(), r), g->members.end());
        g->dirty = true;
    }
    r->g = nullptr;
    r->finished = true;
    sv->running--;
    const double t = sv->now();
    if (ok) {
        sv->completed++;
        sv->lat.push_back(t - r->t_arrive);
        sv->point_steps += (double)r->rq.nx * r->rq.ny * r->rq.nz * (double)r->rq.nsteps;
        sv->last_done = t;
    } else if (how == End::Cancelled) {
        sv->cancelled++;
    } else {
        sv->failed++;
    }
    if (ok && (r->rq.flags & EIFP_REQ_KEEP_RESULT)) {
        // keep the final state; the snapshot buffer goes back to the budget
        r->kept = true;
        if (!sv->dry)
            for (void* p : {r->snap, r->spec, r->work})
                if (p) (void)hipFree(p);
        const long long extra = (long long)(!(r->rq.flags & EIFP_REQ_NO_SNAPSHOT)) +
                                (long long)((r->rq.flags & EIFP_REQ_ANCHORED) != 0) +
                                (long long)uses_work(r->state_bytes, r->rq.flags);
        sv->used -= extra * r->state_bytes;
        r->bytes -= extra * r->state_bytes;
        r->snap = r->spec = r->work = nullptr;
        r->has_snap = false;
    } else {
        req_free_device(sv, r);
        sv->reqs.erase(r->id);  // r is dead after this
    }
}

void fail_group(eifp_server* sv, Group* g, eifp_status st) {
    std::vector<Req*> ms = g->members;
    for (Req* r : ms) {
        push_event(sv, r, EIFP_EV_ERROR, st, nullptr);
        retire(sv, r, End::Failed);
    }
    g->in_flight = false;
}

// End the requests asked to cancel wherever that is safe now: queued ones at once,
// members of a batch with no chunk in flight and no field copy reading them.  Returns
// whether any ended.
bool reap_cancelled(eifp_server* sv) {
    bool progress = false;
    for (auto it = sv->pending.begin(); it != sv->pending.end();) {
        Req* r = *it;
        if (!r->cancel) {
            ++it;
            continue;
        }
        it = sv->pending.erase(it);
        push_event(sv, r, EIFP_EV_ERROR, EIFP_ERR_CANCELLED, nullptr);
        sv->cancel_asks--;
        sv->cancelled++;
        sv->reqs.erase(r->id);  // r is dead after this
        progress = true;
    }
    for (auto& kv : sv->groups) {
        Group* g = kv.second.get();
        if (g->in_flight) continue;
        const std::vector<Req*> ms = g->members;
        for (Req* r : ms)
            if (r->cancel && r->readers == 0) {
                // admitted but not yet stepped: its upload (enqueued on the idle group's
                // stream, reading the host copy) may still be running
                if (!sv->dry && (!r->host64.empty() || !r->host32.empty())) (void)hipStreamSynchronize(g->st);
                push_event(sv, r, EIFP_EV_ERROR, EIFP_ERR_CANCELLED, nullptr);
                retire(sv, r, End::Cancelled);
                progress = true;
            }
    }
    return progress;
}

// ------------------------------- admission -------------------------------------------

Group* get_group(eifp_server* sv, const Key& k, eifp_status* st) {
    auto it = sv->groups.find(k);
    if (it != sv->groups.end()) return it->second.get();
    std::unique_ptr<Group> g(new Group);
    g->key = k;
    g->bytes = group_bytes_of(k, sv->max_batch);
    g->nparts = nparts_of(k);
    if (!sv->dry) {
        *st = group_alloc(g.get(), sv->max_batch);
        if (*st) {
            group_free(g.get());
            return nullptr;
        }
    }
    sv->used += g->bytes;
    sv->peak = std::max(sv->peak, sv->used);
    Group* raw = g.get();
    sv->groups[k] = std::move(g);
    return raw;
}

// Allocate the request's device memory and enqueue its upload on the group's stream
// (the group is idle, so the next chunk is ordered after the upload).
eifp_status admit_one(eifp_server* sv, Req* r, Group* g) {
    r->state_bytes = state_bytes_of(r->rq.nx, r->rq.ny, r->rq.nz, r->rq.prec);
    const long long fp = footprint_of(r->rq.nx, r->rq.ny, r->rq.nz, r->rq.prec, r->rq.flags);
    if (!sv->dry) {
        if (hipMalloc(&r->state, r->state_bytes) != hipSuccess ||
            (!(r->rq.flags & EIFP_REQ_NO_SNAPSHOT) && hipMalloc(&r->snap, r->state_bytes) != hipSuccess) ||
            ((r->rq.flags & EIFP_REQ_ANCHORED) && hipMalloc(&r->spec, r->state_bytes) != hipSuccess) ||
            (uses_work(r->state_bytes, r->rq.flags) && hipMalloc(&r->work, r->state_bytes) != hipSuccess)) {
            (void)hipGetLastError();
            req_free_buffers(sv, r);
            return fail(EIFP_ERR_OUT_OF_MEMORY, "request allocation failed");
        }
        const void* src = r->rq.prec == EIFP_FP64 ? (const void*)r->host64.data() : (const void*)r->host32.data();
        EIFP_HIP_TRY(hipMemcpyAsync(r->state, src, r->state_bytes, hipMemcpyHostToDevice, g->st));
    }
    r->bytes = fp;
    sv->used += fp;
    sv->peak = std::max(sv->peak, sv->used);
    r->g = g;
    r->t_admit = sv->now();
    g->members.push_back(r);
    g->dirty = true;
    sv->admitted++;
    sv->running++;
    sv->peak_running = std::max(sv->peak_running, sv->running);
    return EIFP_OK;
}

bool admit(eifp_server* sv) {
    bool progress = false;
    const double t = sv->now();
    for (auto it = sv->pending.begin(); it != sv->pending.end();) {
        Req* r = *it;
        if ((sv->flags & EIFP_SERVER_SERIAL) && sv->running > 0) break;
        const Key k = key_of(r->rq);
        auto git = sv->groups.find(k);
        Group* g = git == sv->groups.end() ? nullptr : git->second.get();
        const long long need = footprint_of(k.nx, k.ny, k.nz, k.prec, r->rq.flags) +
                               (g ? 0 : group_bytes_of(k, sv->max_batch));
        const bool slot = !g || (!g->in_flight && g->readers == 0 && (int)g->members.size() < sv->max_batch);
        const bool fits = sv->used + need <= sv->budget;
        if (slot && fits) {
            eifp_status st = EIFP_OK;
            if (!g) g = get_group(sv, k, &st);
            if (g) st = admit_one(sv, r, g);
            it = sv->pending.erase(it);
            progress = true;
            if (st != EIFP_OK) {
                // the request never ran: report and drop it
                r->done = 0;
                push_event(sv, r, EIFP_EV_ERROR, st, nullptr);
                sv->failed++;
                if (r->cancel) sv->cancel_asks--;
                if (r->state || r->snap || r->spec) req_free_device(sv, r);
                sv->reqs.erase(r->id);
            }
            continue;
        }
        // keep arrival order once the head has waited long enough (no starvation of
        // large requests behind a stream of small ones)
        if (it == sv->pending.begin() && !fits && t - r->t_arrive > kHeadAgingS) break;
        ++it;
    }
    return progress;
}

// ------------------------------- chunks ----------------------------------------------

long long next_boundary(const Req* r) {
    const long long c = r->rq.cadence;
    long long b = r->rq.nsteps;
    if (c > 0) b = std::min(b, (r->done / c + 1) * c);
    return b;
}

eifp_status capture_step_graph(Group* g, int nm, bool want_inv, hipGraphExec_t* out) {
    hipGraph_t graph = nullptr;
    EIFP_HIP_TRY(hipStreamBeginCapture(g->st, hipStreamCaptureModeThreadLocal));
    const eifp_status st = g->en.passes(Z_STEP, g->desc_dev, nm, g->st, nullptr, want_inv);
    const hipError_t e = hipStreamEndCapture(g->st, &graph);
    if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(EIFP_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    const hipError_t ei = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(EIFP_ERR_DEVICE, "graph instantiate failed: %s", hipGetErrorString(ei));
    return EIFP_OK;
}

// A chunk of a jump group: members not yet anchored get their spectrum stored (forward
// transform into spec, through the second descriptor region), then every member jumps
// from its anchor to its own next output point (descriptor region one, rewritten each
// chunk since the time spans change).  Every jump ends at an output point, so the
// invariants are always reduced.
eifp_status launch_jump_chunk(eifp_server* sv, Group* g) {
    const int nm = (int)g->members.size();
    const Grid3& gg = g->en.g;
    if (!sv->dry) {
        int na = 0;
        for (Req* r : g->members)
            if (!r->anchored) {
                const PropParams p0 = make_params(gg.nx, gg.ny, gg.nz, r->rq.dom, r->rq.mu, r->rq.eps, 0.0);
                g->desc_host[sv->max_batch + na++] = DescImage{r->state, r->spec, nullptr, nullptr, nullptr, p0};
            }
        for (int i = 0; i < nm; ++i) {
            Req* r = g->members[i];
            const double span = r->rq.tau * (double)next_boundary(r);
            g->desc_host[i] = DescImage{r->state, r->state, g->partials + (size_t)i * g->nparts * INV_NPART,
                                        g->inv_dev + (size_t)i * 8, r->spec,
                                        make_params(gg.nx, gg.ny, gg.nz, r->rq.dom, r->rq.mu, r->rq.eps, span)};
        }
        EIFP_HIP_TRY(hipMemcpyAsync(g->desc_dev, g->desc_host, (size_t)(sv->max_batch + na) * sizeof(DescImage),
                                    hipMemcpyHostToDevice, g->st));
        EIFP_HIP_TRY(hipEventRecord(g->ev0, g->st));
        eifp_status st;
        if (na && (st = g->en.forward_spectrum((const char*)g->desc_dev + sv->max_batch * sizeof(DescImage), na, g->st)))
            return st;
        if ((st = g->en.jump(g->desc_dev, nm, g->st, true))) return st;
        for (Req* r : g->members)
            if (r->snap && next_boundary(r) < r->rq.nsteps)
                EIFP_HIP_TRY(hipMemcpyAsync(r->snap, r->state, r->state_bytes, hipMemcpyDeviceToDevice, g->st));
        EIFP_HIP_TRY(hipMemcpyAsync(g->inv_host, g->inv_dev, (size_t)nm * 64, hipMemcpyDeviceToHost, g->st));
        EIFP_HIP_TRY(hipEventRecord(g->ev1, g->st));
    }
    long long kmax = 0;
    for (Req* r : g->members) {
        r->anchored = true;
        r->target = next_boundary(r);
        kmax = std::max(kmax, r->target - r->done);
    }
    g->dirty = false;
    g->k = (int)std::min<long long>(kmax, 1 << 30);
    g->nm_flight = nm;
    g->in_flight = true;
    sv->chunks++;
    sv->batch_sum += nm;
    return EIFP_OK;
}

eifp_status launch_chunk(eifp_server* sv, Group* g) {
    const int nm = (int)g->members.size();
    long long k = 1LL << 40;
    for (Req* r : g->members) k = std::min(k, next_boundary(r) - r->done);
    const double est = g->ms_per_member_step > 0
                           ? g->ms_per_member_step * nm
                           : 1e3 * 10.0 * (double)state_bytes_of(g->key.nx, g->key.ny, g->key.nz, g->key.prec) * nm /
                                 kModelBw;
    const long long kcap = std::max(1LL, (long long)(kChunkTargetMs / std::max(est, 1e-6)));
    k = std::max(1LL, std::min(k, kcap));
    if (!sv->dry) {
        if (g->dirty) {
            for (int i = 0; i < nm; ++i) {
                Req* r = g->members[i];
                g->desc_host[i] = DescImage{r->state, r->work ? r->work : r->state,
                                            g->partials + (size_t)i * g->nparts * INV_NPART,
                                            g->inv_dev + (size_t)i * 8, nullptr, r->pp};
            }
            EIFP_HIP_TRY(hipMemcpyAsync(g->desc_dev, g->desc_host, nm * sizeof(DescImage), hipMemcpyHostToDevice, g->st));
        }
        // invariants are reduced only on the chunk's last step, and only if a member
        // reaches an output point there
        bool out_at_end = false;
        for (Req* r : g->members) out_at_end |= r->done + k == next_boundary(r);
        EIFP_HIP_TRY(hipEventRecord(g->ev0, g->st));
        const bool combine = uses_work(state_bytes_of(g->key.nx, g->key.ny, g->key.nz, g->key.prec), 0);
        if (combine) {
            // every member has a work buffer: the chunk's steps as one sequence, the x
            // inverse of a step and the x forward of the next as one kernel
            eifp_status st = g->en.steps(g->desc_dev, nm, k, g->st, nullptr, out_at_end ? k - 1 : k, true);
            if (st) return st;
        }
        for (long long s = 0; s < (combine ? 0 : k); ++s) {
            const bool inv = out_at_end && s == k - 1;
            if (sv->flags & EIFP_SERVER_NO_GRAPHS) {
                eifp_status st = g->en.passes(Z_STEP, g->desc_dev, nm, g->st, nullptr, inv);
                if (st) return st;
                continue;
            }
            hipGraphExec_t& ge = g->graphs[std::make_pair(nm, inv)];
            if (!ge) {
                eifp_status st = capture_step_graph(g, nm, inv, &ge);
                if (st) {
                    g->graphs.erase(std::make_pair(nm, inv));
                    return st;
                }
            }
            EIFP_HIP_TRY(hipGraphLaunch(ge, g->st));
        }
        for (Req* r : g->members)
            if (r->snap && r->done + k == next_boundary(r) && r->done + k < r->rq.nsteps)
                EIFP_HIP_TRY(hipMemcpyAsync(r->snap, r->state, r->state_bytes, hipMemcpyDeviceToDevice, g->st));
        EIFP_HIP_TRY(hipMemcpyAsync(g->inv_host, g->inv_dev, (size_t)nm * 64, hipMemcpyDeviceToHost, g->st));
        EIFP_HIP_TRY(hipEventRecord(g->ev1, g->st));
    }
    g->dirty = false;
    for (Req* r : g->members) r->target = r->done + k;
    g->k = (int)k;
    g->nm_flight = nm;
    g->in_flight = true;
    sv->chunks++;
    sv->batch_sum += nm;
    return EIFP_OK;
}

// Returns true if the group's chunk has completed (and processes it).
bool poll_group(eifp_server* sv, Group* g) {
    if (!sv->dry) {
        const hipError_t q = hipEventQuery(g->ev1);
        if (q == hipErrorNotReady) return false;
        if (q != hipSuccess) {
            fail(EIFP_ERR_DEVICE, "chunk failed: %s", hipGetErrorString(q));
            fail_group(sv, g, EIFP_ERR_DEVICE);
            return true;
        }
        float ms = 0.f;
        if (!g->key.anchored && hipEventElapsedTime(&ms, g->ev0, g->ev1) == hipSuccess && g->k > 0 &&
            g->nm_flight > 0) {
            const double m = (double)ms / ((double)g->k * g->nm_flight);
            g->ms_per_member_step = g->ms_per_member_step > 0 ? 0.5 * (g->ms_per_member_step + m) : m;
        }
    }
    g->in_flight = false;
    std::vector<Req*> ms = g->members;
    for (int i = 0; i < (int)ms.size(); ++i) {
        Req* r = ms[i];
        r->done = r->target;
        // the upload buffer is no longer needed once a chunk has run after it
        if (!r->host64.empty()) std::vector<double>().swap(r->host64);
        if (!r->host32.empty()) std::vector<float>().swap(r->host32);
        const bool at_end = r->done >= r->rq.nsteps;
        const bool at_out = r->rq.cadence > 0 && r->done % r->rq.cadence == 0;
        if (!at_end && !at_out) continue;
        const double* inv = sv->dry ? nullptr : g->inv_host + 8 * i;
        bool finite = true;
        if (inv)
            for (int q = 0; q < 7; ++q) finite = finite && std::isfinite(inv[q]);
        if (!finite) {
            push_event(sv, r, EIFP_EV_ERROR, EIFP_ERR_NONFINITE, inv);
            retire(sv, r, End::Failed);
            continue;
        }
        if (r->snap && !at_end) {
            r->has_snap = true;
            r->snap_step = r->done;
        }
        push_event(sv, r, at_end ? EIFP_EV_DONE : EIFP_EV_OUTPUT, EIFP_OK, inv);
        if (at_end) retire(sv, r, End::Done);
    }
    return true;
}

void drop_idle_groups(eifp_server* sv) {
    for (auto it = sv->groups.begin(); it != sv->groups.end();) {
        Group* g = it->second.get();
        if (g->members.empty() && !g->in_flight && g->readers == 0) {
            if (!sv->dry) group_free(g);
            sv->used -= g->bytes;
            it = sv->groups.erase(it);
        } else {
            ++it;
        }
    }
}

void scheduler(eifp_server* sv) {
    if (!sv->dry) (void)hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    while (!sv->stop) {
        bool progress = false, busy = false;
        for (auto& kv : sv->groups) {
            Group* g = kv.second.get();
            if (g->in_flight) progress |= poll_group(sv, g);
        }
        if (sv->cancel_asks > 0) progress |= reap_cancelled(sv);
        progress |= admit(sv);
        for (auto& kv : sv->groups) {
            Group* g = kv.second.get();
            if (!g->in_flight && !g->members.empty() && g->readers == 0) {
                eifp_status st;
                if (sv->fault_chunk > 0 && ++sv->chunk_attempts == sv->fault_chunk)
                    st = fail(EIFP_ERR_DEVICE, "injected fault at chunk %lld (EIFP_SERVER_FAULT_CHUNK)", sv->fault_chunk);
                else
                    st = g->key.anchored ? launch_jump_chunk(sv, g) : launch_chunk(sv, g);
                if (st) fail_group(sv, g, st);
                progress = true;
            }
            busy |= g->in_flight;
        }
        // empty groups keep their tables (a later request of the same shape reuses them)
        // until a queued request is waiting for device memory
        if (!sv->pending.empty()) drop_idle_groups(sv);
        if (sv->pending.empty() && sv->running == 0) sv->cv_ev.notify_all();  // drained
        if (progress) {
            // let host calls take the lock between iterations (a dry-run scheduler never
            // waits on the device, so without this it could hold the lock indefinitely)
            lk.unlock();
            if (sv->dry)
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            else
                std::this_thread::yield();
            lk.lock();
            continue;
        }
        if (busy)
            sv->cv_sched.wait_for(lk, std::chrono::microseconds(50));
        else
            sv->cv_sched.wait(lk);
    }
    // shutdown: wait for in-flight chunks, then free everything
    for (auto& kv : sv->groups)
        if (!sv->dry && kv.second->st) (void)hipStreamSynchronize(kv.second->st);
    for (auto& kv : sv->reqs) req_free_buffers(sv, kv.second.get());
    sv->reqs.clear();
    sv->pending.clear();
    for (auto& kv : sv->groups)
        if (!sv->dry) group_free(kv.second.get());
    sv->groups.clear();
    sv->cv_ev.notify_all();
}

eifp_status validate_request(const eifp_request* rq) {
    if (!rq) return fail(EIFP_ERR_INVALID_ARG, "NULL request");
    if (!rq->H0 || !rq->E0) return fail(EIFP_ERR_INVALID_ARG, "NULL field pointer");
    eifp_status st;
    if ((st = validate_shape(rq->nx, rq->ny, rq->nz)) || (st = validate_problem(&rq->dom, rq->mu, rq->eps)) ||
        (st = validate_tau(rq->tau)))
        return st;
    if (rq->prec != EIFP_FP64 && rq->prec != EIFP_FP32) return fail(EIFP_ERR_INVALID_ARG, "unknown precision");
    if (rq->nsteps < 1) return fail(EIFP_ERR_INVALID_ARG, "nsteps must be >= 1");
    if (rq->cadence < 0) return fail(EIFP_ERR_INVALID_ARG, "cadence must be >= 0");
    return EIFP_OK;
}

}  // namespace

extern "C" {

eifp_status eifp_server_create(eifp_server** out, long long hbm_budget_bytes, int max_batch, int flags) {
    clear_error();
    if (!out) return fail(EIFP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (hbm_budget_bytes <= 0) return fail(EIFP_ERR_INVALID_ARG, "budget must be positive");
    if (max_batch < 1 || max_batch > 1024) return fail(EIFP_ERR_INVALID_ARG, "max_batch must be in 1..1024");
    eifp_server* sv = new (std::nothrow) eifp_server;
    if (!sv) return fail(EIFP_ERR_OUT_OF_MEMORY, "host allocation failed");
    sv->budget = hbm_budget_bytes;
    sv->max_batch = (flags & EIFP_SERVER_SERIAL) ? 1 : max_batch;
    sv->flags = flags;
    sv->dry = (flags & EIFP_SERVER_DRY_RUN) != 0;
    if (const char* f = std::getenv("EIFP_SERVER_FAULT_CHUNK")) sv->fault_chunk = std::atoll(f);
    if (!sv->dry && hipGetDevice(&sv->device) != hipSuccess) {
        delete sv;
        return fail(EIFP_ERR_DEVICE, "no HIP device");
    }
    try {
        sv->th = std::thread(scheduler, sv);
    } catch (...) {
        delete sv;
        return fail(EIFP_ERR_DEVICE, "scheduler thread creation failed");
    }
    *out = sv;
    return EIFP_OK;
}

long long eifp_server_footprint(int nx, int ny, int nz, eifp_precision prec, int flags) {
    if (validate_shape(nx, ny, nz) != EIFP_OK || (prec != EIFP_FP64 && prec != EIFP_FP32)) {
        clear_error();
        return 0;
    }
    return footprint_of(nx, ny, nz, prec, flags);
}

eifp_status eifp_server_submit(eifp_server* sv, const eifp_request* rq, long long* req_id) {
    clear_error();
    if (!sv || !req_id) return fail(EIFP_ERR_INVALID_ARG, "NULL argument");
    eifp_status st = validate_request(rq);
    if (st) return st;
    const Key k = key_of(*rq);
    const long long need = footprint_of(k.nx, k.ny, k.nz, k.prec, rq->flags) + group_bytes_of(k, sv->max_batch);
    if (need > sv->budget)
        return fail(EIFP_ERR_OUT_OF_MEMORY, "request needs %lld bytes, budget is %lld", need, sv->budget);
    const long long n3 = 3LL * rq->nx * rq->ny * rq->nz;
    std::unique_ptr<Req> r(new (std::nothrow) Req);
    if (!r) return fail(EIFP_ERR_OUT_OF_MEMORY, "host allocation failed");
    // copy (and for FP32 round once, to nearest, as the device conversion does)
    try {
        if (rq->prec == EIFP_FP64) r->host64.resize(2 * n3);
        else r->host32.resize(2 * n3);
    } catch (...) {
        return fail(EIFP_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
    for (int part = 0; part < 2; ++part) {
        const double* src = part ? rq->E0 : rq->H0;
        for (long long q = 0; q < n3; ++q) {
            const double v = src[q];
            if (!std::isfinite(v))
                return fail(EIFP_ERR_NONFINITE, "initial field holds NaN/Inf at flat index %lld", part * n3 + q);
            if (rq->prec == EIFP_FP64) r->host64[part * n3 + q] = v;
            else r->host32[part * n3 + q] = (float)v;
        }
    }
    r->rq = *rq;
    r->rq.H0 = r->rq.E0 = nullptr;
    r->pp = make_params(rq->nx, rq->ny, rq->nz, rq->dom, rq->mu, rq->eps, rq->tau);
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return fail(EIFP_ERR_STATE, "server is shutting down");
    r->id = sv->next_id++;
    r->t_arrive = sv->now();
    if (sv->first_arrive < 0) sv->first_arrive = r->t_arrive;
    *req_id = r->id;
    sv->pending.push_back(r.get());
    sv->reqs[r->id] = std::move(r);
    sv->submitted++;
    sv->cv_sched.notify_one();
    return EIFP_OK;
}

eifp_status eifp_server_poll(eifp_server* sv, eifp_event* ev, int max_events, int* n_events, int wait_ms) {
    clear_error();
    if (!sv || !n_events || (max_events > 0 && !ev) || max_events < 0) return fail(EIFP_ERR_INVALID_ARG, "bad argument");
    *n_events = 0;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto ready = [&] { return !sv->events.empty() || sv->stop || (sv->pending.empty() && sv->running == 0); };
    if (wait_ms > 0)
        sv->cv_ev.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !sv->events.empty() || sv->stop; });
    else if (wait_ms < 0)
        sv->cv_ev.wait(lk, ready);
    int n = 0;
    while (n < max_events && !sv->events.empty()) {
        ev[n++] = sv->events.front();
        sv->events.pop_front();
    }
    *n_events = n;
    return EIFP_OK;
}

eifp_status eifp_server_fields(eifp_server* sv, long long req_id, double* H, double* E, long long* step) {
    clear_error();
    if (!sv || !H || !E) return fail(EIFP_ERR_INVALID_ARG, "NULL argument");
    Req* r = nullptr;
    Group* g = nullptr;
    const void* src = nullptr;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(req_id);
        if (it == sv->reqs.end()) return fail(EIFP_ERR_INVALID_ARG, "unknown request %lld", req_id);
        r = it->second.get();
        if (sv->dry) return fail(EIFP_ERR_STATE, "dry-run server holds no fields");
        if (!r->finished && r->g) {
            // hold the group idle: no new chunk is launched while readers > 0; wait for
            // the one in flight (which may finish, or drop, this request)
            g = r->g;
            g->readers++;
            while (g->in_flight) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(50));
                lk.lock();
            }
            it = sv->reqs.find(req_id);
            r = it == sv->reqs.end() ? nullptr : it->second.get();
        }
        long long at = 0;
        if (r && r->kept) {
            src = r->state;
            at = r->done;
        } else if (r && !r->finished && r->has_snap) {
            src = r->snap;
            at = r->snap_step;
        }
        if (src && step) *step = at;
        if (!src) {
            if (g) {
                g->readers--;
                sv->cv_sched.notify_one();
            }
            return r ? fail(EIFP_ERR_STATE, "request %lld has no fields to copy yet", req_id)
                     : fail(EIFP_ERR_STATE, "request %lld finished without keeping its result", req_id);
        }
        r->readers++;
    }
    const long long n3 = 3LL * r->rq.nx * r->rq.ny * r->rq.nz;
    hipError_t e = hipSuccess;
    hipStream_t io = nullptr;
    e = hipStreamCreateWithFlags(&io, hipStreamNonBlocking);
    if (e == hipSuccess) {
        if (r->rq.prec == EIFP_FP64) {
            e = hipMemcpyAsync(H, src, n3 * 8, hipMemcpyDeviceToHost, io);
            if (e == hipSuccess) e = hipMemcpyAsync(E, (const char*)src + n3 * 8, n3 * 8, hipMemcpyDeviceToHost, io);
            if (e == hipSuccess) e = hipStreamSynchronize(io);
        } else {
            std::vector<float> tmp(2 * n3);
            e = hipMemcpyAsync(tmp.data(), src, 2 * n3 * 4, hipMemcpyDeviceToHost, io);
            if (e == hipSuccess) e = hipStreamSynchronize(io);
            if (e == hipSuccess)
                for (long long q = 0; q < n3; ++q) {
                    H[q] = tmp[q];
                    E[q] = tmp[n3 + q];
                }
        }
        (void)hipStreamDestroy(io);
    }
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        r->readers--;
        if (g) g->readers--;
        sv->cv_sched.notify_one();
    }
    if (e != hipSuccess) return fail(EIFP_ERR_DEVICE, "field copy failed: %s", hipGetErrorString(e));
    return EIFP_OK;
}

eifp_status eifp_server_release(eifp_server* sv, long long req_id) {
    clear_error();
    if (!sv) return fail(EIFP_ERR_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(req_id);
    if (it == sv->reqs.end()) return fail(EIFP_ERR_INVALID_ARG, "unknown request %lld", req_id);
    Req* r = it->second.get();
    if (!r->kept) return fail(EIFP_ERR_STATE, "request %lld is not a kept result", req_id);
    if (r->readers) return fail(EIFP_ERR_STATE, "request %lld is being copied", req_id);
    req_free_device(sv, r);
    sv->reqs.erase(it);
    sv->cv_sched.notify_one();
    return EIFP_OK;
}

eifp_status eifp_server_cancel(eifp_server* sv, long long req_id) {
    clear_error();
    if (!sv) return fail(EIFP_ERR_INVALID_ARG, "NULL server");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(req_id);
    if (it == sv->reqs.end()) return fail(EIFP_ERR_INVALID_ARG, "unknown request %lld", req_id);
    Req* r = it->second.get();
    if (r->finished) return fail(EIFP_ERR_STATE, "request %lld has finished (kept result: release it)", req_id);
    if (!r->cancel) {
        r->cancel = true;
        sv->cancel_asks++;
    }
    sv->cv_sched.notify_one();
    return EIFP_OK;
}

eifp_status eifp_server_stats(eifp_server* sv, eifp_server_stat_set* out) {
    clear_error();
    if (!sv || !out) return fail(EIFP_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    eifp_server_stat_set s{};
    s.submitted = sv->submitted;
    s.admitted = sv->admitted;
    s.completed = sv->completed;
    s.failed = sv->failed;
    s.queued = (long long)sv->pending.size();
    s.running = sv->running;
    s.peak_running = sv->peak_running;
    s.p50_s = pct(sv->lat, 0.50);
    s.p99_s = pct(sv->lat, 0.99);
    double sum = 0, mx = 0;
    for (double v : sv->lat) {
        sum += v;
        mx = std::max(mx, v);
    }
    s.mean_s = sv->lat.empty() ? 0.0 : sum / (double)sv->lat.size();
    s.max_s = mx;
    s.point_steps = sv->point_steps;
    s.wall_s = sv->first_arrive >= 0 && sv->completed ? sv->last_done - sv->first_arrive : 0.0;
    s.point_steps_per_s = s.wall_s > 0 ? s.point_steps / s.wall_s : 0.0;
    s.bytes_in_use = sv->used;
    s.peak_bytes = sv->peak;
    s.budget_bytes = sv->budget;
    s.chunks = sv->chunks;
    s.mean_batch = sv->chunks ? sv->batch_sum / (double)sv->chunks : 0.0;
    s.cancelled = sv->cancelled;
    *out = s;
    return EIFP_OK;
}

eifp_status eifp_server_drain(eifp_server* sv, int timeout_ms) {
    clear_error();
    if (!sv) return fail(EIFP_ERR_INVALID_ARG, "NULL server");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto idle = [&] { return sv->stop || (sv->pending.empty() && sv->running == 0); };
    sv->cv_sched.notify_one();
    if (timeout_ms >= 0) {
        if (!sv->cv_ev.wait_for(lk, std::chrono::milliseconds(timeout_ms), idle))
            return fail(EIFP_ERR_STATE, "drain timed out");
    } else {
        sv->cv_ev.wait(lk, idle);
    }
    return EIFP_OK;
}

eifp_status eifp_server_destroy(eifp_server* sv) {
    clear_error();
    if (!sv) return EIFP_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv_sched.notify_all();
        sv->cv_ev.notify_all();
    }
    if (sv->th.joinable()) sv->th.join();
    delete sv;
    return EIFP_OK;
}

}  // extern "C"
