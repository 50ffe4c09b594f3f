// Served form: a scheduler thread that keeps many runs of Alg. 1 resident on one device and
// advances them together (continuous batching). Each step:
//   1. drops cancelled requests and admits queued ones in arrival order while the slot and
//      device-byte limits hold (memory comes from a first-fit allocator over the caller's
//      arena);
//   2. copies the admitted graphs into their arena blocks and initialises their populations
//      (Alg. 1 phases 1-2), then runs one generation of every resident request in shared
//      multi-item launches, each request at its own generation and buffer parity;
//   3. ranks the requests that have completed their T generations (phase 4), copies their
//      fronts to the host and frees their blocks.
// A request's arithmetic depends only on its own graph, parameters and buffers, so its front
// is the same as in a run alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "host.hpp"
#include "run.hpp"

namespace hpm {
namespace {

using Clock = std::chrono::steady_clock;

// Steps in flight: the scheduler launches a step, then waits for the oldest of the others and
// settles it (fronts to the host, memory released), so host work of up to SERVER_DEPTH - 1
// steps' length can pass without the device waiting for the next launch.
constexpr int SERVER_DEPTH = 3;
constexpr size_t SERVER_STAGE_DEFAULT = (size_t)384 << 20;  // per flight
constexpr size_t SERVER_STAGE_MIN = 4096;  // smaller regions are not allocated (no staging)

// First-fit allocator over [0, size) with coalescing of free neighbours.
class Arena {
public:
    void reset(size_t size)
    {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

private:
    std::map<size_t, size_t> free_;  // offset -> length
};

struct Request {
    int64_t ticket = 0;
    HostGraph hg;
    hpmocd_params p{};
    size_t graph_bytes = 0, bytes = 0;
    int state = HPMOCD_REQ_QUEUED;
    int status = HPMOCD_OK;
    bool cancel = false;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int32_t steps = 0, max_mix = 0;
    size_t off = 0;               // arena block (resident requests)
    hpmocd_graph graph;           // device arrays inside the block
    Pop pop;
    int32_t gens_done = 0;
    bool fresh = false;           // admitted this step: needs initialisation
    hpmocd_front *front = nullptr;
};

}  // namespace
}  // namespace hpm

using namespace hpm;

// One launched step that has not been completed yet. Its host-side table copies, the host
// graphs of the requests it admitted, the fronts of the requests it finished and the memory
// of requests cancelled while it ran are settled only once its event has fired.
struct Flight {
    bool valid = false;
    hipEvent_t done = nullptr;
    Meta m_init, m_gen, m_final;
    std::vector<Request *> admitted, finals, released;
    std::vector<StagedFront> staged;  // per final: its front's copies (ks null: none enqueued)
};

struct hpmocd_server {
    hpmocd_server_config cfg{};
    char *arena = nullptr;        // caller's device memory
    size_t table_bytes = 0;       // SERVER_DEPTH sets of three item tables at the arena's start
    hipStream_t stream = nullptr;
    hipStream_t copy_stream = nullptr;  // front extraction beside the next step
    hipStream_t up_stream = nullptr;    // graph uploads beside the step in flight
    hipEvent_t up_done[SERVER_DEPTH] = {};
    int device = 0;
    Tuning tuning;
    Fork fork;  // side streams of the mutation classes
    Flight flight[SERVER_DEPTH];
    // page-locked staging of each flight's step, free again once that step has completed:
    // graph and table uploads, and the fronts of the requests it finishes
    Pinned up_stage[SERVER_DEPTH], front_stage[SERVER_DEPTH];
    Clock::time_point epoch;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    int broken = HPMOCD_OK;       // sticky HIP failure
    int64_t next_ticket = 1;
    std::map<int64_t, std::unique_ptr<Request>> reqs;
    std::deque<Request *> queue;
    std::vector<Request *> active;  // resident and still running; scheduler thread only
    Arena alloc;
    size_t used = 0;
    hpmocd_server_stats stats{};
    std::thread worker;

    double now() const { return std::chrono::duration<double>(Clock::now() - epoch).count(); }
    void run();
    int launch(Flight &f, int set, std::vector<Request *> &admitted);
    int complete(Flight &f);
    int run_fifo(Request *r);
    void release(Request *r, int status);  // caller holds mu
    void finish(Request *r, int status);   // caller holds mu
    ~hpmocd_server()
    {
        for (Flight &f : flight)
            if (f.done) (void)hipEventDestroy(f.done);
        if (copy_stream) (void)hipStreamDestroy(copy_stream);
        if (up_stream) (void)hipStreamDestroy(up_stream);
        for (hipEvent_t e : up_done)
            if (e) (void)hipEventDestroy(e);
        for (int i = 0; i < SERVER_DEPTH; ++i)
            for (Pinned *p : {&up_stage[i], &front_stage[i]})
                if (p->base) (void)hipHostFree(p->base);
    }
};

size_t hpmocd_server_arena_overhead(int32_t max_active)
{
    return 3 * SERVER_DEPTH * align_up(meta_bytes(std::max(1, max_active)));
}

void hpmocd_server::finish(Request *r, int st)
{
    r->status = st;
    r->state = HPMOCD_REQ_DONE;
    r->t_done = now();
    if (st == HPMOCD_ERR_CANCELLED)
        ++stats.cancelled;
    else if (st == HPMOCD_OK)
        ++stats.completed;
}

void hpmocd_server::release(Request *r, int st)
{
    alloc.release(r->off, r->bytes);
    used -= r->bytes;
    finish(r, st);
}

static void drop_host_graph(Request *r) { r->hg = HostGraph(); }

// FIFO baseline: the one resident request as a plain hipGraph-replayed run (synchronous).
int hpmocd_server::run_fifo(Request *r)
{
    up_stage[0].used = 0;  // the previous run drained the stream
    int rc = place_graph(r->hg, arena + r->off, stream, &r->graph, &up_stage[0]);
    if (rc) return rc;
    const hpmocd_graph *gp = &r->graph;
    rc = run_batch(&gp, 1, &r->p, arena + r->off + r->graph_bytes, r->bytes - r->graph_bytes,
                   stream, 0, nullptr, nullptr, nullptr, &r->front);
    if (rc) return rc;  // run_batch returns with the stream drained
    drop_host_graph(r);
    r->steps = 1;
    r->max_mix = 1;
    std::lock_guard<std::mutex> lk(mu);
    release(r, HPMOCD_OK);
    active.clear();
    cv_done.notify_all();
    return HPMOCD_OK;
}

// Launches one step over `active` (admitted requests included) into table set `set`, without
// waiting: copies the new graphs, initialises the new populations, advances every running
// request one generation and ranks those that reach T (which leave `active`).
int hpmocd_server::launch(Flight &f, int set, std::vector<Request *> &admitted)
{
    f.admitted = admitted;
    f.finals.clear();
    f.staged.clear();
    // this set's staging was last read by the step launched into it SERVER_DEPTH steps ago,
    // which has completed
    Pinned *stage = &up_stage[set];
    stage->used = 0;
    // stage every new graph on the host first, then issue all their copies: the stream
    // does not wait on host-side staging between copies
    std::vector<PendingCopy> copies;
    for (Request *r : admitted) {
        place_graph_deferred(r->hg, arena + r->off, &r->graph, stage, copies);
        r->pop.setup(&r->graph, r->p, arena + r->off + r->graph_bytes, tuning, 1, false);
        r->fresh = true;
    }
    // the copies run on their own stream beside the step still in flight (the blocks of newly
    // admitted requests are not used by it); this step's kernels wait for them
    if (!copies.empty()) {
        for (const PendingCopy &c : copies)
            HIP_TRY(hipMemcpyAsync(c.dst, c.src, c.bytes, hipMemcpyHostToDevice, up_stream));
        HIP_TRY(hipEventRecord(up_done[set], up_stream));
        HIP_TRY(hipStreamWaitEvent(stream, up_done[set], 0));
    }
    int64_t nodes = 0;
    for (Request *r : active) nodes += r->graph.n;
    std::vector<Item> init_items, gen_items, final_items;
    std::vector<Request *> gen_reqs;
    for (Request *r : active) {
        r->pop.shape(tuning, nodes);
        if (r->fresh) init_items.push_back(r->pop.item(ITEM_INIT));
        if (r->gens_done < r->p.generations) {
            gen_items.push_back(r->pop.item(r->pop.cur == 0 ? ITEM_PARITY0 : ITEM_PARITY1));
            gen_reqs.push_back(r);
        }
    }
    const size_t tb = align_up(meta_bytes(cfg.max_active));
    char *tables = arena + (size_t)set * 3 * tb;
    if (!init_items.empty()) {
        int rc = f.m_init.upload(init_items, tables, stream, stage);
        if (rc) return rc;
        HIP_TRY(launch_init_seq(f.m_init, stream, &fork));
    }
    if (!gen_items.empty()) {
        int rc = f.m_gen.upload(gen_items, tables + tb, stream, stage);
        if (rc) return rc;
        HIP_TRY(launch_generation(f.m_gen, stream, nullptr, &fork));
        for (Request *r : gen_reqs) {
            r->pop.cur = 1 - r->pop.cur;
            ++r->gens_done;
        }
    }
    for (Request *r : active) {
        r->fresh = false;
        ++r->steps;
        r->max_mix = std::max<int32_t>(r->max_mix, (int32_t)active.size());
        if (r->gens_done == r->p.generations) {
            final_items.push_back(r->pop.item(ITEM_PARITY0));
            f.finals.push_back(r);
        }
    }
    if (!final_items.empty()) {
        int rc = f.m_final.upload(final_items, tables + 2 * tb, stream, stage);
        if (rc) return rc;
        HIP_TRY(f.m_final.one(ONE_FINAL, stream));
        // the fronts' copies follow in the same stream, into page-locked memory, so that
        // no host round trip interrupts the stream (fronts that do not fit are copied when
        // the step completes)
        front_stage[set].used = 0;
        f.staged.assign(f.finals.size(), StagedFront{});
        for (size_t i = 0; i < f.finals.size(); ++i) {
            hipError_t e = hipSuccess;
            if (!enqueue_front(f.finals[i]->pop, stream, &front_stage[set], &f.staged[i], &e))
                f.staged[i] = StagedFront{};
            if (e != hipSuccess) return HPMOCD_ERR_HIP;
        }
        active.erase(std::remove_if(active.begin(), active.end(),
                                    [](Request *r) { return r->gens_done == r->p.generations; }),
                     active.end());
    }
    HIP_TRY(hipEventRecord(f.done, stream));
    f.valid = true;
    return HPMOCD_OK;
}

// Waits for a launched step, then settles it: host graphs of its admissions, fronts of its
// finished requests (extracted on the copy stream, beside the step launched after it),
// memory of its finished and cancelled requests.
int hpmocd_server::complete(Flight &f)
{
    HIP_TRY(hipEventSynchronize(f.done));
    for (Request *r : f.admitted) drop_host_graph(r);
    for (size_t i = 0; i < f.finals.size(); ++i) {
        Request *r = f.finals[i];
        const bool staged = i < f.staged.size() && f.staged[i].ks;
        int rc = staged ? front_from_staged(r->pop, f.staged[i], &r->front)
                        : extract_front(r->pop, copy_stream, &r->front);
        if (rc) return rc;
    }
    f.staged.clear();
    std::lock_guard<std::mutex> lk(mu);
    for (Request *r : f.finals) release(r, HPMOCD_OK);
    for (Request *r : f.released) release(r, HPMOCD_ERR_CANCELLED);
    if (!f.finals.empty() || !f.released.empty()) cv_done.notify_all();
    f.admitted.clear();
    f.finals.clear();
    f.released.clear();
    f.valid = false;
    return HPMOCD_OK;
}

void hpmocd_server::run()
{
    if (hipSetDevice(device) != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        broken = HPMOCD_ERR_HIP;
    }
    const bool fifo = (cfg.flags & HPMOCD_SERVER_FIFO) != 0;
    // flight[cur] takes the next launch; flight[(cur + 1) % SERVER_DEPTH] is the oldest in
    // flight, flight[(cur + SERVER_DEPTH - 1) % SERVER_DEPTH] the newest
    int cur = 0;
    auto any_in_flight = [&] {
        for (const Flight &f : flight)
            if (f.valid) return true;
        return false;
    };
    try {
        for (;;) {
            std::vector<Request *> admitted;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    return stop || !queue.empty() || !active.empty() || any_in_flight();
                });
                if (stop || broken) break;
                // resident requests cancelled since the last launch: the steps in flight may still
                // use their memory, so it is released when the newest of them completes
                Flight &newest = flight[(cur + SERVER_DEPTH - 1) % SERVER_DEPTH];
                for (Request *r : active)
                    if (r->cancel) {
                        if (newest.valid)
                            newest.released.push_back(r);
                        else
                            release(r, HPMOCD_ERR_CANCELLED);
                    }
                active.erase(std::remove_if(active.begin(), active.end(),
                                            [](Request *r) { return r->cancel; }),
                             active.end());
                cv_done.notify_all();
                while (!queue.empty() && (int32_t)active.size() < cfg.max_active &&
                       !(fifo && !active.empty())) {
                    Request *r = queue.front();
                    if (used + r->bytes > cfg.hbm_budget) break;  // arrival order: no overtaking
                    admitted.reserve(admitted.size() + 1);  // may throw: r is still queued
                    active.reserve(active.size() + 1);
                    size_t off = 0;
                    if (!alloc.alloc(r->bytes, &off)) break;
                    queue.pop_front();
                    r->off = off;
                    used += r->bytes;
                    r->state = HPMOCD_REQ_RUNNING;
                    r->t_admit = now();
                    active.push_back(r);
                    admitted.push_back(r);
                    ++stats.admitted;
                }
                stats.peak_active = std::max<int32_t>(stats.peak_active, (int32_t)active.size());
                stats.peak_bytes = std::max<int64_t>(stats.peak_bytes, (int64_t)used);
            }
            const double t0 = now();
            int rc = HPMOCD_OK;
            bool launched = false;
            if (!active.empty()) {
                rc = fifo ? run_fifo(active.front()) : launch(flight[cur], cur, admitted);
                launched = true;
            }
            Flight &oldest = flight[(cur + 1) % SERVER_DEPTH];
            if (!rc && oldest.valid) rc = complete(oldest);
            std::lock_guard<std::mutex> lk(mu);
            stats.busy_s += now() - t0;
            if (launched) ++stats.steps;
            if (rc) {
                broken = rc;
                break;
            }
            cur = (cur + 1) % SERVER_DEPTH;
        }
    } catch (...) {  // host resources ran out (an allocation): the server stops like on a failure
        std::lock_guard<std::mutex> lk(mu);
        if (!broken) broken = HPMOCD_ERR_NOMEM;
    }
    // shutdown or failure: settle what was launched, then nothing queued will run
    (void)hipStreamSynchronize(up_stream);
    (void)hipStreamSynchronize(stream);
    (void)hipStreamSynchronize(copy_stream);
    std::lock_guard<std::mutex> lk(mu);
    const int fail = broken ? broken : HPMOCD_ERR_CANCELLED;
    for (Flight &f : flight) {
        for (Request *r : f.finals)
            if (r->state != HPMOCD_REQ_DONE) release(r, fail);
        for (Request *r : f.released)
            if (r->state != HPMOCD_REQ_DONE) release(r, fail);
        f.admitted.clear();
        f.finals.clear();
        f.released.clear();
        f.valid = false;
    }
    for (Request *r : active)
        if (r->state != HPMOCD_REQ_DONE) release(r, fail);
    active.clear();
    for (Request *r : queue) finish(r, fail);
    queue.clear();
    cv_done.notify_all();
}

extern "C" {

int hpmocd_server_create(const hpmocd_server_config *cfg, void *d_arena, size_t arena_bytes,
                         void *stream, hpmocd_server **out)
{
    return c_guard([&]() -> int {
        if (!cfg || !d_arena || !out) return HPMOCD_ERR_ARG;
        if (cfg->max_active < 1 || cfg->max_active > HPMOCD_SERVER_MAX_ACTIVE) return HPMOCD_ERR_ARG;
        if (cfg->parents_per_child < 1 || cfg->parents_per_child > HPMOCD_MAX_PARENTS)
            return HPMOCD_ERR_ARG;
        if (cfg->flags & ~HPMOCD_SERVER_FIFO) return HPMOCD_ERR_ARG;
        const size_t over = hpmocd_server_arena_overhead(cfg->max_active);
        if (arena_bytes < over || arena_bytes - over < cfg->hbm_budget || cfg->hbm_budget == 0)
            return HPMOCD_ERR_WORKSPACE;
        if ((uintptr_t)d_arena % 256) return HPMOCD_ERR_ARG;
        hpmocd_server *s = new (std::nothrow) hpmocd_server;
        if (!s) return HPMOCD_ERR_NOMEM;
        s->cfg = *cfg;
        // resident requests share every launch, like a batch (FIFO runs go through run_batch alone)
        s->tuning = default_tuning(cfg->max_active);
        s->arena = (char *)d_arena;
        s->table_bytes = over;
        s->stream = (hipStream_t)stream;
        s->epoch = Clock::now();
        bool ok = hipGetDevice(&s->device) == hipSuccess && s->fork.init() == HPMOCD_OK;
        ok = ok && hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking) == hipSuccess;
        ok = ok && hipStreamCreateWithFlags(&s->up_stream, hipStreamNonBlocking) == hipSuccess;
        for (hipEvent_t &e : s->up_done)
            ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
        for (Flight &f : s->flight)
            ok = ok && hipEventCreateWithFlags(&f.done, hipEventDisableTiming) == hipSuccess;
        // staging per in-flight step: a third for the step's new graphs and tables, two thirds
        // for the fronts it finishes; copies that do not fit use pageable memory
        const size_t stage = cfg->host_stage_bytes ? cfg->host_stage_bytes : SERVER_STAGE_DEFAULT;
        for (int i = 0; i < SERVER_DEPTH; ++i)
            for (Pinned *p : {&s->up_stage[i], &s->front_stage[i]}) {
                const bool front = p == &s->front_stage[i];
                const size_t bytes = (front ? 2 * (stage / 3) : stage / 3) / 256 * 256;
                if (bytes < SERVER_STAGE_MIN) continue;
                p->size = bytes;
                ok = ok && hipHostMalloc((void **)&p->base, p->size, hipHostMallocDefault) == hipSuccess;
            }
        if (!ok) {
            delete s;
            return HPMOCD_ERR_HIP;
        }
        // block offsets are relative to the arena start; the tables come first
        s->alloc.reset(0);
        s->alloc.release(over, arena_bytes - over);
        try {
            s->worker = std::thread([s] { s->run(); });
        } catch (...) {
            delete s;
            return HPMOCD_ERR_NOMEM;
        }
        *out = s;
        return HPMOCD_OK;
    });
}

int hpmocd_server_submit(hpmocd_server *s, int32_t n, const int32_t *row_ptr, const int32_t *col,
                         const hpmocd_params *p, int64_t *ticket, size_t *device_bytes)
{
    return c_guard([&]() -> int {
        if (!s || !ticket) return HPMOCD_ERR_ARG;
        int rc = check_params(p);
        if (rc) return rc;
        if (p->parents_per_child != s->cfg.parents_per_child) return HPMOCD_ERR_ARG;
        std::unique_ptr<Request> r(new (std::nothrow) Request);
        if (!r) return HPMOCD_ERR_NOMEM;
        if ((rc = prepare_graph(n, row_ptr, col, &r->hg))) return rc;
        r->p = *p;
        r->graph_bytes = align_up(graph_block_bytes(r->hg.n, r->hg.m2, (int32_t)r->hg.small.size(),
                                                    (int32_t)r->hg.large.size()));
        if (s->cfg.flags & HPMOCD_SERVER_FIFO) {  // a plain run's workspace
            hpmocd_graph shape;
            shape.n = r->hg.n;
            shape.max_deg = r->hg.max_deg;
            const hpmocd_graph *gp = &shape;
            r->bytes = r->graph_bytes + align_up(batch_workspace(&gp, 1, p, false));
        } else {
            r->bytes = r->graph_bytes +
                       align_up(carve_run(nullptr, r->hg.n, p->pop_size, p->parents_per_child,
                                          r->hg.max_deg, s->tuning, false)
                                    .bytes);
        }
        if (r->bytes > s->cfg.hbm_budget) return HPMOCD_ERR_BUDGET;
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->broken) return s->broken;
        if (s->stop) return HPMOCD_ERR_CANCELLED;
        r->ticket = s->next_ticket++;
        r->t_submit = s->now();
        *ticket = r->ticket;
        if (device_bytes) *device_bytes = r->bytes;
        s->queue.push_back(r.get());
        s->reqs[r->ticket] = std::move(r);
        s->cv_work.notify_one();
        return HPMOCD_OK;
    });
}

int hpmocd_server_poll(hpmocd_server *s, int64_t ticket, int32_t *state)
{
    return c_guard([&]() -> int {
        if (!s || !state) return HPMOCD_ERR_ARG;
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return HPMOCD_ERR_ARG;
        *state = it->second->state;
        return HPMOCD_OK;
    });
}

int hpmocd_server_wait(hpmocd_server *s, int64_t ticket, double timeout_s, hpmocd_front **out,
                       hpmocd_request_info *info)
{
    return c_guard([&]() -> int {
        if (!s || !out) return HPMOCD_ERR_ARG;
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->reqs.find(ticket) == s->reqs.end()) return HPMOCD_ERR_ARG;
        // looked up again at every wake-up: another thread's wait on the same ticket may have
        // consumed it meanwhile
        auto settled = [&] {
            auto i = s->reqs.find(ticket);
            return i == s->reqs.end() || i->second->state == HPMOCD_REQ_DONE;
        };
        if (timeout_s < 0) {
            s->cv_done.wait(lk, settled);
        } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), settled)) {
            return HPMOCD_ERR_TIMEOUT;
        }
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return HPMOCD_ERR_ARG;
        Request *r = it->second.get();
        const int st = r->status;
        if (st == HPMOCD_OK) {
            *out = r->front;
            r->front = nullptr;
            if (info) {
                info->submit_s = r->t_submit;
                info->admit_s = r->t_admit;
                info->done_s = r->t_done;
                info->device_bytes = (int64_t)r->bytes;
                info->steps = r->steps;
                info->max_mix = r->max_mix;
            }
        }
        hpmocd_front_free(r->front);
        s->reqs.erase(it);
        return st;
    });
}

int hpmocd_server_cancel(hpmocd_server *s, int64_t ticket)
{
    return c_guard([&]() -> int {
        if (!s) return HPMOCD_ERR_ARG;
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end()) return HPMOCD_ERR_ARG;
        Request *r = it->second.get();
        if (r->state == HPMOCD_REQ_QUEUED) {
            s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
            s->finish(r, HPMOCD_ERR_CANCELLED);
            s->cv_done.notify_all();
        } else if (r->state == HPMOCD_REQ_RUNNING) {
            r->cancel = true;
            s->cv_work.notify_one();
        }
        return HPMOCD_OK;
    });
}

int hpmocd_server_stats_get(hpmocd_server *s, hpmocd_server_stats *out)
{
    return c_guard([&]() -> int {
        if (!s || !out) return HPMOCD_ERR_ARG;
        std::lock_guard<std::mutex> lk(s->mu);
        *out = s->stats;
        return HPMOCD_OK;
    });
}

void hpmocd_server_destroy(hpmocd_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto &kv : s->reqs) hpmocd_front_free(kv.second->front);
    delete s;
}

}  // extern "C"
