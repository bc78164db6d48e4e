// server.hip -- continuous-batching walk server.
//
// Walks are independent (the FN-Multi paragraph of Section 3.4 of the paper
// runs them in rounds to bound memory), so requests can be admitted and cut
// into chunks freely without changing any result.  A scheduler thread:
//   - admits queued requests into the caller's device pool as space frees
//     up (first fit; a request that does not fit may be passed by later,
//     smaller ones until it has waited long enough, then it blocks the line);
//   - cuts admitted requests into chunks of walks and, each tick, writes a
//     table of chunks taken round-robin from all running requests;
//   - replays one captured hipGraph per tick: copy of the table to the device
//     and one launch of the persistent kernel over all chunks of the table;
//   - keeps two ticks in flight so the next table is built while the GPU
//     runs the current one, and stamps completion from tick events.
// Chunk c of a request covering its walks [a, a+k) is the job with walk ids
// a.., so every walk uses the same random stream as in a single n2v_walk.
#include <time.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "prims.hpp"
#include "walk.hpp"

namespace n2v {

namespace {

uint64_t now_ns()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

enum ReqState { QUEUED, RUNNING, DONE, FAILED };

struct Req {
    uint64_t ticket;
    std::vector<uint32_t> starts;  // host copy of the start ids until admission
    uint32_t n, L, A_ret, A_out, approx_t;
    uint64_t seed;
    uint64_t submit_ns = 0, start_ns = 0, done_ns = 0;
    size_t off = 0, bytes = 0;  // pool allocation
    uint32_t next = 0;          // first walk not yet scheduled
    uint32_t done_walks = 0;
    ReqState state = QUEUED;
    int err = N2V_OK;
    uint32_t *d_starts = nullptr, *d_out = nullptr;
};

// First-fit allocator over [0, size) in 256-byte units.
struct Pool {
    std::map<size_t, size_t> free_;  // offset -> length
    size_t size = 0;
    void init(size_t s)
    {
        size = s & ~(size_t)255;
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(size_t bytes, size_t *off)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t at = it->first + bytes;
                free_.erase(it);
                if (rest) free_[at] = rest;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = (bytes + 255) & ~(size_t)255;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Tick {
    bool busy = false;
    uint64_t seq = 0;            // launch order
    TableHdr *host = nullptr;    // pinned
    TableHdr *dev = nullptr;     // in the pool's reserved head
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    std::vector<std::pair<uint64_t, uint32_t>> chunks;  // (ticket, walks)
};

constexpr uint64_t STARVE_NS = 200ull * 1000 * 1000;
constexpr size_t RING_BYTES = 64ull << 20;  // pinned staging for start ids

}  // namespace

}  // namespace n2v

using namespace n2v;

struct n2v_server {
    const n2v_graph *g;
    Exec E;
    hipStream_t st;
    bool own_stream;
    n2v_server_opts o;
    char *pool_base;
    Pool pool;
    Tick ticks[2];
    int next_tick = 0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;
    std::map<uint64_t, Req> reqs;
    std::vector<uint64_t> running;  // admission order
    uint64_t next_ticket = 1;
    bool stop = false;
    int fatal = N2V_OK;
    std::thread th;
    // Pinned staging ring for start ids.  Space is handed out in admission
    // order; a piece is reused once the first tick launched after its copy
    // has retired (the copy precedes that tick on the stream).
    char *ring = nullptr;
    size_t ring_head = 0, ring_used = 0;
    std::deque<std::pair<size_t, uint64_t>> ring_live;  // (bytes incl. wrap padding, tick seq)
    uint64_t tick_seq = 0;                              // seq of the next tick to launch
    uint64_t retired_seq = 0;                           // every tick with seq < this has retired

    bool ring_alloc(size_t n, size_t *off)
    {
        n = (n + 255) & ~(size_t)255;
        if (n > RING_BYTES) return false;
        size_t at = ring_head, waste = 0;
        if (at + n > RING_BYTES) {
            waste = RING_BYTES - at;
            at = 0;
        }
        if (ring_used + waste + n > RING_BYTES) return false;
        ring_used += waste + n;
        ring_live.push_back({waste + n, tick_seq});
        ring_head = at + n;
        *off = at;
        return true;
    }

    void ring_retire()
    {
        while (!ring_live.empty() && ring_live.front().second < retired_seq) {
            ring_used -= ring_live.front().first;
            ring_live.pop_front();
        }
        if (ring_live.empty()) ring_head = ring_used = 0;
    }

    int capture(Tick &t)
    {
        N2V_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        hipError_t e1 = hipMemcpyAsync(t.dev, t.host, sizeof(TableHdr), hipMemcpyHostToDevice, st);
        int rc = launch_job_table(E, t.dev, full_grid_blocks(g->device), st);
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(st, &graph);
        if (e1 != hipSuccess) return hip_fail(e1, "hipMemcpyAsync (capture)");
        if (rc) return rc;
        if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
        hipError_t e3 = hipGraphInstantiate(&t.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e3 != hipSuccess) return hip_fail(e3, "hipGraphInstantiate");
        return N2V_OK;
    }

    // Called with mu held.
    void admit()
    {
        const uint64_t now = now_ns();
        for (auto it = queue.begin(); it != queue.end();) {
            Req &r = reqs[*it];
            size_t off;
            if (pool.alloc(r.bytes, &off)) {
                size_t roff = 0;
                const bool staged = ring_alloc((size_t)r.n * 4, &roff);
                if (!staged && (size_t)r.n * 4 <= RING_BYTES) {  // staging full: admit later, in order
                    pool.release(off, r.bytes);
                    break;
                }
                r.off = off;
                r.d_starts = (uint32_t *)(pool_base + off);
                r.d_out = (uint32_t *)(pool_base + off + (((size_t)r.n * 4 + 255) & ~(size_t)255));
                hipError_t e;
                if (staged) {
                    memcpy(ring + roff, r.starts.data(), (size_t)r.n * 4);
                    e = hipMemcpyAsync(r.d_starts, ring + roff, (size_t)r.n * 4, hipMemcpyHostToDevice, st);
                } else {
                    e = hipMemcpyAsync(r.d_starts, r.starts.data(), (size_t)r.n * 4, hipMemcpyHostToDevice, st);
                    (void)hipStreamSynchronize(st);
                }
                std::vector<uint32_t>().swap(r.starts);
                if (e != hipSuccess) {
                    r.state = FAILED;
                    r.err = hip_fail(e, "hipMemcpyAsync (starts)");
                    r.done_ns = now_ns();
                } else {
                    r.state = RUNNING;
                    r.start_ns = now;
                    running.push_back(r.ticket);
                }
                it = queue.erase(it);
                continue;
            }
            // the oldest waiting request stops later ones once it has starved
            if (it == queue.begin() && now - r.submit_ns > STARVE_NS) break;
            ++it;
        }
    }

    // Called with mu held: fills tick t with chunks; returns the walk count.
    // Requests with the least remaining work go first (shortest remaining
    // processing first keeps small requests' latency low); a tick holds at
    // most tick_walks walks so that newly admitted requests wait at most
    // about one tick.
    uint32_t build(Tick &t)
    {
        TableHdr *h = t.host;
        t.chunks.clear();
        uint32_t nj = 0, total = 0;
        const uint32_t maxj = std::min<uint32_t>(o.max_inflight, MAX_TABLE_JOBS);
        std::vector<std::pair<uint32_t, uint64_t>> order;  // (remaining walks, ticket)
        for (uint64_t tk : running) {
            const Req &r = reqs[tk];
            if (r.next < r.n) order.push_back({r.n - r.next, tk});
        }
        std::sort(order.begin(), order.end());
        for (auto &e : order) {
            Req &r = reqs[e.second];
            while (r.next < r.n && nj < maxj && total < o.tick_walks) {
                const uint32_t k = std::min(std::min(o.chunk_walks, r.n - r.next), o.tick_walks - total);
                JobRec &jr = h->jobs[nj];
                jr.c.out = r.d_out + (uint64_t)r.next * (r.L + 1);
                jr.c.cnt = nullptr;
                jr.c.checksum = nullptr;
                jr.c.wbase = r.next;
                jr.c.L = r.L;
                jr.c.k0 = (uint32_t)r.seed;
                jr.c.k1 = (uint32_t)(r.seed >> 32);
                jr.c.A_ret = r.A_ret;
                jr.c.A_out = r.A_out;
                jr.c.approx_t = r.approx_t;
                jr.starts = r.d_starts + r.next;
                jr.n = k;
                h->jstart[nj] = total;
                total += k;
                ++nj;
                r.next += k;
                t.chunks.push_back({r.ticket, k});
            }
            if (nj >= maxj || total >= o.tick_walks) break;
        }
        h->njobs = nj;
        h->total = total;
        h->cursor = 0;
        h->jstart[nj] = total;
        return total;
    }

    // Called with mu held.
    void retire(Tick &t, int status)
    {
        const uint64_t now = now_ns();
        if (t.seq + 1 > retired_seq) retired_seq = t.seq + 1;
        ring_retire();
        for (auto &c : t.chunks) {
            auto it = reqs.find(c.first);
            if (it == reqs.end()) continue;
            Req &r = it->second;
            if (status != N2V_OK && r.state == RUNNING) {
                r.state = FAILED;
                r.err = status;
            }
            r.done_walks += c.second;
            if (r.state == RUNNING && r.done_walks == r.n) {
                r.state = DONE;
                r.done_ns = now;
            }
            if (r.state != RUNNING) running.erase(std::remove(running.begin(), running.end(), r.ticket), running.end());
        }
        t.chunks.clear();
        t.busy = false;
    }

    void loop()
    {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            // retire finished ticks
            for (Tick &t : ticks) {
                if (!t.busy) continue;
                hipError_t q = hipEventQuery(t.done);
                if (q == hipSuccess) retire(t, N2V_OK);
                else if (q != hipErrorNotReady) retire(t, hip_fail(q, "tick"));
            }
            admit();
            Tick &t = ticks[next_tick];
            bool launched = false;
            if (!t.busy && fatal == N2V_OK) {
                if (build(t) > 0) {
                    t.seq = tick_seq++;
                    hipError_t e = hipGraphLaunch(t.exec, st);
                    if (e == hipSuccess) e = hipEventRecord(t.done, st);
                    t.busy = true;
                    if (e != hipSuccess) retire(t, hip_fail(e, "hipGraphLaunch"));
                    next_tick ^= 1;
                    launched = true;
                }
            }
            const bool any_busy = ticks[0].busy || ticks[1].busy;
            if (stop && !any_busy) break;
            if (launched) continue;
            // submissions and releases wake the loop early
            cv.wait_for(lk, any_busy ? std::chrono::microseconds(100) : std::chrono::milliseconds(5));
        }
    }
};

extern "C" void n2v_server_opts_default(n2v_server_opts *o)
{
    if (!o) return;
    o->max_queue = 4096;
    o->chunk_walks = 65536;
    o->max_inflight = 64;
    o->tick_walks = 1u << 19;
}

extern "C" int n2v_server_create(const n2v_graph *g, void *pool, size_t pool_bytes, const n2v_server_opts *opts,
                                 void *stream, n2v_server **out)
{
    if (!g || !pool || !out) return set_error(N2V_EINVAL, "n2v_server_create: null argument");
    if (((uintptr_t)pool & 255) != 0) return set_error(N2V_EINVAL, "n2v_server_create: pool not 256-byte aligned");
    const size_t reserve = 2 * ((sizeof(TableHdr) + 255) & ~(size_t)255);
    if (pool_bytes < reserve + 4096) return set_error(N2V_ENOMEM, "n2v_server_create: pool too small");
    n2v_server *s = new n2v_server();
    s->g = g;
    // the graph's sketch memory and rows stay fixed while a server replays
    // ticks captured with them (attaching returns N2V_EINVAL meanwhile)
    __atomic_fetch_add(&const_cast<n2v_graph *>(g)->servers, 1, __ATOMIC_ACQ_REL);
    n2v_server_opts_default(&s->o);
    if (opts) s->o = *opts;
    if (s->o.chunk_walks < 1) s->o.chunk_walks = 1;
    if (s->o.max_inflight < 1) s->o.max_inflight = 1;
    if (s->o.tick_walks < 1) s->o.tick_walks = 1;
    n2v_exec_opts eo;
    n2v_exec_opts_default(g, &eo);
    make_exec(g, eo, &s->E);
    s->own_stream = stream == nullptr;
    if (s->own_stream) {
        hipError_t e = hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking);
        if (e != hipSuccess) {
            __atomic_fetch_sub(&const_cast<n2v_graph *>(g)->servers, 1, __ATOMIC_ACQ_REL);
            delete s;
            return hip_fail(e, "hipStreamCreateWithFlags");
        }
    } else {
        s->st = (hipStream_t)stream;
    }
    s->pool_base = (char *)pool + reserve;
    s->pool.init(pool_bytes - reserve);
    for (int i = 0; i < 2; ++i) {
        Tick &t = s->ticks[i];
        t.dev = (TableHdr *)((char *)pool + i * (reserve / 2));
        void *h = nullptr;
        hipError_t e = hipHostMalloc(&h, sizeof(TableHdr), hipHostMallocDefault);
        if (e != hipSuccess) {
            n2v_server_destroy(s);
            return hip_fail(e, "hipHostMalloc");
        }
        t.host = (TableHdr *)h;
        memset(t.host, 0, sizeof(TableHdr));
        e = hipEventCreateWithFlags(&t.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            n2v_server_destroy(s);
            return hip_fail(e, "hipEventCreate");
        }
        int rc = s->capture(t);
        if (rc) {
            n2v_server_destroy(s);
            return rc;
        }
    }
    {
        void *h = nullptr;
        hipError_t e = hipHostMalloc(&h, RING_BYTES, hipHostMallocDefault);
        if (e != hipSuccess) {
            n2v_server_destroy(s);
            return hip_fail(e, "hipHostMalloc (staging ring)");
        }
        s->ring = (char *)h;
    }
    s->th = std::thread([s] { s->loop(); });
    *out = s;
    return N2V_OK;
}

extern "C" int n2v_server_destroy(n2v_server *s)
{
    if (!s) return N2V_OK;
    if (s->th.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
            s->queue.clear();
            // nothing new is scheduled once stopping: drop unscheduled work
            for (auto &kv : s->reqs) kv.second.next = kv.second.n;
        }
        s->cv.notify_all();
        s->th.join();
    }
    (void)hipStreamSynchronize(s->st);
    if (s->ring) (void)hipHostFree(s->ring);
    for (Tick &t : s->ticks) {
        if (t.done) (void)hipEventSynchronize(t.done);
        if (t.exec) (void)hipGraphExecDestroy(t.exec);
        if (t.done) (void)hipEventDestroy(t.done);
        if (t.host) (void)hipHostFree(t.host);
    }
    if (s->own_stream) (void)hipStreamDestroy(s->st);
    __atomic_fetch_sub(&const_cast<n2v_graph *>(s->g)->servers, 1, __ATOMIC_ACQ_REL);
    delete s;
    return N2V_OK;
}

extern "C" int n2v_submit(n2v_server *s, const n2v_request *r, uint64_t *ticket)
{
    if (!s || !r || !ticket) return set_error(N2V_EINVAL, "n2v_submit: null argument");
    if (r->n_starts == 0 || !r->host_starts) return set_error(N2V_EINVAL, "n2v_submit: empty request");
    if (r->L < 1) return set_error(N2V_EINVAL, "n2v_submit: L must be >= 1");
    uint32_t A_ret, A_out;
    if (walk_multipliers(r->p, r->q, &A_ret, &A_out)) return set_error(N2V_EINVAL, "n2v_submit: bad p or q");
    for (uint32_t i = 0; i < r->n_starts; ++i)
        if (r->host_starts[i] >= s->g->dg.n) return set_error(N2V_EINVAL, "n2v_submit: start id %u >= n", r->host_starts[i]);
    const size_t bytes = (((size_t)r->n_starts * 4 + 255) & ~(size_t)255) + (size_t)r->n_starts * (r->L + 1) * 4;
    if (((bytes + 255) & ~(size_t)255) > s->pool.size)
        return set_error(N2V_ETOOBIG, "n2v_submit: request needs %zu bytes, pool has %zu", bytes, s->pool.size);
    Req q;
    q.starts.assign(r->host_starts, r->host_starts + r->n_starts);
    q.n = r->n_starts;
    q.L = r->L;
    q.A_ret = A_ret;
    q.A_out = A_out;
    q.approx_t = r->approx_t;
    q.seed = r->seed;
    q.bytes = bytes;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop || s->queue.size() >= s->o.max_queue) {
            if (s->stop) return set_error(N2V_EINVAL, "n2v_submit: server is stopping");
            return set_error(N2V_EAGAIN, "n2v_submit: queue full");
        }
        q.ticket = s->next_ticket++;
        q.submit_ns = now_ns();
        *ticket = q.ticket;
        s->queue.push_back(q.ticket);
        s->reqs.emplace(q.ticket, std::move(q));
    }
    s->cv.notify_all();
    return N2V_OK;
}

extern "C" int n2v_poll(n2v_server *s, uint64_t ticket, n2v_result *res)
{
    if (!s) return set_error(N2V_EINVAL, "n2v_poll: null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return set_error(N2V_ENOTFOUND, "n2v_poll: unknown ticket %llu", (unsigned long long)ticket);
    Req &r = it->second;
    if (r.state == FAILED) return set_error(r.err ? r.err : N2V_EDEVICE, "n2v_poll: request failed");
    if (r.state != DONE) return N2V_PENDING;
    if (res) {
        res->d_out = r.d_out;
        res->n_starts = r.n;
        res->L = r.L;
        res->submit_ns = r.submit_ns;
        res->start_ns = r.start_ns;
        res->done_ns = r.done_ns;
    }
    return N2V_OK;
}

extern "C" int n2v_release(n2v_server *s, uint64_t ticket)
{
    if (!s) return set_error(N2V_EINVAL, "n2v_release: null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(ticket);
        if (it == s->reqs.end())
            return set_error(N2V_ENOTFOUND, "n2v_release: unknown ticket %llu", (unsigned long long)ticket);
        Req &r = it->second;
        if (r.state == QUEUED || r.state == RUNNING)
            return set_error(N2V_EINVAL, "n2v_release: request %llu is not complete", (unsigned long long)ticket);
        if (r.d_starts) s->pool.release(r.off, r.bytes);
        s->reqs.erase(it);
    }
    s->cv.notify_all();
    return N2V_OK;
}

extern "C" int n2v_server_stats(n2v_server *s, uint32_t *queued, uint32_t *running, uint32_t *done)
{
    if (!s) return set_error(N2V_EINVAL, "n2v_server_stats: null server");
    std::lock_guard<std::mutex> lk(s->mu);
    uint32_t q = 0, r = 0, d = 0;
    for (auto &kv : s->reqs) {
        if (kv.second.state == QUEUED) ++q;
        else if (kv.second.state == RUNNING) ++r;
        else ++d;
    }
    if (queued) *queued = q;
    if (running) *running = r;
    if (done) *done = d;
    return N2V_OK;
}
