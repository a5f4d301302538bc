// hsd_server.hip -- serving loop: continuous batching of distance requests.
//
// Requests are copied at submit and queued (FIFO).  A scheduler thread
// admits queued requests into free slots while the sum of admitted device
// footprints stays within the server budget; every slot owns a HIP stream
// and its scratch buffers, so the work of admitted requests overlaps on the
// device.  An admitted request's direct sum is enqueued in chunks of
// directions (a bounded number in flight per slot), so newly admitted
// requests start within one chunk of the others and a cancelled request
// stops between chunks.  After the last chunk the slot enqueues the
// finalize, the two-level reduction and an 8-byte readback, and the
// scheduler completes the ticket when the slot's completion event fires.
//
// Per-request arithmetic does not depend on the mix: triangle splits and
// lane layout are functions of the request alone, chunk boundaries only
// select which lanes a launch runs, and every reduction has a fixed order,
// so a result is bitwise the same alone or in any mix.
//
// The scheduling core talks to an Executor.  The device executor runs the
// kernels; a fake executor (CPU only, simulated durations) lets the queue,
// admission, cancellation and failure paths be tested without a GPU.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <functional>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hsd_internal.hpp"

namespace hsd {

using Clock = std::chrono::steady_clock;

struct Job {
    uint64_t ticket = 0;
    int64_t tag = 0;
    std::vector<double> v1, v2;
    std::vector<int32_t> t1, t2;
    bool has_nu = false;
    hsd_rule *rule = nullptr;
    hsd_params params{};
    int64_t footprint = 0;
    // progress
    int slot = -1;
    int64_t next_chunk = 0, n_chunks = 0;
    int inflight = 0;
    bool finalizing = false, cancel = false;
    hsd_status fail = HSD_OK;     // executor error that stopped the request
    std::string errmsg;           // message of the failing executor call
    hsd_status status = HSD_PENDING;
    hsd_result result{};
    hsd_request_times times{};
};

// ---------------------------------------------------------------------------
// executors
// ---------------------------------------------------------------------------
struct Executor {
    virtual ~Executor() = default;
    virtual int slots() const = 0;
    virtual int64_t footprint(const Job &j) = 0;
    virtual hsd_status start(int s, Job &j) = 0;            // upload / plan; sets n_chunks
    virtual hsd_status enqueue_chunk(int s, Job &j) = 0;    // next chunk (j.next_chunk)
    virtual int chunks_done(int s, Job &j) = 0;             // completed chunks so far
    virtual hsd_status enqueue_finish(int s, Job &j) = 0;   // finalize + reduce + readback
    virtual bool finished(int s, Job &j) = 0;               // readback complete
    virtual hsd_status collect(int s, Job &j) = 0;          // fill j.result
    virtual void release(int s, Job &j) = 0;
};

struct DeviceSlot {
    hipStream_t stream = nullptr;
    Scratch partial, nodebuf, redbuf;
    NufftScratch nufft;
    hsd_mesh *mu = nullptr, *nu = nullptr;
    std::vector<hipEvent_t> chunk_ev;
    hipEvent_t ev_begin = nullptr, ev_done = nullptr;
    double *host_result = nullptr;
    int K = 1;
    int64_t chunk_dirs = 0;
};


struct DeviceExecutor : Executor {
    hsd_ctx *ctx;
    int64_t chunk_pairs;
    std::vector<DeviceSlot> sl;

    DeviceExecutor(hsd_ctx *c, int n, int64_t cp) : ctx(c), chunk_pairs(cp), sl(n)
    {
        for (auto &s : sl) {
            (void)hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
            (void)hipEventCreateWithFlags(&s.ev_begin, hipEventDefault);
            (void)hipEventCreateWithFlags(&s.ev_done, hipEventDefault);   // timed against ev_begin
            (void)hipHostMalloc((void **)&s.host_result, 64, hipHostMallocDefault);
        }
    }
    ~DeviceExecutor() override
    {
        (void)hipSetDevice(ctx->device);
        for (auto &s : sl) {
            (void)hipStreamSynchronize(s.stream);
            for (auto e : s.chunk_ev) (void)hipEventDestroy(e);
            if (s.mu) hsd_mesh_destroy(s.mu);
            if (s.nu) hsd_mesh_destroy(s.nu);
            s.partial.buf.release();
            s.nodebuf.buf.release();
            s.redbuf.buf.release();
            (void)hipEventDestroy(s.ev_begin);
            (void)hipEventDestroy(s.ev_done);
            (void)hipHostFree(s.host_result);
            (void)hipStreamDestroy(s.stream);
        }
    }
    int slots() const override { return (int)sl.size(); }

    static int64_t n_dirs(const hsd_rule *r) { return r->kind == HSD_RULE_SPHERICAL_PRODUCT ? r->n_dir : r->n_nodes; }
    static int64_t nodes_per_dir(const hsd_rule *r) { return r->kind == HSD_RULE_SPHERICAL_PRODUCT ? r->n_rad : 1; }

    int k_of(const Job &j) const
    {
        const int64_t nt = (int64_t)(j.t1.size() + j.t2.size()) / 3;
        return j.rule->kind == HSD_RULE_SPHERICAL_PRODUCT
                   ? choose_k_splits_sp(j.rule, nt, j.params.form, ctx->num_cu, j.params.k_splits)
                   : choose_k_splits_gen(j.rule->n_nodes, nt, ctx->num_cu, j.params.k_splits);
    }

    int64_t footprint(const Job &j) override
    {
        const int64_t nt = (int64_t)(j.t1.size() + j.t2.size()) / 3;
        const int64_t nv = (int64_t)(j.v1.size() + j.v2.size()) / 3;
        const int64_t N = j.rule->n_nodes;
        const int64_t mesh = nt * (int64_t)(sizeof(TriRec) + 24) + nv * 28 + 8;
        return mesh + (int64_t)k_of(j) * N * 16 + (N / 256 + 2) * 8;
    }

    hsd_status start(int s, Job &j) override
    {
        DeviceSlot &d = sl[s];
        hsd_status st;
        HSD_HIP_TRY(hipSetDevice(ctx->device));
        if ((st = create_mesh_on(ctx, d.stream, j.v1.data(), (int64_t)j.v1.size() / 3, j.t1.data(),
                                 (int64_t)j.t1.size() / 3, HSD_MEM_HOST, &d.mu)) != HSD_OK)
            return st;
        if (j.has_nu && (st = create_mesh_on(ctx, d.stream, j.v2.data(), (int64_t)j.v2.size() / 3, j.t2.data(),
                                             (int64_t)j.t2.size() / 3, HSD_MEM_HOST, &d.nu)) != HSD_OK)
            return st;
        const double *w = nullptr, *nuv = nullptr;
        if ((st = rule_tables(j.rule, &j.params, d.stream, &w, &nuv)) != HSD_OK) return st;
        d.K = k_of(j);
        const int64_t N = j.rule->n_nodes;
        if ((st = d.partial.ensure(ctx, (size_t)d.K * N * sizeof(double2))) != HSD_OK) return st;
        const int64_t pairs_per_dir = (int64_t)(j.t1.size() + j.t2.size()) / 3 * nodes_per_dir(j.rule);
        int64_t cd = std::max<int64_t>(1, chunk_pairs / std::max<int64_t>(pairs_per_dir, 1));
        if (j.params.method == HSD_METHOD_NUFFT3) cd = n_dirs(j.rule);   // one chunk
        d.chunk_dirs = std::min<int64_t>(cd, n_dirs(j.rule));
        j.n_chunks = (n_dirs(j.rule) + d.chunk_dirs - 1) / d.chunk_dirs;
        for (auto e : d.chunk_ev) (void)hipEventDestroy(e);
        d.chunk_ev.assign((size_t)j.n_chunks, nullptr);
        for (auto &e : d.chunk_ev) HSD_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HSD_HIP_TRY(hipEventRecord(d.ev_begin, d.stream));
        return HSD_OK;
    }

    hsd_status enqueue_chunk(int s, Job &j) override
    {
        DeviceSlot &d = sl[s];
        HSD_HIP_TRY(hipSetDevice(ctx->device));
        const int64_t c = j.next_chunk;
        const int64_t d0 = c * d.chunk_dirs;
        const int64_t dc = std::min<int64_t>(d.chunk_dirs, n_dirs(j.rule) - d0);
        MeshPair mp;
        mp.A = d.mu->tris.as<const TriRec>();
        mp.nA = d.mu->nt;
        if (d.nu) { mp.B = d.nu->tris.as<const TriRec>(); mp.nB = d.nu->nt; }
        hsd_status st = HSD_OK;
        const int64_t N = j.rule->n_nodes;
        if (j.params.method == HSD_METHOD_NUFFT3) {
            double pairs = 0;
            st = nufft_transform_rule(ctx, d.stream, d.nufft, d.mu, d.nu, j.rule, &j.params, d.partial.buf.as<double2>(),
                                      &pairs);
            j.result.pairs = pairs;
        } else if (mp.nA + mp.nB == 0) {
            HSD_HIP_TRY(hipMemsetAsync(d.partial.buf.ptr, 0, (size_t)N * sizeof(double2), d.stream));
        } else if (j.rule->kind == HSD_RULE_SPHERICAL_PRODUCT) {
            st = launch_direct_sp_range(d.stream, mp, j.rule, j.params.form, j.params.taylor_tau, d.K, d0, dc,
                                        d.partial.buf.as<double2>());
        } else {
            st = launch_direct_gen_range(d.stream, mp, j.rule->d_nodes.as<const double>(), N, j.params.form,
                                         j.params.taylor_tau, d.K, d0, dc, d.partial.buf.as<double2>());
        }
        if (st != HSD_OK) return st;
        HSD_HIP_TRY(hipEventRecord(d.chunk_ev[(size_t)c], d.stream));
        return HSD_OK;
    }

    // hipEventQuery reports hipErrorNotReady through the thread's last-error
    // state as well; clear it so the next launch check does not see it.
    static bool event_done(hipEvent_t e)
    {
        const hipError_t r = hipEventQuery(e);
        if (r == hipErrorNotReady) (void)hipGetLastError();
        return r == hipSuccess;
    }

    int chunks_done(int s, Job &j) override
    {
        DeviceSlot &d = sl[s];
        int n = 0;
        for (int64_t c = 0; c < j.next_chunk; ++c)
            if (event_done(d.chunk_ev[(size_t)c])) ++n;
        return n;
    }

    hsd_status enqueue_finish(int s, Job &j) override
    {
        DeviceSlot &d = sl[s];
        HSD_HIP_TRY(hipSetDevice(ctx->device));
        const double *w = nullptr, *nuv = nullptr;
        hsd_status st;
        if ((st = rule_tables(j.rule, &j.params, d.stream, &w, &nuv)) != HSD_OK) return st;
        const int64_t N = j.rule->n_nodes;
        const int64_t nb = finalize_blocks(N);
        if ((st = d.redbuf.ensure(ctx, (size_t)(nb + 1) * sizeof(double))) != HSD_OK) return st;
        const int K = j.params.method == HSD_METHOD_NUFFT3 ? 1 : d.K;
        const bool empty = j.params.method != HSD_METHOD_NUFFT3 && d.mu->nt + (d.nu ? d.nu->nt : 0) == 0;
        if ((st = launch_finalize(d.stream, j.rule, w, nuv, d.partial.buf.as<const double2>(), empty ? 1 : K, N,
                                  !j.has_nu, nullptr, d.redbuf.buf.as<double>(), nb)) != HSD_OK)
            return st;
        double *res = d.redbuf.buf.as<double>() + nb;
        if ((st = launch_final_reduce(d.stream, d.redbuf.buf.as<double>(), nb, res)) != HSD_OK) return st;
        HSD_HIP_TRY(hipMemcpyAsync(d.host_result, res, sizeof(double), hipMemcpyDeviceToHost, d.stream));
        HSD_HIP_TRY(hipEventRecord(d.ev_done, d.stream));
        return HSD_OK;
    }

    bool finished(int s, Job &) override { return event_done(sl[s].ev_done); }

    hsd_status collect(int s, Job &j) override
    {
        DeviceSlot &d = sl[s];
        float ms = 0.0f;
        HSD_HIP_TRY(hipEventElapsedTime(&ms, d.ev_begin, d.ev_done));
        j.result.d2 = d.host_result[0];
        j.result.device_ms = (double)ms;
        if (j.params.method != HSD_METHOD_NUFFT3)
            j.result.pairs = (double)(d.mu->nt + (d.nu ? d.nu->nt : 0)) * (double)j.rule->n_nodes;
        j.result.rel_err_stated = stated_rel_err(&j.params, d.mu->nt);
        return HSD_OK;
    }

    void release(int s, Job &) override
    {
        DeviceSlot &d = sl[s];
        (void)hipStreamSynchronize(d.stream);
        if (d.mu) { hsd_mesh_destroy(d.mu); d.mu = nullptr; }
        if (d.nu) { hsd_mesh_destroy(d.nu); d.nu = nullptr; }
    }
};

// CPU-only executor for tests of the scheduling logic: a chunk "runs" for
// pairs / rate seconds of wall time after it is enqueued; the result is a
// deterministic function of the inputs; tag == -13 makes finish fail.
struct FakeExecutor : Executor {
    struct S {
        Clock::time_point ready;
        std::vector<Clock::time_point> chunk_ready;
        bool finishing = false;
    };
    std::vector<S> sl;
    double rate;             // simulated pairs per second
    int64_t chunk_pairs;
    int64_t n_nodes_fake;
    FakeExecutor(int n, double r, int64_t cp) : sl(n), rate(r), chunk_pairs(cp), n_nodes_fake(1000) {}
    int slots() const override { return (int)sl.size(); }
    int64_t footprint(const Job &j) override
    {
        return (int64_t)(j.t1.size() + j.t2.size()) / 3 * 80 + (int64_t)(j.v1.size() + j.v2.size()) * 8 + 1024;
    }
    hsd_status start(int s, Job &j) override
    {
        const int64_t pairs = (int64_t)(j.t1.size() + j.t2.size()) / 3 * n_nodes_fake;
        j.n_chunks = std::max<int64_t>(1, (pairs + chunk_pairs - 1) / chunk_pairs);
        sl[s].chunk_ready.assign((size_t)j.n_chunks, Clock::now());
        sl[s].ready = Clock::now();
        return HSD_OK;
    }
    hsd_status enqueue_chunk(int s, Job &j) override
    {
        const int64_t pairs = (int64_t)(j.t1.size() + j.t2.size()) / 3 * n_nodes_fake;
        const double sec = (double)std::min<int64_t>(chunk_pairs, pairs) / rate;
        S &x = sl[s];
        const auto t0 = std::max(x.ready, Clock::now());
        x.ready = t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(sec));
        x.chunk_ready[(size_t)j.next_chunk] = x.ready;
        return HSD_OK;
    }
    int chunks_done(int s, Job &j) override
    {
        int n = 0;
        const auto now = Clock::now();
        for (int64_t c = 0; c < j.next_chunk; ++c)
            if (sl[s].chunk_ready[(size_t)c] <= now) ++n;
        return n;
    }
    hsd_status enqueue_finish(int s, Job &j) override
    {
        if (j.tag == -13) { set_error("injected executor failure"); return HSD_EDEVICE; }
        sl[s].finishing = true;
        return HSD_OK;
    }
    bool finished(int s, Job &) override { return Clock::now() >= sl[s].ready; }
    hsd_status collect(int, Job &j) override
    {
        double acc = 0.0;
        for (double v : j.v1) acc += v * v;
        for (double v : j.v2) acc -= v * v;
        j.result.d2 = acc;
        j.result.pairs = (double)(j.t1.size() + j.t2.size()) / 3 * (double)n_nodes_fake;
        return HSD_OK;
    }
    void release(int s, Job &) override { sl[s].finishing = false; }
};

} // namespace hsd

using namespace hsd;

struct hsd_server {
    hsd_ctx *ctx = nullptr;                 // may be null for the fake executor
    std::unique_ptr<Executor> ex;
    hsd_server_cfg cfg{};
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::deque<std::shared_ptr<Job>> queue;
    std::vector<std::shared_ptr<Job>> active;   // per slot
    std::unordered_map<uint64_t, std::shared_ptr<Job>> jobs;
    uint64_t next_ticket = 1;
    int64_t admitted_bytes = 0;
    bool stop = false;
    std::thread th;
    Clock::time_point t0 = Clock::now();

    double now_s() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }

    void complete(const std::shared_ptr<Job> &j, hsd_status st)
    {
        if (st < 0 && j->errmsg.empty())
            j->errmsg = st == HSD_ECANCELED ? "request cancelled" : hsd_last_error();
        j->status = st;
        j->result.status = st;
        j->times.finished_s = now_s();
        done_cv.notify_all();
    }

    void free_slot(int s)
    {
        auto &j = active[s];
        ex->release(s, *j);
        admitted_bytes -= j->footprint;
        j->slot = -1;
        active[s].reset();
    }

    // One scheduler pass under the lock; returns true if anything changed.
    bool pass()
    {
        bool progress = false;
        // admit in arrival order while a slot and budget allow
        for (int s = 0; s < (int)active.size() && !queue.empty(); ++s) {
            if (active[s]) continue;
            auto j = queue.front();
            if (admitted_bytes + j->footprint > (int64_t)cfg.hbm_budget_bytes) break;
            queue.pop_front();
            j->slot = s;
            j->times.admitted_s = now_s();
            j->times.footprint = j->footprint;
            active[s] = j;
            admitted_bytes += j->footprint;
            const hsd_status st = ex->start(s, *j);
            if (st != HSD_OK) {
                complete(j, st);
                free_slot(s);
            }
            progress = true;
        }
        for (int s = 0; s < (int)active.size(); ++s) {
            auto j = active[s];
            if (!j) continue;
            if (j->finalizing) {
                if (ex->finished(s, *j)) {
                    const hsd_status st = ex->collect(s, *j);
                    complete(j, j->cancel ? HSD_ECANCELED : st);
                    free_slot(s);
                    progress = true;
                }
                continue;
            }
            const int done = ex->chunks_done(s, *j);
            if (j->cancel) {
                if (done == j->next_chunk) {   // drain in-flight chunks, then drop
                    complete(j, j->fail != HSD_OK ? j->fail : HSD_ECANCELED);
                    free_slot(s);
                    progress = true;
                }
                continue;
            }
            // keep at most two chunks in flight per slot
            while (j->next_chunk < j->n_chunks && j->next_chunk - done < 2) {
                const hsd_status st = ex->enqueue_chunk(s, *j);
                if (st != HSD_OK) { j->cancel = true; j->fail = st; break; }
                j->next_chunk++;
                progress = true;
            }
            if (j->cancel) continue;
            if (j->next_chunk == j->n_chunks && done == j->n_chunks) {
                const hsd_status st = ex->enqueue_finish(s, *j);
                if (st != HSD_OK) {
                    complete(j, st);
                    free_slot(s);
                } else {
                    j->finalizing = true;
                }
                progress = true;
            }
        }
        return progress;
    }

    void run()
    {
        if (ctx) (void)hipSetDevice(ctx->device);
        std::unique_lock<std::mutex> lk(mu);
        while (!stop) {
            const bool prog = pass();
            bool busy = false;
            for (auto &a : active) busy = busy || (bool)a;
            if (!prog) {
                if (busy) cv.wait_for(lk, std::chrono::microseconds(100));
                else cv.wait_for(lk, std::chrono::milliseconds(50));
            }
        }
        // drain: cancel queued, wait for running
        for (auto &j : queue) complete(j, HSD_ECANCELED);
        queue.clear();
        for (int s = 0; s < (int)active.size(); ++s)
            if (active[s]) {
                active[s]->cancel = true;
                complete(active[s], HSD_ECANCELED);
                free_slot(s);
            }
    }
};

static hsd_status server_make(hsd_ctx *ctx, const hsd_server_cfg *cfg, std::unique_ptr<Executor> ex,
                              hsd_server **out)
{
    auto *s = new hsd_server();
    s->ctx = ctx;
    s->cfg = *cfg;
    s->ex = std::move(ex);
    s->active.assign((size_t)s->ex->slots(), nullptr);
    s->th = std::thread([s] { s->run(); });
    *out = s;
    return HSD_OK;
}

static hsd_status cfg_check(const hsd_server_cfg *cfg)
{
    if (!cfg || cfg->slots <= 0 || cfg->slots > 64 || cfg->queue_capacity <= 0 || cfg->hbm_budget_bytes == 0 ||
        cfg->chunk_pairs <= 0) {
        set_error("server config: slots in 1..64, queue_capacity > 0, budget > 0, chunk_pairs > 0");
        return HSD_EINVAL;
    }
    return HSD_OK;
}

extern "C" {

hsd_status hsd_server_create(hsd_ctx *ctx, const hsd_server_cfg *cfg, hsd_server **out)
{
    if (!ctx || !out) { set_error("NULL argument"); return HSD_EINVAL; }
    hsd_status st;
    if ((st = cfg_check(cfg)) != HSD_OK) return st;
    HSD_HIP_TRY(hipSetDevice(ctx->device));
    ctx_retain(ctx);
    std::unique_ptr<Executor> ex(new DeviceExecutor(ctx, cfg->slots, cfg->chunk_pairs));
    return server_make(ctx, cfg, std::move(ex), out);
}

// Test hook (not in the public header): a server whose executor simulates
// work on the CPU at `pairs_per_s` (each request counts nt x 1000 pairs).
hsd_status hsd__server_create_fake(const hsd_server_cfg *cfg, double pairs_per_s, hsd_server **out)
{
    hsd_status st;
    if ((st = cfg_check(cfg)) != HSD_OK) return st;
    std::unique_ptr<Executor> ex(new FakeExecutor(cfg->slots, pairs_per_s, cfg->chunk_pairs));
    return server_make(nullptr, cfg, std::move(ex), out);
}

hsd_status hsd_submit(hsd_server *s, const hsd_request *req, uint64_t *ticket)
{
    if (!s || !req || !ticket) { set_error("NULL argument"); return HSD_EINVAL; }
    if (req->nv < 0 || req->nt < 0 || req->nv2 < 0 || req->nt2 < 0 || (req->nv && !req->verts) ||
        (req->nt && !req->tris) || (s->ctx && !req->rule)) {
        set_error("bad request arrays");
        return HSD_EINVAL;
    }
    auto j = std::make_shared<Job>();
    j->tag = req->tag;
    j->params = req->params;
    j->rule = const_cast<hsd_rule *>(req->rule);
    if (s->ctx) {
        hsd_status st;
        if ((st = validate_params(&req->params)) != HSD_OK) return st;
        if (req->rule->ctx != s->ctx) { set_error("rule belongs to another context"); return HSD_EINVAL; }
    }
    j->v1.assign(req->verts, req->verts + 3 * req->nv);
    j->t1.assign(req->tris, req->tris + 3 * req->nt);
    if (req->verts2) {
        j->has_nu = true;
        j->v2.assign(req->verts2, req->verts2 + 3 * req->nv2);
        j->t2.assign(req->tris2, req->tris2 + 3 * req->nt2);
    }
    for (double x : j->v1) if (!std::isfinite(x)) { set_error("non-finite vertex"); return HSD_EINVAL; }
    for (double x : j->v2) if (!std::isfinite(x)) { set_error("non-finite vertex"); return HSD_EINVAL; }
    for (int32_t i : j->t1) if (i < 0 || i >= req->nv) { set_error("triangle index out of range"); return HSD_EINVAL; }
    for (int32_t i : j->t2) if (i < 0 || i >= req->nv2) { set_error("triangle index out of range"); return HSD_EINVAL; }
    j->footprint = s->ex->footprint(*j);
    if (j->footprint > (int64_t)s->cfg.hbm_budget_bytes) {
        set_error("request footprint %lld exceeds the server budget %zu", (long long)j->footprint,
                  s->cfg.hbm_budget_bytes);
        return HSD_ENOMEM;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if ((int)s->queue.size() >= s->cfg.queue_capacity) { set_error("queue full"); return HSD_EAGAIN; }
    j->ticket = s->next_ticket++;
    j->times.arrival_s = s->now_s();
    s->jobs[j->ticket] = j;
    s->queue.push_back(j);
    *ticket = j->ticket;
    s->cv.notify_all();
    return HSD_OK;
}

// Copy a ticket's state; a failed request's message becomes the calling
// thread's last error.
static hsd_status fill(const std::shared_ptr<Job> &j, hsd_result *out, hsd_request_times *times)
{
    if (out) *out = j->result;
    if (times) *times = j->times;
    if (j->status < 0) set_error("%s", j->errmsg.c_str());
    return j->status;
}

hsd_status hsd_poll(hsd_server *s, uint64_t ticket, hsd_result *out, hsd_request_times *times)
{
    if (!s) { set_error("NULL server"); return HSD_EINVAL; }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) { set_error("unknown ticket"); return HSD_ENOTFOUND; }
    return fill(it->second, out, times);
}

hsd_status hsd_wait(hsd_server *s, uint64_t ticket, double timeout_s, hsd_result *out, hsd_request_times *times)
{
    if (!s) { set_error("NULL server"); return HSD_EINVAL; }
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) { set_error("unknown ticket"); return HSD_ENOTFOUND; }
    auto j = it->second;
    auto pred = [&] { return j->status != HSD_PENDING; };
    if (timeout_s < 0) s->done_cv.wait(lk, pred);
    else s->done_cv.wait_for(lk, std::chrono::duration<double>(timeout_s), pred);
    return fill(j, out, times);
}

hsd_status hsd_cancel(hsd_server *s, uint64_t ticket)
{
    if (!s) { set_error("NULL server"); return HSD_EINVAL; }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) { set_error("unknown ticket"); return HSD_ENOTFOUND; }
    auto j = it->second;
    if (j->status != HSD_PENDING) return HSD_OK;
    for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
        if (*q == j) {
            s->queue.erase(q);
            s->complete(j, HSD_ECANCELED);
            return HSD_OK;
        }
    j->cancel = true;
    s->cv.notify_all();
    return HSD_OK;
}

hsd_status hsd_release(hsd_server *s, uint64_t ticket)
{
    if (!s) { set_error("NULL server"); return HSD_EINVAL; }
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) { set_error("unknown ticket"); return HSD_ENOTFOUND; }
    if (it->second->status == HSD_PENDING) { set_error("ticket still pending"); return HSD_EAGAIN; }
    s->jobs.erase(it);
    return HSD_OK;
}

void hsd_server_destroy(hsd_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv.notify_all();
    }
    s->th.join();
    hsd_ctx *c = s->ctx;
    s->ex.reset();
    delete s;
    if (c) ctx_release(c);
}

} // extern "C"
