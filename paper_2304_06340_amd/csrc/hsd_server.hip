// hsd_server.hip -- serving loop: continuous batching of distance requests.
//
// Requests are copied at submit and queued (FIFO).  A scheduler thread
// admits queued requests into free slots while the device bytes charged to
// the slots (running requests' footprints, scratch kept by idle slots) stay
// within the server budget; every slot owns a HIP stream and its scratch
// buffers, so the work of admitted requests overlaps on the device.  An admitted request's direct sum is enqueued in chunks of
// directions (a bounded number in flight per slot), so newly admitted
// requests start within one chunk of the others and a cancelled request
// stops between chunks.  After the last chunk the slot enqueues the
// finalize, the two-level reduction and an 8-byte readback, and the
// scheduler completes the ticket when the slot's completion event fires.
//
// Per-request arithmetic does not depend on the mix: triangle splits and
// lane layout are functions of the request alone, chunk boundaries only
// select which lanes a launch runs, and every reduction has a fixed order,
// so a result is bitwise the same alone or in any mix.  (The splits are
// chosen so that each chunk fills the device; they can differ from
// hsd_distance's, and so can the last bits of a result.)
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
    int64_t footprint = 0;        // device bytes the request needs (meshes + scratch)
    int64_t mesh_bytes = 0;       // of which its meshes (freed when it completes)
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
    virtual hsd_status init() { return HSD_OK; }            // streams, events, pinned buffers
    virtual int slots() const = 0;
    virtual int64_t footprint(Job &j) = 0;                  // sets j.mesh_bytes too
    virtual int64_t retained(int s) const = 0;               // device bytes slot s keeps between requests
    virtual void trim(int s) = 0;                            // free them (slot idle)
    virtual hsd_status start(int s, Job &j) = 0;            // upload / plan; sets n_chunks
    virtual hsd_status enqueue_chunk(int s, Job &j) = 0;    // next chunk (j.next_chunk)
    virtual int chunks_done(int s, Job &j) = 0;             // completed chunks so far
    virtual hsd_status enqueue_finish(int s, Job &j) = 0;   // finalize + reduce + readback
    virtual bool finished(int s, Job &j) = 0;               // readback complete
    virtual hsd_status collect(int s, Job &j) = 0;          // fill j.result
    virtual void release(int s, Job &j) = 0;
};

// A slot's device state persists across its requests: the two mesh objects
// are reloaded per request (their record buffers grow, never shrink), and
// the chunk events are a pool; nothing is freed between requests, since a
// free waits for the whole device and would stall the other slots.
struct DeviceSlot {
    hipStream_t stream = nullptr;
    Scratch partial, nodebuf, redbuf;
    NufftScratch nufft;
    hsd_mesh *mu = nullptr, *nu = nullptr;
    std::vector<TriRec> stage_mu, stage_nu;   // host staging of the record uploads
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

    DeviceExecutor(hsd_ctx *c, int n, int64_t cp) : ctx(c), chunk_pairs(cp), sl(n) {}

    hsd_status init() override
    {
        HSD_HIP_TRY(hipSetDevice(ctx->device));
        for (auto &s : sl) {
            for (hsd_mesh **m : {&s.mu, &s.nu}) {
                *m = new hsd_mesh();
                (*m)->ctx = ctx;
                ctx_retain(ctx);
            }
            HSD_HIP_TRY(hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking));
            HSD_HIP_TRY(hipEventCreateWithFlags(&s.ev_begin, hipEventDefault));
            HSD_HIP_TRY(hipEventCreateWithFlags(&s.ev_done, hipEventDefault));   // timed against ev_begin
            HSD_HIP_TRY(hipHostMalloc((void **)&s.host_result, 64, hipHostMallocDefault));
        }
        return HSD_OK;
    }
    ~DeviceExecutor() override
    {
        (void)hipSetDevice(ctx->device);
        for (auto &s : sl) {
            if (s.stream) (void)hipStreamSynchronize(s.stream);
            for (auto e : s.chunk_ev) (void)hipEventDestroy(e);
            if (s.mu) hsd_mesh_destroy(s.mu);
            if (s.nu) hsd_mesh_destroy(s.nu);
            s.partial.buf.release();
            s.nodebuf.buf.release();
            s.redbuf.buf.release();
            s.nufft.release();
            if (s.ev_begin) (void)hipEventDestroy(s.ev_begin);
            if (s.ev_done) (void)hipEventDestroy(s.ev_done);
            if (s.host_result) (void)hipHostFree(s.host_result);
            if (s.stream) (void)hipStreamDestroy(s.stream);
        }
    }
    int slots() const override { return (int)sl.size(); }

    int64_t retained(int s) const override
    {
        const DeviceSlot &d = sl[s];
        return (int64_t)(d.partial.buf.bytes + d.nodebuf.buf.bytes + d.redbuf.buf.bytes + d.nufft.bytes() +
                         (d.mu ? d.mu->tris.bytes : 0) + (d.nu ? d.nu->tris.bytes : 0));
    }

    void trim(int s) override
    {
        DeviceSlot &d = sl[s];
        (void)hipSetDevice(ctx->device);
        (void)hipStreamSynchronize(d.stream);
        d.partial.buf.release();
        d.nodebuf.buf.release();
        d.redbuf.buf.release();
        d.nufft.release();
        if (d.mu) d.mu->tris.release();
        if (d.nu) d.nu->tris.release();
    }

    static int64_t n_dirs(const hsd_rule *r) { return r->kind == HSD_RULE_SPHERICAL_PRODUCT ? r->n_dir : r->n_nodes; }
    static int64_t nodes_per_dir(const hsd_rule *r) { return r->kind == HSD_RULE_SPHERICAL_PRODUCT ? r->n_rad : 1; }

    // Directions per chunk: chunk_pairs worth of pairs (the NUFFT: one chunk).
    int64_t chunk_dirs_of(const Job &j) const
    {
        if (j.params.method == HSD_METHOD_NUFFT3) return n_dirs(j.rule);
        const int64_t pairs_per_dir = (int64_t)(j.t1.size() + j.t2.size()) / 3 * nodes_per_dir(j.rule);
        const int64_t cd = std::max<int64_t>(1, chunk_pairs / std::max<int64_t>(pairs_per_dir, 1));
        return std::min<int64_t>(cd, n_dirs(j.rule));
    }

    // Triangle splits of a request: at least hsd_distance's, and enough that
    // one chunk's launch has about 4096 waves (a full MI355X at 4 waves per
    // SIMD) so that a chunk fills the device, with blocks short enough that
    // other slots' kernels get compute units between them.  A function of
    // the request alone, so results do not depend on the mix.
    int k_of(const Job &j) const
    {
        if (j.params.method == HSD_METHOD_NUFFT3) return 1;
        const int64_t nt = (int64_t)(j.t1.size() + j.t2.size()) / 3;
        int K = k_direct(j);
        if (j.params.k_splits > 0) return K;   // the caller's choice
        if (j.rule->kind == HSD_RULE_SPHERICAL_PRODUCT && nt > 0) {
            const int64_t waves_per_dir = std::max<int64_t>(1, wave_count(j.rule) / std::max<int64_t>(j.rule->n_dir, 1));
            const int64_t cw = chunk_dirs_of(j) * (wave_kernel_applies(j.rule) ? waves_per_dir : 1);
            const int64_t want = ((int64_t)ctx->num_cu * 16 + cw - 1) / cw;
            K = (int)std::max<int64_t>(K, std::min<int64_t>({want, 64, std::max<int64_t>(1, nt / 64)}));
        }
        return K;
    }

    int k_direct(const Job &j) const
    {
        const int64_t nt = (int64_t)(j.t1.size() + j.t2.size()) / 3;
        return j.rule->kind == HSD_RULE_SPHERICAL_PRODUCT
                   ? choose_k_splits_sp(j.rule, nt, j.params.form, ctx->num_cu, j.params.k_splits)
                   : choose_k_splits_gen(j.rule->n_nodes, nt, ctx->num_cu, j.params.k_splits);
    }

    // Device bytes a request needs on its slot: its meshes (records, indices,
    // vertices, adjacency), the partial transforms, the reduction partials,
    // and for the NUFFT method the whole transform plan (points, sort and
    // scan temporaries, spread tiles, spread grid, FFT grid, twiddles, the
    // rule's per-node tables).
    int64_t footprint(Job &j) override
    {
        const int64_t nt = (int64_t)(j.t1.size() + j.t2.size()) / 3;
        const int64_t nv = (int64_t)(j.v1.size() + j.v2.size()) / 3;
        const int64_t N = j.rule->n_nodes;
        const int64_t mesh = nt * (int64_t)(sizeof(TriRec) + 24) + nv * 28 + 8;
        j.mesh_bytes = mesh;
        const int64_t red = (N / 256 + 2) * 8;
        if (j.params.method == HSD_METHOD_NUFFT3) {
            double X = 0.0;
            for (double x : j.v1) X = std::max(X, std::fabs(x));
            for (double x : j.v2) X = std::max(X, std::fabs(x));
            const int64_t plan = nufft_footprint(X, j.rule, &j.params, nt);
            if (plan < 0) return INT64_MAX;
            return mesh + N * 16 + red + plan;
        }
        return mesh + (int64_t)k_of(j) * N * 16 + red;
    }

    const hsd_mesh *nu_of(const DeviceSlot &d, const Job &j) const { return j.has_nu ? d.nu : nullptr; }

    hsd_status start(int s, Job &j) override
    {
        DeviceSlot &d = sl[s];
        hsd_status st;
        HSD_HIP_TRY(hipSetDevice(ctx->device));
        if ((st = mesh_reload(ctx, d.stream, d.mu, j.v1.data(), (int64_t)j.v1.size() / 3, j.t1.data(),
                              (int64_t)j.t1.size() / 3, d.stage_mu)) != HSD_OK)
            return st;
        if (j.has_nu && (st = mesh_reload(ctx, d.stream, d.nu, j.v2.data(), (int64_t)j.v2.size() / 3, j.t2.data(),
                                          (int64_t)j.t2.size() / 3, d.stage_nu)) != HSD_OK)
            return st;
        const double *w = nullptr, *nuv = nullptr;
        if ((st = rule_tables(j.rule, &j.params, d.stream, &w, &nuv)) != HSD_OK) return st;
        // the NUFFT writes one transform per node (no triangle splits)
        d.K = k_of(j);
        const int64_t N = j.rule->n_nodes;
        if ((st = d.partial.ensure(ctx, (size_t)d.K * N * sizeof(double2))) != HSD_OK) return st;
        d.chunk_dirs = chunk_dirs_of(j);
        j.n_chunks = (n_dirs(j.rule) + d.chunk_dirs - 1) / d.chunk_dirs;
        while ((int64_t)d.chunk_ev.size() < j.n_chunks) {
            hipEvent_t e = nullptr;
            HSD_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            d.chunk_ev.push_back(e);
        }
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
        if (j.has_nu) { mp.B = d.nu->tris.as<const TriRec>(); mp.nB = d.nu->nt; }
        hsd_status st = HSD_OK;
        const int64_t N = j.rule->n_nodes;
        if (j.params.method == HSD_METHOD_NUFFT3) {
            double pairs = 0;
            st = nufft_transform_rule(ctx, d.stream, d.nufft, d.mu, nu_of(d, j), j.rule, &j.params,
                                      d.partial.buf.as<double2>(), &pairs);
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
        const bool empty = j.params.method != HSD_METHOD_NUFFT3 && d.mu->nt + (j.has_nu ? d.nu->nt : 0) == 0;
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
            j.result.pairs = (double)(d.mu->nt + (j.has_nu ? d.nu->nt : 0)) * (double)j.rule->n_nodes;
        j.result.rel_err_stated = stated_rel_err(&j.params, d.mu->nt);
        return HSD_OK;
    }

    void release(int s, Job &) override
    {
        // the slot's work has completed (or been drained); its buffers stay
        (void)hipStreamSynchronize(sl[s].stream);
    }
};

#ifdef HSD_TEST_HOOKS
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
    int64_t footprint(Job &j) override
    {
        j.mesh_bytes = (int64_t)(j.t1.size() + j.t2.size()) / 3 * 80 + (int64_t)(j.v1.size() + j.v2.size()) * 8;
        return j.mesh_bytes + 1024;
    }
    int64_t retained(int) const override { return 0; }
    void trim(int) override {}
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

#endif // HSD_TEST_HOOKS

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
    // Device bytes charged per slot: an idle slot is charged the scratch it
    // keeps between requests, a busy one the larger of its request's
    // footprint and that scratch plus the request's meshes (the scratch is
    // reused, grown if needed); the sum stays within cfg.hbm_budget_bytes.
    std::vector<int64_t> charge;
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

    void set_charge(int s, int64_t c)
    {
        admitted_bytes += c - charge[s];
        charge[s] = c;
    }

    void free_slot(int s)
    {
        auto &j = active[s];
        ex->release(s, *j);
        set_charge(s, ex->retained(s));
        j->slot = -1;
        active[s].reset();
    }

    int64_t busy_charge(int s, const Job &j) const { return std::max(j.footprint, charge[s] + j.mesh_bytes); }

    // Whether job j fits into idle slot s; under budget pressure the idle
    // slots' kept scratch is freed first (a device-wide wait, rare).
    bool fits(int s, const Job &j)
    {
        auto need = [&] { return admitted_bytes - charge[s] + busy_charge(s, j); };
        if (need() <= (int64_t)cfg.hbm_budget_bytes) return true;
        for (int t = 0; t < (int)active.size(); ++t)
            if (!active[t] && charge[t] > 0) {
                ex->trim(t);
                set_charge(t, ex->retained(t));
            }
        return need() <= (int64_t)cfg.hbm_budget_bytes;
    }

    // One scheduler pass under the lock; returns true if anything changed.
    bool pass()
    {
        bool progress = false;
        // admit in arrival order while a slot and budget allow
        for (int s = 0; s < (int)active.size() && !queue.empty(); ++s) {
            if (active[s]) continue;
            auto j = queue.front();
            if (!fits(s, *j)) break;
            queue.pop_front();
            j->slot = s;
            j->times.admitted_s = now_s();
            j->times.footprint = j->footprint;
            active[s] = j;
            set_charge(s, busy_charge(s, *j));
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
    s->charge.assign((size_t)s->ex->slots(), 0);
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
    std::unique_ptr<Executor> ex(new DeviceExecutor(ctx, cfg->slots, cfg->chunk_pairs));
    if ((st = ex->init()) != HSD_OK) return st;   // the executor's destructor frees what was created
    ctx_retain(ctx);
    return server_make(ctx, cfg, std::move(ex), out);
}

#ifdef HSD_TEST_HOOKS
// Test hook (not in the public header): a server whose executor simulates
// work on the CPU at `pairs_per_s` (each request counts nt x 1000 pairs).
hsd_status hsd__server_create_fake(const hsd_server_cfg *cfg, double pairs_per_s, hsd_server **out)
{
    hsd_status st;
    if ((st = cfg_check(cfg)) != HSD_OK) return st;
    std::unique_ptr<Executor> ex(new FakeExecutor(cfg->slots, pairs_per_s, cfg->chunk_pairs));
    return server_make(nullptr, cfg, std::move(ex), out);
}
#endif // HSD_TEST_HOOKS

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
