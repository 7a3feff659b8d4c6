// Served form: a request loop that admits community-detection jobs into
// batches while other batches are on the device.
//
// Jobs are queued FIFO with a copy of their CSR (or, submitted as borrowed,
// with the caller's arrays).  A scheduler thread forms a batch whenever a
// worker slot is free and the HBM budget covers the batch's estimated
// footprint: a large job at the queue head alone, else the queued small jobs
// in order (large ones they pass wait for the head); each batch runs on its own worker thread and
// HIP stream through the batched form, so batches admitted at different
// times overlap on the device; a batch's jobs are copied to the device as
// they are and packed there.  A job of at least solo_min_vertices vertices
// is a batch of its own and runs through the single-graph path, which keeps
// a large graph's sweeps at full width (batching pays off for the small,
// latency-bound graphs).  Memory is reserved at admission and returned when
// the batch completes, which may admit the next jobs.  Every job's result is
// the one it gets alone (the batched form is exact per graph).
#include "louvain.h"

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

struct Job {
    uint64_t ticket = 0;
    int64_t n = 0, nnz = 0;
    std::vector<int64_t> off; // the copy of a copied job (empty when borrowed)
    std::vector<int32_t> col, w;
    const int64_t *p_off = nullptr; // the arrays the job reads: its copy or the caller's
    const int32_t *p_col = nullptr, *p_w = nullptr;
    bool solo = false; // runs alone through the single-graph path
    uint64_t bytes = 0;
    // outcome
    int32_t status = -1; // -1 pending, else louvain_status
    bool done = false;
    louvain_graph_result res{};
    std::vector<int32_t> labels;
    double t_submit = 0, t_admit = 0, t_done = 0, t_packed = 0, t_ready = 0;
    int64_t batch_id = -1, batch_graphs = 0;
};

// device bytes a job adds to a batch (mirrors the handle's allocations:
// three CSR copies, two coarse weight arrays, sort buffers, vertex arrays)
uint64_t job_bytes(int64_t n, int64_t nnz)
{
    const uint64_t big = (uint64_t)(nnz > n ? nnz : n) + 1;
    return 3ull * 8 * (n + 1) + 3ull * 4 * nnz + 2ull * 8 * nnz + 4ull * nnz + 5ull * 8 * big + 144ull * n;
}

} // namespace

struct louvain_server_s {
    louvain_server_config cfg{};
    louvain_params params{};
    int dev = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Job>> queue;
    std::map<uint64_t, std::shared_ptr<Job>> jobs;
    uint64_t next_ticket = 1;
    uint64_t reserved = 0;
    int inflight = 0;
    int64_t next_batch = 0;
    bool stop = false;
    int64_t pending = 0; // submitted and not done
    std::thread scheduler;
    struct Worker {
        std::thread thread;
        std::shared_ptr<std::atomic<bool>> finished;
    };
    std::vector<Worker> workers;
    std::string err;

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

typedef louvain_server_s S;
typedef louvain_server_s::Worker Worker;

// Runs jobs [first, last) of `batch` as one batched run on stream st and
// stores each job's outcome in its Job (results under the server's lock).
// Returns the status of the batch initialisation (an invalid job fails it).
louvain_status run_group(S *s, std::vector<std::shared_ptr<Job>> &batch, size_t first, size_t last, hipStream_t st,
                         double t_packed)
{
    const int32_t ng = (int32_t)(last - first);
    std::vector<int64_t> goff(ng + 1, 0), ns(ng), nnzs(ng);
    std::vector<const int64_t *> offs(ng);
    std::vector<const int32_t *> cols(ng), ws(ng);
    bool weighted = false;
    for (int32_t i = 0; i < ng; ++i) {
        const Job &j = *batch[first + i];
        goff[i + 1] = goff[i] + j.n;
        ns[i] = j.n;
        nnzs[i] = j.nnz;
        offs[i] = j.p_off;
        cols[i] = j.p_col;
        ws[i] = j.p_w;
        weighted |= j.p_w != nullptr;
    }
    const int64_t n = goff[ng];
    std::vector<louvain_graph_result> res(ng);
    std::vector<int32_t> labels(n > 0 ? n : 1);
    louvain_batch_t b = nullptr;
    // each job's arrays go to the device as they are; the union is assembled there
    const louvain_status init = louvain_batch_init_graphs(ng, ns.data(), nnzs.data(), offs.data(), cols.data(),
                                                          weighted ? ws.data() : nullptr, LOUVAIN_VALIDATE, st, &b);
    louvain_status rc = init;
    if (rc == LOUVAIN_OK) (void)hipStreamSynchronize(st);
    const double t_ready = s->now();
    if (rc == LOUVAIN_OK) rc = louvain_batch_run(b, &s->params, labels.data(), 0, res.data());
    const std::string msg = rc == LOUVAIN_OK ? "" : louvain_batch_last_error(b);
    louvain_batch_destroy(b);
    if (init != LOUVAIN_OK && ng > 1 && (init == LOUVAIN_E_BAD_CSR || init == LOUVAIN_E_OVERFLOW))
        return init; // the caller retries the jobs one by one
    std::lock_guard<std::mutex> lk(s->mu);
    for (int32_t i = 0; i < ng; ++i) {
        Job &j = *batch[first + i];
        j.status = rc;
        if (rc == LOUVAIN_OK) {
            j.res = res[i];
            j.labels.assign(labels.begin() + goff[i], labels.begin() + goff[i + 1]);
        }
        j.t_packed = t_packed;
        j.t_ready = t_ready;
    }
    if (rc == LOUVAIN_E_HIP) s->err = msg; // device errors are the server's; invalid jobs only their own
    return init;
}

// Runs one job through louvain_init_csr + louvain_run on stream st.
void run_solo(S *s, Job &j, hipStream_t st, double t_packed)
{
    std::vector<int32_t> labels(j.n > 0 ? j.n : 1);
    louvain_graph_t g = nullptr;
    louvain_result r{};
    louvain_status rc = louvain_init_csr(j.n, j.nnz, j.p_off, j.p_col, j.p_w, LOUVAIN_VALIDATE, st, &g);
    const double t_ready = s->now();
    if (rc == LOUVAIN_OK) rc = louvain_run(g, &s->params, labels.data(), 0, &r);
    const std::string msg = rc == LOUVAIN_OK ? "" : louvain_last_error(g);
    louvain_destroy(g);
    std::lock_guard<std::mutex> lk(s->mu);
    j.status = rc;
    if (rc == LOUVAIN_OK) {
        louvain_graph_result &o = j.res;
        o.n = j.n;
        o.nnz = j.nnz;
        o.num_communities = r.num_communities;
        o.phases = r.phases;
        o.iterations = r.iterations;
        o.q_num = r.q_num;
        o.q_den = r.q_den;
        o.q0_num = r.q0_num;
        o.q = r.q;
        o.n_vf = r.n_vf;
        j.labels = std::move(labels);
        j.labels.resize(j.n);
    }
    j.t_packed = t_packed;
    j.t_ready = t_ready;
    if (rc == LOUVAIN_E_HIP) s->err = msg;
}

void run_batch(S *s, std::vector<std::shared_ptr<Job>> batch, int64_t batch_id, uint64_t bytes)
{
    (void)hipSetDevice(s->dev);
    hipStream_t st = nullptr;
    (void)hipStreamCreate(&st); // default priority
    const double t_packed = s->now();
    if (batch.size() == 1 && batch[0]->solo) {
        run_solo(s, *batch[0], st, t_packed);
    } else {
        const louvain_status init = run_group(s, batch, 0, batch.size(), st, t_packed);
        if (batch.size() > 1 && (init == LOUVAIN_E_BAD_CSR || init == LOUVAIN_E_OVERFLOW))
            for (size_t i = 0; i < batch.size(); ++i) run_group(s, batch, i, i + 1, st, t_packed); // isolate the bad job
    }
    (void)hipStreamDestroy(st);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const double t = s->now();
        for (auto &jp : batch) {
            Job &j = *jp;
            j.t_done = t;
            j.batch_id = batch_id;
            j.batch_graphs = (int64_t)batch.size();
            j.done = true;
            j.off.clear();
            j.off.shrink_to_fit();
            j.col.clear();
            j.col.shrink_to_fit();
            j.w.clear();
            j.w.shrink_to_fit();
            j.p_off = nullptr; // a borrowed job's arrays are the caller's again
            j.p_col = j.p_w = nullptr;
            s->pending -= 1;
        }
        s->reserved -= bytes;
        s->inflight -= 1;
    }
    s->cv.notify_all();
}

void reap(S *s)
{
    // join worker threads that finished (called with the lock held; a finished
    // worker has already released the lock for good)
    for (auto it = s->workers.begin(); it != s->workers.end();) {
        if (it->finished->load()) {
            it->thread.join();
            it = s->workers.erase(it);
        } else {
            ++it;
        }
    }
}

void schedule(S *s)
{
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv.wait(lk, [&] {
            return s->stop || (!s->queue.empty() && s->inflight < s->cfg.max_inflight_batches);
        });
        reap(s);
        if (s->queue.empty()) {
            if (s->stop) break;
            continue;
        }
        // admission: a large job at the queue head runs alone; otherwise the
        // batch takes the small jobs in queue order up to the limits, and the
        // large jobs it passes stay queued until they reach the head (small
        // jobs behind a large one need not wait for it to be admitted)
        std::vector<std::shared_ptr<Job>> batch;
        uint64_t bytes = 0;
        int64_t verts = 0;
        auto fail_oom = [&](const std::shared_ptr<Job> &j) { // can never fit
            j->status = LOUVAIN_E_OOM;
            j->done = true;
            j->t_done = s->now();
            s->pending -= 1;
            s->cv.notify_all();
        };
        while (!s->queue.empty() && s->queue.front()->bytes > s->cfg.hbm_budget_bytes) {
            fail_oom(s->queue.front());
            s->queue.pop_front();
        }
        if (!s->queue.empty() && s->queue.front()->solo) {
            auto &j = s->queue.front();
            if (s->reserved + j->bytes <= s->cfg.hbm_budget_bytes) {
                bytes = j->bytes;
                verts = j->n;
                j->t_admit = s->now();
                batch.push_back(j);
                s->queue.pop_front();
            }
        } else {
            for (auto it = s->queue.begin(); it != s->queue.end() && (int64_t)batch.size() < s->cfg.max_batch_graphs;) {
                const std::shared_ptr<Job> j = *it;
                if (j->bytes > s->cfg.hbm_budget_bytes) {
                    fail_oom(j);
                    it = s->queue.erase(it);
                    continue;
                }
                if (j->solo) {
                    ++it;
                    continue;
                }
                if (s->reserved + bytes + j->bytes > s->cfg.hbm_budget_bytes) break;
                if (!batch.empty() && s->cfg.max_batch_vertices > 0 && verts + j->n > s->cfg.max_batch_vertices) break;
                bytes += j->bytes;
                verts += j->n;
                j->t_admit = s->now();
                batch.push_back(j);
                it = s->queue.erase(it);
            }
        }
        if (batch.empty()) {
            // the head needs memory still held by running batches: wait for one to finish
            if (s->queue.empty()) continue;
            const int running = s->inflight;
            s->cv.wait(lk, [&] { return s->stop || s->inflight < running; });
            continue;
        }
        s->reserved += bytes;
        s->inflight += 1;
        const int64_t id = s->next_batch++;
        Worker w;
        w.finished = std::make_shared<std::atomic<bool>>(false);
        auto flag = w.finished;
        w.thread = std::thread([s, b = std::move(batch), id, bytes, flag]() mutable {
            run_batch(s, std::move(b), id, bytes);
            flag->store(true);
            s->cv.notify_all();
        });
        s->workers.push_back(std::move(w));
    }
    reap(s);
}

} // namespace

extern "C" {

void louvain_server_config_default(louvain_server_config *c)
{
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->hbm_budget_bytes = 200ull << 30;
    c->max_inflight_batches = 4;
    c->max_batch_graphs = 4096;
    c->max_batch_vertices = 0;
    c->solo_min_vertices = 100000;
}

louvain_status louvain_server_create(const louvain_server_config *cfg, const louvain_params *params,
                                     louvain_server_t *out)
{
    if (!out || !params) return LOUVAIN_E_INVALID_ARG;
    *out = nullptr;
    if (params->color) return LOUVAIN_E_INVALID_ARG;
    S *s = new S();
    if (cfg) s->cfg = *cfg;
    else louvain_server_config_default(&s->cfg);
    if (s->cfg.max_inflight_batches < 1 || s->cfg.max_batch_graphs < 1 || s->cfg.hbm_budget_bytes == 0 ||
        s->cfg.max_batch_vertices < 0 || s->cfg.solo_min_vertices < 0) {
        delete s;
        return LOUVAIN_E_INVALID_ARG;
    }
    s->params = *params;
    if (hipGetDevice(&s->dev) != hipSuccess) {
        delete s;
        return LOUVAIN_E_HIP;
    }
    s->t0 = std::chrono::steady_clock::now();
    s->scheduler = std::thread(schedule, s);
    *out = s;
    return LOUVAIN_OK;
}

} // extern "C"

namespace {

louvain_status submit(S *s, int64_t n, int64_t nnz, const int64_t *offsets, const int32_t *cols,
                      const int32_t *weights, bool borrow, uint64_t *ticket)
{
    if (!s || !ticket || n < 0 || nnz < 0 || !offsets || (nnz > 0 && !cols)) return LOUVAIN_E_INVALID_ARG;
    if (n >= ((int64_t)1 << 31) - 1) return LOUVAIN_E_INVALID_ARG;
    if (offsets[0] != 0 || offsets[n] != nnz) return LOUVAIN_E_BAD_CSR;
    auto j = std::make_shared<Job>();
    j->n = n;
    j->nnz = nnz;
    if (borrow) {
        // read in place when the job runs; its device validation covers the
        // checks a copied job gets here
        j->p_off = offsets;
        j->p_col = cols;
        j->p_w = weights;
    } else {
        for (int64_t x = 0; x < nnz; ++x)
            if (cols[x] < 0 || cols[x] >= n) return LOUVAIN_E_BAD_CSR;
        j->off.assign(offsets, offsets + n + 1);
        j->col.assign(cols, cols + nnz);
        if (weights) j->w.assign(weights, weights + nnz);
        j->p_off = j->off.data();
        j->p_col = j->col.data();
        j->p_w = weights ? j->w.data() : nullptr;
    }
    j->solo = s->cfg.solo_min_vertices > 0 && n >= s->cfg.solo_min_vertices;
    j->bytes = job_bytes(n, nnz);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        j->ticket = s->next_ticket++;
        j->t_submit = s->now();
        s->jobs[j->ticket] = j;
        s->queue.push_back(j);
        s->pending += 1;
        *ticket = j->ticket;
    }
    s->cv.notify_all();
    return LOUVAIN_OK;
}

} // namespace

extern "C" {

louvain_status louvain_server_submit(louvain_server_t s, int64_t n, int64_t nnz, const int64_t *offsets,
                                     const int32_t *cols, const int32_t *weights, uint64_t *ticket)
{
    return submit(s, n, nnz, offsets, cols, weights, false, ticket);
}

louvain_status louvain_server_submit_borrowed(louvain_server_t s, int64_t n, int64_t nnz, const int64_t *offsets,
                                              const int32_t *cols, const int32_t *weights, uint64_t *ticket)
{
    return submit(s, n, nnz, offsets, cols, weights, true, ticket);
}

louvain_status louvain_server_poll(louvain_server_t s, uint64_t ticket, int32_t *labels_out, louvain_job_result *out,
                                   int32_t *done)
{
    if (!s || !done) return LOUVAIN_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return LOUVAIN_E_INVALID_ARG;
    Job &j = *it->second;
    *done = j.done ? 1 : 0;
    if (!j.done) return LOUVAIN_OK;
    if (out) {
        std::memset(out, 0, sizeof(*out));
        out->result = j.res;
        out->status = j.status;
        out->t_submit = j.t_submit;
        out->t_admit = j.t_admit;
        out->t_done = j.t_done;
        out->batch_id = j.batch_id;
        out->batch_graphs = j.batch_graphs;
        out->t_packed = j.t_packed;
        out->t_ready = j.t_ready;
    }
    if (labels_out && j.status == LOUVAIN_OK && !j.labels.empty())
        std::memcpy(labels_out, j.labels.data(), j.labels.size() * sizeof(int32_t));
    return LOUVAIN_OK;
}

louvain_status louvain_server_release(louvain_server_t s, uint64_t ticket)
{
    if (!s) return LOUVAIN_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end() || !it->second->done) return LOUVAIN_E_INVALID_ARG;
    s->jobs.erase(it);
    return LOUVAIN_OK;
}

louvain_status louvain_server_wait_all(louvain_server_t s)
{
    if (!s) return LOUVAIN_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv.wait(lk, [&] { return s->pending == 0; });
    return s->err.empty() ? LOUVAIN_OK : LOUVAIN_E_HIP;
}

const char *louvain_server_last_error(louvain_server_t s) { return s ? s->err.c_str() : ""; }

void louvain_server_destroy(louvain_server_t s)
{
    if (!s) return;
    louvain_server_wait_all(s);
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->scheduler.joinable()) s->scheduler.join();
    for (auto &w : s->workers)
        if (w.thread.joinable()) w.thread.join();
    delete s;
}

} // extern "C"
