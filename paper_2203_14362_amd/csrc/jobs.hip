// Asynchronous batch jobs: a native executor per context.
//
// spade_batch_submit hands a batch (its polygon set and query kind) to the
// context's worker thread and returns at once; the worker rasterises the
// batch into the caller's canvas set and evaluates it over a resident table
// on the context's stream, and spade_batch_wait blocks until the job is done.
// Jobs of one context run one after another in submission order; jobs of
// different contexts (each with its own stream and worker) overlap on the
// device.  A job's results live in a result buffer the context lends it
// until the job handle is freed; freed buffers go back to a pool per job
// kind, so a serving loop that frees each job before the next one of its
// kind neither allocates nor frees device memory per batch.
#include "common.h"

#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

namespace spade {
struct ResBuf {
    DevBuf a, b;   // ids / counts / pair point ids; pair polygon ids
};
}  // namespace spade

struct spade_job {
    spade_ctx *ctx = nullptr;
    spade_canvas *set = nullptr;
    spade_polys polys{};
    bool rebuild = true;         // false: query the set as it stands
    std::vector<int64_t> qbound;
    const spade_table *table = nullptr;
    int kind = 0;
    // results
    int status = SPADE_OK;
    std::string err;
    bool done = false;
    int64_t n_out = 0;
    std::vector<int64_t> off;
    void *out0 = nullptr, *out1 = nullptr;
    spade::ResBuf *rb = nullptr;   // lent by the context until the handle is freed
};

namespace spade {

struct JobQueue {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<spade_job *> q;
    std::thread worker;
    bool stop = false;
    std::vector<ResBuf *> all;       // every result buffer of the context
    std::vector<ResBuf *> idle[4];   // returned ones, per job kind
    int64_t guess = 1 << 20;         // first output capacity tried
};

// A result buffer for a job of `kind`: a returned one of that kind (its
// memory sized by an earlier job) or a new, empty one.
static ResBuf *take_buf(JobQueue *jq, int kind)
{
    std::lock_guard<std::mutex> lk(jq->mu);
    auto &v = jq->idle[kind];
    if (!v.empty()) {
        ResBuf *b = v.back();
        v.pop_back();
        return b;
    }
    ResBuf *b = new (std::nothrow) ResBuf();
    if (b) jq->all.push_back(b);
    return b;
}

static void run_job(JobQueue *jq, spade_job *j)
{
    spade_ctx *ctx = j->ctx;
    ResBuf *rb = j->rb = take_buf(jq, j->kind);
    int rc = !rb ? set_error(ctx, SPADE_E_NOMEM, "host allocation failed")
             : j->rebuild ? spade_batch_rebuild(ctx, &j->polys, (int32_t)(j->qbound.size() - 1), j->qbound.data(), j->set)
                          : SPADE_OK;
    if (rc == SPADE_OK) {
        const int nq = (int)j->qbound.size() - 1;
        if (j->kind == SPADE_JOB_COUNT) {
            const int64_t M = j->qbound.back();
            if (ensure(ctx, rb->a, sizeof(uint64_t) * (size_t)std::max<int64_t>(M, 1))) rc = SPADE_E_NOMEM;
            else rc = spade_batch_join_count(ctx, j->set, j->table, (uint64_t *)rb->a.p);
            j->out0 = rb->a.p;
            j->n_out = M;
        } else if (j->kind == SPADE_JOB_SELECT) {
            j->off.assign((size_t)nq + 1, 0);
            int64_t cap = jq->guess;
            for (int attempt = 0; attempt < 2; ++attempt) {
                if (ensure(ctx, rb->a, sizeof(uint32_t) * (size_t)std::max<int64_t>(cap, 1))) {
                    rc = SPADE_E_NOMEM;
                    break;
                }
                cap = (int64_t)(rb->a.cap / sizeof(uint32_t));
                rc = spade_batch_select(ctx, j->set, j->table, (uint32_t *)rb->a.p, cap, j->off.data());
                if (rc != SPADE_E_CAPACITY) break;
                cap = j->off.back();
                jq->guess = std::max(jq->guess, cap);
            }
            j->out0 = rb->a.p;
            j->n_out = j->off.empty() ? 0 : j->off.back();
        } else {
            int64_t cap = jq->guess, n = 0;
            for (int attempt = 0; attempt < 2; ++attempt) {
                if (ensure(ctx, rb->a, sizeof(uint32_t) * (size_t)std::max<int64_t>(cap, 1)) ||
                    ensure(ctx, rb->b, sizeof(uint32_t) * (size_t)std::max<int64_t>(cap, 1))) {
                    rc = SPADE_E_NOMEM;
                    break;
                }
                cap = (int64_t)(std::min(rb->a.cap, rb->b.cap) / sizeof(uint32_t));
                rc = spade_batch_join_pairs(ctx, j->set, j->table, (uint32_t *)rb->a.p, (uint32_t *)rb->b.p,
                                            cap, &n);
                if (rc != SPADE_E_CAPACITY) break;
                cap = n;
                jq->guess = std::max(jq->guess, cap);
            }
            j->out0 = rb->a.p;
            j->out1 = rb->b.p;
            j->n_out = n;
        }
    }
    j->status = rc;
    if (rc) j->err = ctx->err;
}

static void worker_loop(JobQueue *jq, int device)
{
    (void)hipSetDevice(device);
    while (true) {
        spade_job *j = nullptr;
        {
            std::unique_lock<std::mutex> lk(jq->mu);
            jq->cv.wait(lk, [&] { return jq->stop || !jq->q.empty(); });
            if (jq->q.empty()) return;
            j = jq->q.front();
        }
        {
            SPADE_CTX_LOCK(j->ctx);
            run_job(jq, j);
        }
        {
            std::lock_guard<std::mutex> lk(jq->mu);
            jq->q.pop_front();
            j->done = true;
        }
        jq->cv.notify_all();
    }
}

size_t jobs_bytes(const spade_ctx *ctx)
{
    JobQueue *jq = (JobQueue *)ctx->jobs;
    if (!jq) return 0;
    std::lock_guard<std::mutex> lk(jq->mu);
    size_t b = 0;
    for (const ResBuf *r : jq->all) b += r->a.cap + r->b.cap;
    return b;
}

void jobs_shutdown(spade_ctx *ctx)
{
    JobQueue *jq = (JobQueue *)ctx->jobs;
    if (!jq) return;
    {
        std::lock_guard<std::mutex> lk(jq->mu);
        jq->stop = true;
    }
    jq->cv.notify_all();
    if (jq->worker.joinable()) jq->worker.join();
    for (ResBuf *r : jq->all) {
        free_buf(r->a);
        free_buf(r->b);
        delete r;
    }
    delete jq;
    ctx->jobs = nullptr;
}

}  // namespace spade

using namespace spade;

extern "C" {

int spade_batch_submit(spade_ctx *ctx, spade_canvas *set, const spade_polys *polys, int32_t nq, const int64_t *qbound,
                       const spade_table *t, int kind, spade_job **out)
{
    if (!ctx || !out) return SPADE_E_INVALID;
    *out = nullptr;
    if (!set || !t || (polys && (!qbound || nq < 1)))
        return set_error(ctx, SPADE_E_INVALID, "NULL argument or nq < 1");
    if (kind != SPADE_JOB_SELECT && kind != SPADE_JOB_COUNT && kind != SPADE_JOB_PAIRS)
        return set_error(ctx, SPADE_E_INVALID, "unknown job kind");
    if (set == ctx->plain) return set_error(ctx, SPADE_E_INVALID, "not a caller-owned canvas set");
    spade_job *j = new (std::nothrow) spade_job();
    if (!j) return set_error(ctx, SPADE_E_NOMEM, "host allocation failed");
    j->ctx = ctx;
    j->set = set;
    if (polys) {
        j->polys = *polys;
        j->polys.bbox = nullptr;   // the host array need not outlive the call
        j->qbound.assign(qbound, qbound + nq + 1);
    } else {
        // query only: the set's own query bounds
        SPADE_CTX_LOCK(ctx);
        j->rebuild = false;
        j->qbound.resize((size_t)set->nc + 1);
        for (int q = 0; q < set->nc; ++q) j->qbound[(size_t)q] = set->descs[(size_t)q].poly_base;
        j->qbound[(size_t)set->nc] = set->nc ? set->descs.back().poly_base + set->descs.back().M : 0;
    }
    j->table = t;
    j->kind = kind;
    JobQueue *jq = (JobQueue *)ctx->jobs;
    if (!jq) {
        jq = new (std::nothrow) JobQueue();
        if (!jq) {
            delete j;
            return set_error(ctx, SPADE_E_NOMEM, "host allocation failed");
        }
        try {
            jq->worker = std::thread(worker_loop, jq, ctx->device);
        } catch (...) {
            delete jq;
            delete j;
            return set_error(ctx, SPADE_E_NOMEM, "could not start the context's worker thread");
        }
        ctx->jobs = jq;
    }
    {
        std::lock_guard<std::mutex> lk(jq->mu);
        jq->q.push_back(j);
    }
    jq->cv.notify_all();
    *out = j;
    return SPADE_OK;
}

int spade_batch_wait(spade_job *j, spade_job_result *res)
{
    if (!j || !res) return SPADE_E_INVALID;
    JobQueue *jq = (JobQueue *)j->ctx->jobs;
    {
        std::unique_lock<std::mutex> lk(jq->mu);
        jq->cv.wait(lk, [&] { return j->done; });
    }
    res->status = j->status;
    res->n_out = j->n_out;
    res->out0 = j->out0;
    res->out1 = j->out1;
    res->off = j->off.empty() ? nullptr : j->off.data();
    res->n_off = (int64_t)j->off.size();
    if (j->status) j->ctx->err = j->err;
    return j->status;
}

int spade_job_query(const spade_job *j)
{
    if (!j) return SPADE_E_INVALID;
    JobQueue *jq = (JobQueue *)j->ctx->jobs;
    std::lock_guard<std::mutex> lk(jq->mu);
    return j->done ? 1 : 0;
}

void spade_job_free(spade_job *j)
{
    if (!j) return;
    JobQueue *jq = (JobQueue *)j->ctx->jobs;
    if (jq) {
        std::unique_lock<std::mutex> lk(jq->mu);
        jq->cv.wait(lk, [&] { return j->done; });
        if (j->rb) jq->idle[j->kind].push_back(j->rb);
    }
    delete j;
}

}  // extern "C"
