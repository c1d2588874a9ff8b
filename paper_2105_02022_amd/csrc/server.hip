// Serving loop: partition jobs that arrive over time, with continuous batching.
//
// Submitted jobs wait in arrival order.  Each worker thread owns a HIP stream.
// When a worker is free it opens a batch with the oldest waiting job, provided
// its estimated device footprint fits the free part of the HBM budget (or
// nothing else runs), and adds later waiting jobs of the same size class
// (n + m within a factor of four of the first job's) and the same
// initial-bipartitioning options whose footprints still fit, at most the
// waiting jobs per worker, between kMinBatchJobs and kMaxBatchJobs (a long
// queue forms large batches for throughput, a short one small batches that
// finish soon); the others keep their place in the queue.  The batch is
// partitioned in one level-by-level union pass (as kmp_partition_batch).
// Jobs that arrive while other batches run are admitted by the next free
// worker, so their work overlaps on the device with the batches already
// running, and small jobs are not held behind a large one of the same
// batch.  Every job's result is the one kmp_partition gives for it alone
// with the options that were current when it was submitted.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <list>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>

#include "kmp_dev.h"

struct kmp_server {
    using clk = std::chrono::steady_clock;
    struct Job {
        kmp_graph_desc d;
        kmp_options opt = {};  // fm_passes, ip_pool, adaptive_eps, pq_balance, async_lp current at submission
        int size_class = 0;    // floor(log2(n + m + 1)) / 2
        size_t foot = 0;
        int state = 0;  // 0 waiting, 1 running, 2 done
        kmp_job_result res;
        clk::time_point t_submit, t_start, t_done;
    };
    int device = 0;
    size_t budget = 0, in_use = 0;
    std::vector<std::thread> workers;
    int nworkers = 1;  // set before the workers start
    std::vector<hipStream_t> streams;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::list<uint64_t> queue;  // waiting jobs in arrival order
    std::unordered_map<uint64_t, Job> jobs;
    uint64_t next_id = 1;
    int running = 0;
    bool stop = false;
    kmp_server_stats st = {};
    kmp_options opt = {};  // the options given to jobs submitted from now on
};

namespace kmp {
namespace {

constexpr int kMaxBatchJobs = 256;
constexpr int kMinBatchJobs = 64;

// Device bytes a job may hold at its peak: the union copy of its CSR, LP and
// contraction work arrays, and the coarse levels (which can stay close to the
// input size on skewed graphs, where coarsening is slow).
size_t footprint(const kmp_graph_desc& d)
{
    const double n = (double)(d.n > 0 ? d.n : 0), m = (double)(d.m > 0 ? d.m : 0);
    return (size_t)(160.0 * n + 96.0 * m) + ((size_t)1 << 20);
}

int size_class_of(const kmp_graph_desc& d)
{
    const uint64_t w = (uint64_t)(d.n > 0 ? d.n : 0) + (uint64_t)(d.m > 0 ? d.m : 0) + 1;
    int b = 0;
    while ((w >> (b + 1)) != 0) ++b;
    return b / 2;
}

bool same_options(const kmp_options& a, const kmp_options& b)
{
    return a.fm_passes == b.fm_passes && a.ip_pool == b.ip_pool && a.adaptive_eps == b.adaptive_eps &&
           a.pq_balance == b.pq_balance && a.async_lp == b.async_lp && a.ip_multilevel == b.ip_multilevel;
}

void worker_main(kmp_server* s, int w)
{
    (void)hipSetDevice(s->device);
    hipStream_t stream = s->streams[w];
    std::vector<uint64_t> ids;
    std::vector<kmp_graph_desc> descs;
    std::vector<kmp_job_result> res;
    kmp_options opt = {};
    for (;;) {
        size_t reserved = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            // the oldest waiting job fits, or nothing else is running (a job
            // larger than the whole budget then runs alone)
            s->cv_work.wait(lk, [&] {
                if (s->stop && s->queue.empty()) return true;
                if (s->queue.empty()) return false;
                const size_t f = s->jobs[s->queue.front()].foot;
                return s->in_use + f <= s->budget || s->in_use == 0;
            });
            if (s->queue.empty()) return;  // stopping and drained
            ids.clear();
            const kmp_server::Job& head = s->jobs[s->queue.front()];
            const int cls = head.size_class;
            opt = head.opt;
            // batch entries and nodes stay below 2^30 each (the union's indices are int32)
            int64_t sum_n = 0, sum_m = 0;
            const int share = (int)(s->queue.size() / (size_t)s->nworkers);
            const int limit = std::min(kMaxBatchJobs, std::max(kMinBatchJobs, share));
            for (auto it = s->queue.begin(); it != s->queue.end() && (int)ids.size() < limit;) {
                kmp_server::Job& jb = s->jobs[*it];
                const bool first = ids.empty();
                bool take = first;
                if (!first) {
                    take = same_options(jb.opt, opt) && jb.size_class >= cls - 1 && jb.size_class <= cls + 1 &&
                           s->in_use + reserved + jb.foot <= s->budget && sum_n + jb.d.n < (int64_t(1) << 30) &&
                           sum_m + jb.d.m < (int64_t(1) << 30);
                }
                if (!take) {
                    ++it;
                    continue;
                }
                reserved += jb.foot;
                sum_n += jb.d.n > 0 ? jb.d.n : 0;
                sum_m += jb.d.m > 0 ? jb.d.m : 0;
                jb.state = 1;
                jb.t_start = kmp_server::clk::now();
                ids.push_back(*it);
                it = s->queue.erase(it);
            }
            s->in_use += reserved;
            ++s->running;
            descs.resize(ids.size());
            for (size_t i = 0; i < ids.size(); ++i) descs[i] = s->jobs[ids[i]].d;
        }
        res.assign(ids.size(), kmp_job_result{});
        const int rc = run_batch(descs.data(), (int32_t)ids.size(), res.data(), stream, &opt, nullptr);
        const auto t_done = kmp_server::clk::now();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (size_t i = 0; i < ids.size(); ++i) {
                kmp_server::Job& jb = s->jobs[ids[i]];
                jb.res = res[i];
                if (rc < 0) jb.res.status = rc;  // the whole batch failed
                jb.state = 2;
                jb.t_done = t_done;
            }
            s->in_use -= reserved;
            --s->running;
            s->st.batches += 1;
            s->st.jobs_done += (int64_t)ids.size();
            if ((int64_t)ids.size() > s->st.max_batch_jobs) s->st.max_batch_jobs = (int64_t)ids.size();
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
}

int take_result(kmp_server* s, uint64_t id, kmp_job_result* result, double* latency_ms, bool block)
{
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->jobs.find(id) == s->jobs.end()) return KMP_EINVAL;
    // look the job up again after every wake-up: submissions may rehash the
    // map, and another thread waiting on the same id may have taken it
    if (block)
        s->cv_done.wait(lk, [&] {
            auto it = s->jobs.find(id);
            return it == s->jobs.end() || it->second.state == 2;
        });
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) return KMP_EINVAL;  // taken by another caller meanwhile
    if (it->second.state != 2) return 0;
    if (result) *result = it->second.res;
    if (latency_ms)
        *latency_ms = std::chrono::duration<double, std::milli>(it->second.t_done - it->second.t_submit).count();
    s->jobs.erase(it);
    return 1;
}

}  // namespace
}  // namespace kmp

using namespace kmp;

extern "C" {

kmp_server* kmp_server_create(size_t hbm_budget_bytes, int32_t workers)
{
    if (workers < 1 || workers > 16 || hbm_budget_bytes == 0) return nullptr;
    kmp_server* s = new (std::nothrow) kmp_server();
    if (!s) return nullptr;
    bool ok = hipGetDevice(&s->device) == hipSuccess;
    s->budget = hbm_budget_bytes;
    s->nworkers = workers;
    for (int w = 0; ok && w < workers; ++w) {
        hipStream_t st = nullptr;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (ok) s->streams.push_back(st);
    }
    try {
        for (int w = 0; ok && w < workers; ++w) s->workers.emplace_back(worker_main, s, w);
    } catch (...) {
        ok = false;
    }
    if (!ok) {
        kmp_server_destroy(s);  // joins the workers that did start (nothing is queued)
        return nullptr;
    }
    return s;
}

int kmp_server_set_options(kmp_server* s, const kmp_options* opt)
{
    if (!s) return KMP_EINVAL;
    kmp_options o = {};
    if (opt) {
        if (opt->fm_passes < 0 || opt->fm_passes > kmp::kFmMaxPasses || (opt->ip_pool != 0 && opt->ip_pool != 1) ||
            (opt->adaptive_eps != 0 && opt->adaptive_eps != 1) || (opt->pq_balance != 0 && opt->pq_balance != 1) || opt->async_lp < 0 ||
            opt->async_lp > 2 || (opt->ip_multilevel != 0 && opt->ip_multilevel != 1))
            return KMP_EINVAL;
        o.fm_passes = opt->fm_passes;
        o.ip_pool = opt->ip_pool;
        o.adaptive_eps = opt->adaptive_eps;
        o.pq_balance = opt->pq_balance;
        o.async_lp = opt->async_lp;
        o.ip_multilevel = opt->ip_multilevel;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->opt = o;
    return KMP_OK;
}

int kmp_server_submit(kmp_server* s, const kmp_graph_desc* job, uint64_t* job_id)
{
    if (!s || !job || !job_id) return KMP_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return KMP_EINVAL;
    const uint64_t id = s->next_id++;
    kmp_server::Job& jb = s->jobs[id];
    jb.d = *job;
    jb.opt = s->opt;
    jb.size_class = size_class_of(*job);
    jb.foot = footprint(*job);
    jb.t_submit = kmp_server::clk::now();
    s->queue.push_back(id);
    s->st.jobs_submitted += 1;
    *job_id = id;
    s->cv_work.notify_one();
    return KMP_OK;
}

int kmp_server_poll(kmp_server* s, uint64_t job_id, kmp_job_result* result, double* latency_ms)
{
    if (!s) return KMP_EINVAL;
    return take_result(s, job_id, result, latency_ms, false);
}

int kmp_server_wait(kmp_server* s, uint64_t job_id, kmp_job_result* result, double* latency_ms)
{
    if (!s) return KMP_EINVAL;
    return take_result(s, job_id, result, latency_ms, true);
}

int kmp_server_stats_get(kmp_server* s, kmp_server_stats* out)
{
    if (!s || !out) return KMP_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->queued = (int64_t)s->queue.size();
    out->running_batches = s->running;
    out->hbm_in_use = (int64_t)s->in_use;
    return KMP_OK;
}

void kmp_server_destroy(kmp_server* s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->workers) t.join();
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    delete s;
}

}  // extern "C"
