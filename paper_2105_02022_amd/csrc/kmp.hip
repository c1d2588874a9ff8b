// libkmp C ABI and the deep-MGP scheduler (paper Alg. 1 unrolled into level
// loops, Alg. 2 per level, Sec. 4 "Handling General k").
//
//   coarsen:  while n_l > 2C (and < 64 levels): U_l (Sec. 5.1), LP clustering,
//             two-hop, stop when the level shrank by less than 5%, contract.
//   uncoarsen: from the coarsest level down: project, bipartition blocks until
//             the level has k'_l = min(k, ceil2(n_l / C)) blocks (k at level 0,
//             at least 2), balance, refine with k-way LP.
// Host code only orchestrates; every data-parallel step runs in the kernels
// of prims/lp/coarsen/ip/balance.hip.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <mutex>

#include "kmp_dev.h"

namespace kmp {

namespace {

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t) { return std::chrono::duration<double, std::milli>(clk::now() - t).count(); }

void init_pool_once()
{
    static std::once_flag once;
    std::call_once(once, [] {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipMemPool_t pool;
            if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
                uint64_t thr = UINT64_MAX;
                (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
            }
        }
    });
}

// ---------------------------------------------------------------- validation
__global__ void k_check_rows(const int32_t* __restrict__ xadj, int32_t n, int64_t* bad)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > n) return;
    bool b = (v == 0 && xadj[0] != 0) || (v > 0 && xadj[v] < xadj[v - 1]);
    if (b) atomicAdd((unsigned long long*)bad, 1ull);
}

__global__ void k_check_entries(const int32_t* __restrict__ xadj, const int32_t* __restrict__ adjncy,
                                const int32_t* __restrict__ vwgt, const int32_t* __restrict__ adjwgt, int32_t n,
                                uint32_t* __restrict__ src, uint32_t* __restrict__ dst, int64_t* bad)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    bool b = vwgt && vwgt[v] <= 0;
    for (int32_t e = xadj[v]; e < xadj[v + 1]; ++e) {
        const int32_t u = adjncy[e];
        b |= u < 0 || u >= n || u == v || (adjwgt && adjwgt[e] <= 0);
        src[e] = (uint32_t)v;
        dst[e] = (uint32_t)(u < 0 || u >= n ? 0 : u);
    }
    if (b) atomicAdd((unsigned long long*)bad, 1ull);
}

__global__ void k_gather_pair(const uint32_t* __restrict__ a, const uint32_t* __restrict__ perm, int64_t m,
                              uint32_t* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] = a[perm[i]];
}

// forward (src,dst,w) sorted by (src,dst) vs reverse (dst,src,w) sorted the same way
__global__ void k_compare_sorted(const uint32_t* __restrict__ fs, const uint32_t* __restrict__ fd,
                                 const uint32_t* __restrict__ fperm, const uint32_t* __restrict__ rs,
                                 const uint32_t* __restrict__ rd, const uint32_t* __restrict__ rperm,
                                 const int32_t* __restrict__ adjwgt, int64_t m, int64_t* bad)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    bool b = fs[i] != rs[i] || fd[i] != rd[i];
    if (adjwgt) b |= adjwgt[fperm[i]] != adjwgt[rperm[i]];
    if (i > 0) b |= fs[i] == fs[i - 1] && fd[i] == fd[i - 1];  // duplicate entry
    if (b) atomicAdd((unsigned long long*)bad, 1ull);
}

// sort (major, minor) pairs, carrying a permutation of entry ids
void sort_pairs(Ctx& c, const uint32_t* major, const uint32_t* minor, int64_t m, int bits, uint32_t* out_major,
                uint32_t* out_minor, uint32_t* perm)
{
    DBuf<uint32_t> k(c, m), k2(c, m), v2(c, m);
    iota_i32(c, reinterpret_cast<int32_t*>(perm), m);
    KMP_HIP(hipMemcpyAsync(k.p, minor, sizeof(uint32_t) * m, hipMemcpyDeviceToDevice, c.stream));
    radix_sort_pairs(c, k.p, perm, k2.p, v2.p, m, bits);
    hipLaunchKernelGGL(k_gather_pair, dim3(grid_for(m)), dim3(kBlock), 0, c.stream, major, perm, m, k.p);
    KMP_LAUNCH_CHECK();
    radix_sort_pairs(c, k.p, perm, k2.p, v2.p, m, bits);
    KMP_HIP(hipMemcpyAsync(out_major, k.p, sizeof(uint32_t) * m, hipMemcpyDeviceToDevice, c.stream));
    hipLaunchKernelGGL(k_gather_pair, dim3(grid_for(m)), dim3(kBlock), 0, c.stream, minor, perm, m, out_minor);
    KMP_LAUNCH_CHECK();
}

}  // namespace

int validate_graph(Ctx& c, const DGraph& g)
{
    const int32_t n = g.n;
    const int64_t m = g.m;
    int64_t* bad = c.counters() + 12;
    c.zero(bad, sizeof(int64_t));
    hipLaunchKernelGGL(k_check_rows, dim3(grid_for((int64_t)n + 1)), dim3(kBlock), 0, c.stream, g.xadj, n, bad);
    KMP_LAUNCH_CHECK();
    if (c.read1(bad)) return KMP_EGRAPH;
    if (m == 0) return KMP_OK;
    DBuf<uint32_t> src(c, m), dst(c, m);
    hipLaunchKernelGGL(k_check_entries, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, g.xadj, g.adjncy, g.vwgt,
                       g.adjwgt, n, src.p, dst.p, bad);
    KMP_LAUNCH_CHECK();
    if (c.read1(bad)) return KMP_EGRAPH;
    const int bits = bits_for((uint64_t)(n > 0 ? n - 1 : 0));
    DBuf<uint32_t> fs(c, m), fd(c, m), fp(c, m), rs(c, m), rd(c, m), rp(c, m);
    sort_pairs(c, src.p, dst.p, m, bits, fs.p, fd.p, fp.p);
    sort_pairs(c, dst.p, src.p, m, bits, rs.p, rd.p, rp.p);
    hipLaunchKernelGGL(k_compare_sorted, dim3(grid_for(m)), dim3(kBlock), 0, c.stream, fs.p, fd.p, fp.p, rs.p, rd.p,
                       rp.p, g.adjwgt, m, bad);
    KMP_LAUNCH_CHECK();
    return c.read1(bad) ? KMP_EGRAPH : KMP_OK;
}

namespace {

__global__ void k_iota_weights(const int32_t* __restrict__ vwgt, int32_t n, int32_t* __restrict__ label,
                               int64_t* __restrict__ cw, uint32_t* __restrict__ fav)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    label[v] = (int32_t)v;
    cw[v] = vwgt ? vwgt[v] : 1;
    if (fav) fav[v] = kNone;
}

__global__ void k_final_ids(const int32_t* __restrict__ part, const int32_t* __restrict__ first, int32_t n,
                            int32_t* __restrict__ out)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) out[v] = first[part[v]];
}

// ---------------------------------------------------------------- batches: union of the jobs' graphs
struct JobPtrs {
    const int32_t* xadj;
    const int32_t* adjncy;
    const int32_t* vwgt;
    const int32_t* adjwgt;
    int32_t* out;
};

// largest i in [0, cnt) with off[i] <= x (off nondecreasing, off[0] = 0 <= x)
__device__ inline int32_t find_member(const int64_t* __restrict__ off, int32_t cnt, int64_t x)
{
    int32_t lo = 0, hi = cnt - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// xadj[n] of every member job (compared with the m it was given)
__global__ void k_job_tails(const JobPtrs* __restrict__ P, const int32_t* __restrict__ mjob,
                            const int64_t* __restrict__ moff, int32_t cnt, int32_t* __restrict__ out)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) out[i] = P[mjob[i]].xadj[moff[i + 1] - moff[i]];
}

// per-job sums of node weights (jobs with vwgt) and edge weights (jobs with
// adjwgt), read from the inputs at their position in the union
__global__ __launch_bounds__(kBlock) void k_job_sums(const JobPtrs* __restrict__ P, const int32_t* __restrict__ mjob,
                                                     const int64_t* __restrict__ off, int32_t cnt, int64_t total,
                                                     bool nodes, int64_t* out)
{
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < total; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = base + threadIdx.x;
        int32_t j = -1;
        int64_t w = 0;
        if (x < total) {
            const int32_t i = find_member(off, cnt, x);
            j = mjob[i];
            const int32_t* a = nodes ? P[j].vwgt : P[j].adjwgt;
            w = a ? a[x - off[i]] : 1;
        }
        job_add(out, j, w);
    }
}

__global__ void k_union_nodes(const JobPtrs* __restrict__ P, const int32_t* __restrict__ mjob,
                              const int64_t* __restrict__ moff, const int64_t* __restrict__ meoff, int32_t cnt,
                              int32_t N, int32_t* __restrict__ xadj, int32_t* __restrict__ vwgt,
                              int32_t* __restrict__ gid)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    const int32_t i = find_member(moff, cnt, v);
    const int32_t j = mjob[i];
    const int64_t l = v - moff[i];
    xadj[v] = (int32_t)(meoff[i] + P[j].xadj[l]);
    if (vwgt) vwgt[v] = P[j].vwgt ? P[j].vwgt[l] : 1;
    gid[v] = j;
}

__global__ void k_union_entries(const JobPtrs* __restrict__ P, const int32_t* __restrict__ mjob,
                                const int64_t* __restrict__ moff, const int64_t* __restrict__ meoff, int32_t cnt,
                                int64_t M, int32_t* __restrict__ adjncy, int32_t* __restrict__ adjwgt)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= M) return;
    const int32_t i = find_member(meoff, cnt, e);
    const int32_t j = mjob[i];
    const int64_t l = e - meoff[i];
    adjncy[e] = (int32_t)(moff[i] + P[j].adjncy[l]);
    if (adjwgt) adjwgt[e] = P[j].adjwgt ? P[j].adjwgt[l] : 1;
}

__global__ void k_fill_gid(const int32_t* __restrict__ mjob, const int64_t* __restrict__ moff, int32_t cnt, int32_t N,
                           int32_t* __restrict__ gid)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < N) gid[v] = mjob[find_member(moff, cnt, v)];
}

__global__ void k_gather_at(const int32_t* __restrict__ a, const int64_t* __restrict__ idx, int32_t cnt,
                            int64_t* __restrict__ out)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) out[i] = a[idx[i]];
}

__global__ void k_final_ids_jobs(const int32_t* __restrict__ part, const int32_t* __restrict__ first,
                                 const int32_t* __restrict__ gid, const int32_t* __restrict__ noff,
                                 const JobPtrs* __restrict__ P, int32_t N)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    const int32_t j = gid[v];
    P[j].out[v - noff[j]] = first[part[v]];
}

// ---------------------------------------------------------------- scheduler
int64_t eps_ppm(double eps) { return (int64_t)std::llround(eps * (double)kPPM); }

int64_t level_U(int32_t n_l, int32_t& kc, int64_t cV, int64_t e)
{
    while (kc > 2 && (int64_t)n_l <= (int64_t)(kc / 2) * kC) kc = std::max(2, kc / 2);
    return e * cV / (kPPM * (int64_t)kc);
}

int32_t ceil2_div_C(int32_t n_l)
{
    int64_t p = 1;
    while (p * kC < n_l) p *= 2;
    return p > INT32_MAX ? INT32_MAX : (int32_t)p;
}

int check_args(const int32_t* xadj, int32_t n, int64_t m, int32_t k, double eps, const int32_t* out)
{
    if (n < 0 || k < 1 || !(eps >= 0.0) || eps > 1000.0 || m < 0 || m > INT32_MAX) return KMP_EINVAL;
    if (n > 0 && (!xadj || !out)) return KMP_EINVAL;
    return KMP_OK;
}

// Checks m == xadj[n] and the int32 bounds of the weight sums; returns c(V)
// and the largest degree.
int64_t prepare(Ctx& c, const DGraph& g, int32_t& maxdeg)
{
    int64_t xn = 0;
    entries_and_max_degree(c, g.xadj, g.n, xn, maxdeg);
    if (xn != g.m) throw Error(KMP_EINVAL, "m != xadj[n]");
    if (g.m > 0 && !g.adjncy) throw Error(KMP_EINVAL, "adjncy is NULL");
    int64_t sums[2] = {node_weight_sum(c, g.vwgt, g.n), edge_weight_sum(c, g.adjwgt, g.m)};
    if (sums[0] > INT32_MAX || sums[1] / 2 > INT32_MAX) throw Error(KMP_EOVERFLOW, "weight sum exceeds int32");
    return sums[0];
}

// One job of a pass: its input, parameters and results.
struct JobRun {
    DGraph g;
    int32_t k = 1;
    double eps = 0;
    uint64_t seed = 0;
    int32_t* out = nullptr;
    int status = KMP_OK;
    bool run = false;         // takes part in the multilevel pass
    int64_t cV = 0, e = 0, lk = 0;
    int32_t kc = 0;           // k' of the coarsening bound (Sec. 5.1)
    int32_t L = -1;           // coarsest level
    int64_t cut = 0, maxw = 0;
    int32_t maxdeg = -1;      // largest degree of the input (one graph)
    std::vector<int32_t> level_n;
    std::vector<int64_t> level_m;
};

// A level of the pass: the member jobs' level graphs (one graph, or their
// disjoint union in job order).
struct Level {
    DGraph g;
    OwnedGraph own;               // storage for unions and coarse levels
    DBuf<int32_t> map;            // to the next coarser level (-1: the job's coarsest level is this one)
    std::unique_ptr<LPSchedule> sched;
    bool sched_full = false;      // the schedule holds every node (refinement can reuse it)
    std::unique_ptr<LPSchedule> asched;  // asynchronous LP: visit-order schedule
    bool asched_full = false;
    std::vector<int32_t> mem;     // member jobs, ascending
    std::vector<int64_t> moff;    // by member: first node; moff[mem.size()] = n
    std::vector<int32_t> nn;      // by job: nodes at this level
    std::vector<int64_t> mm;      // by job: directed entries at this level
    DBuf<int32_t> gid;            // batches: job of every node
    DBuf<int32_t> dnoff, dgend;   // batches: by job, first node / end of the job's node range
    DBuf<int32_t> dmjob;          // batches: by member
    DBuf<int64_t> dmoff;
    int32_t maxdeg = -1;          // one graph: largest degree (-1: not known)
};

struct Totals {
    int64_t moves_cl = 0, moves_ref = 0, rated = 0, contracted = 0;
    int32_t bip = 0, brounds = 0, exact = 0;
    double ms_lp = 0, ms_con = 0, ms_ip = 0, ms_ref = 0;
};

template <typename T>
DBuf<T> upload(Ctx& c, const std::vector<T>& v)
{
    DBuf<T> d(c, v.size());
    if (!v.empty()) c.write(d.p, v.data(), sizeof(T) * v.size());
    return d;
}

// Per-job device tables of a batch level (gid, per-job node offsets / range
// ends, member lists) from its member list and per-job node counts.
void set_level_tables(Ctx& c, Level& L, int32_t nj)
{
    const int32_t cnt = (int32_t)L.mem.size();
    std::vector<int32_t> noff(nj, 0), gend(nj, 0);
    for (int32_t i = 0; i < cnt; ++i) {
        noff[L.mem[i]] = (int32_t)L.moff[i];
        gend[L.mem[i]] = (int32_t)L.moff[i + 1];
    }
    L.dnoff = upload(c, noff);
    L.dgend = upload(c, gend);
    L.dmjob = upload(c, L.mem);
    L.dmoff = upload(c, L.moff);
    if (!L.gid.p) {
        L.gid = DBuf<int32_t>(c, (size_t)std::max(L.g.n, 1));
        if (L.g.n > 0) {
            hipLaunchKernelGGL(k_fill_gid, dim3(grid_for(L.g.n)), dim3(kBlock), 0, c.stream, L.dmjob.p, L.dmoff.p,
                               cnt, L.g.n, L.gid.p);
            KMP_LAUNCH_CHECK();
        }
    }
}

JobTabs tabs_of(const Level& L, const DBuf<uint32_t>& ghash)
{
    JobTabs t;
    t.gid = L.gid.p;
    t.ghash = ghash.p;
    t.noff = L.dnoff.p;
    return t;
}

// Jobs with run = true in job order, with their node / entry offsets in the union.
void batch_members(const std::vector<JobRun>& jobs, std::vector<int32_t>& mem, std::vector<int64_t>& moff,
                   std::vector<int64_t>& meoff)
{
    mem.clear();
    moff.assign(1, 0);
    meoff.assign(1, 0);
    for (int32_t j = 0; j < (int32_t)jobs.size(); ++j)
        if (jobs[j].run) {
            mem.push_back(j);
            moff.push_back(moff.back() + jobs[j].g.n);
            meoff.push_back(meoff.back() + jobs[j].g.m);
        }
}

// Checks every job of a batch on the device at once: m == xadj[n] and the
// int32 bounds of the weight sums (failing jobs leave the pass with their
// code); computes c(V).  Uploads the per-job pointer table.
void check_batch(Ctx& c, std::vector<JobRun>& jobs, DBuf<JobPtrs>& dptr)
{
    const int32_t nj = (int32_t)jobs.size();
    std::vector<JobPtrs> ptr(nj);
    for (int32_t j = 0; j < nj; ++j)
        ptr[j] = JobPtrs{jobs[j].g.xadj, jobs[j].g.adjncy, jobs[j].g.vwgt, jobs[j].g.adjwgt, jobs[j].out};
    dptr = upload(c, ptr);
    auto members = [&](std::vector<int32_t>& mem, std::vector<int64_t>& moff, std::vector<int64_t>& meoff) {
        batch_members(jobs, mem, moff, meoff);
    };
    std::vector<int32_t> mem;
    std::vector<int64_t> moff, meoff;
    members(mem, moff, meoff);
    int32_t cnt = (int32_t)mem.size();
    if (cnt == 0) return;
    {   // m == xadj[n]
        DBuf<int32_t> dm = upload(c, mem);
        DBuf<int64_t> dmo = upload(c, moff);
        DBuf<int32_t> tails(c, (size_t)cnt);
        hipLaunchKernelGGL(k_job_tails, dim3(grid_for(cnt)), dim3(kBlock), 0, c.stream, dptr.p, dm.p, dmo.p, cnt,
                           tails.p);
        KMP_LAUNCH_CHECK();
        std::vector<int32_t> ht(cnt);
        c.read(ht.data(), tails.p, sizeof(int32_t) * cnt);
        for (int32_t i = 0; i < cnt; ++i)
            if ((int64_t)ht[i] != jobs[mem[i]].g.m || (jobs[mem[i]].g.m > 0 && !jobs[mem[i]].g.adjncy)) {
                jobs[mem[i]].status = KMP_EINVAL;
                jobs[mem[i]].run = false;
            }
    }
    members(mem, moff, meoff);
    cnt = (int32_t)mem.size();
    if (cnt == 0) return;
    {   // weight sums (int64), only for jobs that carry weights
        bool any_vw = false, any_ew = false;
        for (int32_t j : mem) {
            any_vw |= jobs[j].g.vwgt != nullptr;
            any_ew |= jobs[j].g.adjwgt != nullptr;
        }
        std::vector<int64_t> vs(nj, 0), es(nj, 0);
        DBuf<int32_t> dm = upload(c, mem);
        DBuf<int64_t> dmo = upload(c, moff), dme = upload(c, meoff);
        DBuf<int64_t> acc(c, (size_t)nj);
        if (any_vw) {
            c.zero(acc.p, sizeof(int64_t) * nj);
            hipLaunchKernelGGL(k_job_sums, dim3(grid_for(moff[cnt], kBlock, 1024)), dim3(kBlock), 0, c.stream, dptr.p,
                               dm.p, dmo.p, cnt, moff[cnt], true, acc.p);
            KMP_LAUNCH_CHECK();
            c.read(vs.data(), acc.p, sizeof(int64_t) * nj);
        }
        if (any_ew && meoff[cnt] > 0) {
            c.zero(acc.p, sizeof(int64_t) * nj);
            hipLaunchKernelGGL(k_job_sums, dim3(grid_for(meoff[cnt], kBlock, 1024)), dim3(kBlock), 0, c.stream,
                               dptr.p, dm.p, dme.p, cnt, meoff[cnt], false, acc.p);
            KMP_LAUNCH_CHECK();
            c.read(es.data(), acc.p, sizeof(int64_t) * nj);
        }
        for (int32_t j : mem) {
            const int64_t cV = jobs[j].g.vwgt ? vs[j] : jobs[j].g.n;
            const int64_t ew = jobs[j].g.adjwgt ? es[j] : jobs[j].g.m;
            if (cV > INT32_MAX || ew / 2 > INT32_MAX) {
                jobs[j].status = KMP_EOVERFLOW;
                jobs[j].run = false;
            }
            jobs[j].cV = cV;
        }
    }
}

// Level 0 of a batch: the jobs with run = true concatenated in job order.
void build_union(Ctx& c, const std::vector<JobRun>& jobs, const DBuf<JobPtrs>& dptr, Level& L0)
{
    const int32_t nj = (int32_t)jobs.size();
    std::vector<int32_t> mem;
    std::vector<int64_t> moff, meoff;
    batch_members(jobs, mem, moff, meoff);
    const int32_t cnt = (int32_t)mem.size();
    if (cnt == 0) return;
    const int64_t N = moff[cnt], M = meoff[cnt];
    if (N >= INT32_MAX || M > INT32_MAX) throw Error(KMP_EINVAL, "batch exceeds int32 node or entry range");
    bool any_vw = false, any_ew = false;
    for (int32_t j : mem) {
        any_vw |= jobs[j].g.vwgt != nullptr;
        any_ew |= jobs[j].g.adjwgt != nullptr;
    }
    L0.mem = mem;
    L0.moff = moff;
    L0.nn.assign(nj, 0);
    L0.mm.assign(nj, 0);
    for (int32_t j : mem) {
        L0.nn[j] = jobs[j].g.n;
        L0.mm[j] = jobs[j].g.m;
    }
    L0.own.xadj = DBuf<int32_t>(c, (size_t)N + 1);
    L0.own.adjncy = DBuf<int32_t>(c, (size_t)std::max<int64_t>(M, 1));
    if (any_vw) L0.own.vwgt = DBuf<int32_t>(c, (size_t)N);
    if (any_ew) L0.own.adjwgt = DBuf<int32_t>(c, (size_t)std::max<int64_t>(M, 1));
    L0.gid = DBuf<int32_t>(c, (size_t)N);
    set_level_tables(c, L0, nj);  // gid is filled below
    DBuf<int64_t> dme = upload(c, meoff);
    hipLaunchKernelGGL(k_union_nodes, dim3(grid_for(N)), dim3(kBlock), 0, c.stream, dptr.p, L0.dmjob.p, L0.dmoff.p,
                       dme.p, cnt, (int32_t)N, L0.own.xadj.p, L0.own.vwgt.p, L0.gid.p);
    KMP_LAUNCH_CHECK();
    fill_i32(c, L0.own.xadj.p + N, (int32_t)M, 1);
    if (M > 0) {
        hipLaunchKernelGGL(k_union_entries, dim3(grid_for(M)), dim3(kBlock), 0, c.stream, dptr.p, L0.dmjob.p,
                           L0.dmoff.p, dme.p, cnt, M, L0.own.adjncy.p, L0.own.adjwgt.p);
        KMP_LAUNCH_CHECK();
    }
    L0.g = L0.own.view((int32_t)N, M);
}

// The deep-MGP pass (Alg. 1 unrolled) over the jobs with run = true.  One
// job works on its own graph; several run level by level on the union of
// their level graphs, each job with its own parameters and stopping points.
// Batches: the jobs of level L whose LP runs in the one-workgroup kernel (small
// enough, no node of degree above the tier-1 cut-off); `part` (may be NULL)
// marks the jobs that take part.
// Labels of job j: clustering, its nodes (lfirst / lcount NULL); refinement,
// its blocks.
void pick_small_jobs(const Ctx& c, const Level& L, const std::vector<uint8_t>* part, int32_t nj, LPState& ls,
                     const std::vector<int32_t>* lfirst = nullptr, const std::vector<int32_t>* lcount = nullptr)
{
    ls.njobs = nj;
    for (size_t mi = 0; mi < L.mem.size(); ++mi) {
        const int32_t j = L.mem[mi];
        if (part && !(*part)[j]) continue;
        const int32_t nl = lcount ? (*lcount)[j] : L.nn[j];
        if (small_job_fits(c, L.nn[j], nl) && L.sched->job_maxdeg[j] <= c.tune.cut[1]) {
            ls.small_jobs.push_back(j);
            ls.small_start.push_back((int32_t)L.moff[mi]);
            ls.small_count.push_back(L.nn[j]);
            ls.small_loff.push_back(lfirst ? (*lfirst)[j] : (int32_t)L.moff[mi]);
            ls.small_nlab.push_back(nl);
        }
    }
}

void run_jobs(Ctx& c, std::vector<JobRun>& jobs, bool batch, const DBuf<JobPtrs>& dptr, const kmp_options* opt,
              Totals& t)
{
    const int32_t nj = (int32_t)jobs.size();
    const bool phase_sync = opt && opt->profile >= 2;
    // moves of the one-workgroup LP calls (clustering, refinement), read once at the end
    DBuf<int64_t> dmoves(c, 2 * (kRounds + 1));
    c.zero(dmoves.p, sizeof(int64_t) * 2 * (kRounds + 1));
    std::vector<std::unique_ptr<Level>> lv;
    lv.emplace_back(new Level());
    if (batch) {
        build_union(c, jobs, dptr, *lv[0]);
        if (lv[0]->mem.empty()) return;
    } else {
        Level& L0 = *lv[0];
        L0.g = jobs[0].g;
        L0.mem = {0};
        L0.moff = {0, jobs[0].g.n};
        L0.nn = {jobs[0].g.n};
        L0.mm = {jobs[0].g.m};
        L0.maxdeg = jobs[0].maxdeg;
    }
    std::vector<uint32_t> hseed(nj);
    std::vector<uint64_t> seeds(nj);
    std::vector<int64_t> lkv(nj);
    std::vector<AdaptiveJob> adapt(nj);
    for (int32_t j = 0; j < nj; ++j) {
        hseed[j] = seed_hash(jobs[j].seed);
        seeds[j] = jobs[j].seed;
        lkv[j] = jobs[j].lk;
        adapt[j] = AdaptiveJob{jobs[j].cV, jobs[j].k, jobs[j].e};
    }
    DBuf<uint32_t> dghash;
    if (batch) dghash = upload(c, hseed);
    const uint64_t seed0 = jobs[lv[0]->mem[0]].seed;  // scalar hash prefixes (one job)

    // ---------------- coarsening
    for (int32_t l = 0;; ++l) {
        Level& L = *lv[l];
        const DGraph& g = L.g;
        for (int32_t j : L.mem) {
            jobs[j].level_n.push_back(L.nn[j]);
            jobs[j].level_m.push_back(L.mm[j]);
        }
        auto t0 = clk::now();
        std::vector<uint8_t> takes(nj, 0);
        std::vector<int64_t> U(nj, 0);
        int32_t ntake = 0;
        for (int32_t j : L.mem) {
            if (L.nn[j] > 2 * kC && l < kMaxLevels) {
                takes[j] = 1;
                U[j] = level_U(L.nn[j], jobs[j].kc, jobs[j].cV, jobs[j].e);
                ++ntake;
            } else {
                jobs[j].L = l;
            }
        }
        if (ntake == 0) break;
        const bool full = ntake == (int32_t)L.mem.size();
        const JobTabs jt = tabs_of(L, dghash);
        DBuf<uint8_t> dtakes;
        DBuf<int64_t> dU;
        if (batch) {
            dU = upload(c, U);
            if (!full) dtakes = upload(c, takes);
        }
        // a small single graph skips the schedule: its LP builds its own class lists
        const bool small_lp = !batch && L.maxdeg >= 0 && L.maxdeg <= c.tune.cut[1] && small_job_fits(c, g.n, g.n);
        if (c.async_lp) {
            L.asched.reset(new LPSchedule());
            lp_build_async_schedule(c, g, l, seed0, *L.asched, jt, dtakes.p);
            L.asched_full = full;
        } else if (!small_lp) {
            L.sched.reset(new LPSchedule());
            lp_build_schedule(c, g, l, seed0, *L.sched, jt, dtakes.p, nj);
            L.sched_full = full;
        }
        DBuf<int32_t> label(c, (size_t)g.n);
        DBuf<int64_t> cw(c, (size_t)g.n);
        DBuf<uint32_t> fav(c, (size_t)g.n);
        hipLaunchKernelGGL(k_iota_weights, dim3(grid_for(g.n)), dim3(kBlock), 0, c.stream, g.vwgt, g.n, label.p, cw.p,
                           fav.p);
        KMP_LAUNCH_CHECK();
        LPState ls{label.p, cw.p, g.n, nullptr, batch ? 0 : U[0], fav.p, TAG_CL, jt,
                   batch ? L.dnoff.p : nullptr, batch ? dU.p : nullptr};
        if (batch && !c.async_lp) pick_small_jobs(c, L, &takes, nj, ls);
        ls.moves_out = dmoves.p;
        LPStats lps = lp_run(c, g, l, seed0, c.async_lp ? L.asched.get() : small_lp ? nullptr : L.sched.get(), ls);
        for (int r = 0; r < kRounds; ++r) t.moves_cl += lps.moves[r];
        t.exact += lps.exact_subrounds;
        std::vector<int64_t> nc;
        DBuf<int32_t> cid;  // one graph: the coarse ids, computed once for the test and the contraction
        if (!batch) {
            int32_t nonempty = -1;  // known when no two-hop merge ran
            two_hop(c, g, U[0], label.p, cw.p, fav.p, false, &nonempty);
            nc.assign(1, contract_ids(c, g, cw.p, cid, JobTabs{}, nullptr, nonempty));
        } else {
            count_nonempty_jobs(c, cw.p, g.n, jt, nj, nc);
            std::vector<int64_t> lim(nj, 0);
            bool any = false;
            for (int32_t j : L.mem)
                if (takes[j] && nc[j] > L.nn[j] / 2) {
                    lim[j] = nc[j] - L.nn[j] / 2;
                    any = true;
                }
            if (any) {
                DBuf<int64_t> dlim = upload(c, lim);
                two_hop_jobs(c, g, jt, dU.p, dlim.p, L.dgend.p, nj, label.p, cw.p, fav.p);
                count_nonempty_jobs(c, cw.p, g.n, jt, nj, nc);
            }
        }
        t.ms_lp += ms_since(t0);
        std::vector<uint8_t> keep(nj, 0);
        int32_t nkeep = 0;
        for (int32_t j : L.mem) {
            if (!takes[j]) continue;
            if (20LL * nc[j] > 19LL * L.nn[j]) {
                jobs[j].L = l;  // converged: this level is the job's coarsest
            } else {
                keep[j] = 1;
                ++nkeep;
            }
        }
        if (nkeep == 0) break;
        auto t1 = clk::now();
        std::unique_ptr<Level> next(new Level());
        L.map = DBuf<int32_t>(c, (size_t)g.n);
        int32_t cn = 0;
        int64_t cm = 0;
        DBuf<uint8_t> dkeep;
        if (batch) dkeep = upload(c, keep);
        if (batch) contract(c, g, label.p, cw.p, L.map.p, next->own, cn, cm, jt, dkeep.p);
        else
            contract(c, g, label.p, cw.p, L.map.p, next->own, cn, cm, jt, nullptr, &cid, (int32_t)nc[0],
                     &next->maxdeg);
        next->g = next->own.view(cn, cm);
        next->nn.assign(nj, 0);
        next->mm.assign(nj, 0);
        next->moff.assign(1, 0);
        for (int32_t j : L.mem)
            if (keep[j]) {
                next->mem.push_back(j);
                next->nn[j] = (int32_t)nc[j];
                next->moff.push_back(next->moff.back() + nc[j]);
                t.contracted += L.mm[j];
            }
        if (!batch) {
            next->mm[0] = cm;
        } else {
            set_level_tables(c, *next, nj);
            const int32_t cnt = (int32_t)next->mem.size();
            DBuf<int64_t> ends(c, (size_t)cnt + 1);
            hipLaunchKernelGGL(k_gather_at, dim3(grid_for(cnt + 1)), dim3(kBlock), 0, c.stream, next->own.xadj.p,
                               next->dmoff.p, cnt + 1, ends.p);
            KMP_LAUNCH_CHECK();
            std::vector<int64_t> he(cnt + 1);
            c.read(he.data(), ends.p, sizeof(int64_t) * (cnt + 1));
            for (int32_t i = 0; i < cnt; ++i) next->mm[next->mem[i]] = he[i + 1] - he[i];
        }
        if (phase_sync) c.sync();
        t.ms_con += ms_since(t1);
        lv.push_back(std::move(next));
    }
    int32_t Lmax = 0;
    for (int32_t j : lv[0]->mem) Lmax = std::max(Lmax, jobs[j].L);

    // ---------------- uncoarsening
    BlockTab bt;
    DBuf<int32_t> part;
    DBuf<int64_t> wt, cap;
    for (int32_t l = Lmax; l >= 0; --l) {
        Level& L = *lv[l];
        const DGraph& g = L.g;
        const JobTabs jt = tabs_of(L, dghash);
        auto t0 = clk::now();
        // block table: projected jobs keep their blocks; a job whose coarsest
        // level is this one starts with the single block (0, k)
        BlockTab nt;
        std::vector<int32_t> remap(std::max(bt.size(), 1)), start(nj, -1);
        int32_t ob = 0;
        for (int32_t j : L.mem) {
            if (jobs[j].L == l) {
                start[j] = nt.size();
                nt.first.push_back(0);
                nt.f.push_back(jobs[j].k);
                nt.job.push_back(j);
            } else {
                while (ob < bt.size() && bt.job[ob] == j) {
                    remap[ob] = nt.size();
                    nt.first.push_back(bt.first[ob]);
                    nt.f.push_back(bt.f[ob]);
                    nt.job.push_back(j);
                    ++ob;
                }
            }
        }
        DBuf<int32_t> fine(c, (size_t)std::max(g.n, 1));
        if (!batch) {
            if (l == Lmax) c.zero(fine.p, sizeof(int32_t) * (size_t)g.n);
            else project(c, part.p, L.map.p, fine.p, g.n);
        } else {
            DBuf<int32_t> dremap = upload(c, remap), dstart = upload(c, start);
            project_jobs(c, l == Lmax ? nullptr : part.p, l == Lmax ? nullptr : L.map.p, dremap.p, L.gid.p,
                         dstart.p, fine.p, g.n);
        }
        part = std::move(fine);
        bt = std::move(nt);
        // bipartition blocks until every job has k'_l blocks (Alg. 1, Sec. 4)
        std::vector<int32_t> kp(nj, 0);
        for (int32_t j : L.mem) {
            kp[j] = (l == 0) ? jobs[j].k : std::min(jobs[j].k, ceil2_div_C(L.nn[j]));
            kp[j] = std::max(kp[j], 2);
        }
        auto t1 = clk::now();
        for (;;) {
            std::vector<int32_t> nbj(nj, 0);
            for (int32_t b = 0; b < bt.size(); ++b) ++nbj[bt.job[b]];
            std::vector<uint8_t> split(bt.size());
            bool any = false;
            for (int32_t b = 0; b < bt.size(); ++b) {
                split[b] = bt.f[b] >= 2 && nbj[bt.job[b]] < kp[bt.job[b]];
                any |= split[b] != 0;
            }
            if (!any) break;
            t.bip += bipartition_round(c, g, l, part.p, bt, split, lkv, hseed, c.adaptive_eps ? &adapt : nullptr,
                                       &seeds);
        }
        if (phase_sync) c.sync();
        t.ms_ip += ms_since(t1);
        auto t2 = clk::now();
        const int32_t nb = bt.size();
        wt = DBuf<int64_t>(c, (size_t)nb);
        cap = DBuf<int64_t>(c, (size_t)nb);
        block_weights(c, g, part.p, nb, wt.p);
        std::vector<int64_t> hcap(nb);
        std::vector<int32_t> boff(nj, 0);
        for (int32_t b = nb - 1; b >= 0; --b) {
            hcap[b] = (int64_t)bt.f[b] * jobs[bt.job[b]].lk;
            boff[bt.job[b]] = b;
        }
        c.write(cap.p, hcap.data(), sizeof(int64_t) * nb);
        DBuf<int32_t> dboff;
        if (batch) dboff = upload(c, boff);
        auto level_sched = [&]() -> const LPSchedule& {
            if (!L.sched || !L.sched_full) {
                L.sched.reset(new LPSchedule());
                lp_build_schedule(c, g, l, seed0, *L.sched, jt, nullptr, nj);
                L.sched_full = true;
            }
            return *L.sched;
        };
        const bool small_lp = !batch && L.maxdeg >= 0 && L.maxdeg <= c.tune.cut[1] && small_job_fits(c, g.n, nb);
        if (!small_lp) level_sched();
        t.brounds += (c.pq_balance ? balance_pq : balance)(c, g, l, batch ? seeds : std::vector<uint64_t>{seed0},
                                                            level_sched, part.p, wt.p, bt, cap.p, jt, dboff.p,
                                                            &hcap);
        LPState ls{part.p, wt.p, nb, cap.p, 0, nullptr, TAG_REF, jt, dboff.p, nullptr};
        if (batch && !c.async_lp) {
            std::vector<int32_t> nbk(nj, 0);
            for (int32_t b = 0; b < nb; ++b) ++nbk[bt.job[b]];
            pick_small_jobs(c, L, nullptr, nj, ls, &boff, &nbk);
        }
        ls.moves_out = dmoves.p + kRounds + 1;
        const LPSchedule* rsched = nullptr;
        if (c.async_lp) {
            if (!L.asched || !L.asched_full) {
                L.asched.reset(new LPSchedule());
                lp_build_async_schedule(c, g, l, seed0, *L.asched, jt, nullptr);
                L.asched_full = true;
            }
            rsched = L.asched.get();
        } else if (!small_lp) {
            rsched = &level_sched();
        }
        LPStats lps = lp_run(c, g, l, seed0, rsched, ls);
        for (int r = 0; r < kRounds; ++r) t.moves_ref += lps.moves[r];
        t.exact += lps.exact_subrounds;
        if (phase_sync) c.sync();
        t.ms_ref += ms_since(t2) + (ms_since(t0) - ms_since(t1));
        // the coarser level is no longer needed
        if (l < Lmax) lv[l + 1].reset();
    }
    // ---------------- final block ids, cuts and statuses
    Level& L0 = *lv[0];
    const int32_t nb = bt.size();
    DBuf<int32_t> dfirst = upload(c, bt.first);
    if (!batch) {
        hipLaunchKernelGGL(k_final_ids, dim3(grid_for(L0.g.n)), dim3(kBlock), 0, c.stream, part.p, dfirst.p, L0.g.n,
                           jobs[0].out);
        KMP_LAUNCH_CHECK();
    } else {
        hipLaunchKernelGGL(k_final_ids_jobs, dim3(grid_for(L0.g.n)), dim3(kBlock), 0, c.stream, part.p, dfirst.p,
                           L0.gid.p, L0.dnoff.p, dptr.p, L0.g.n);
        KMP_LAUNCH_CHECK();
    }
    // block weights, rated entries, move counts (and one graph's cut) in one read-back
    if (!batch) edge_cut_launch(c, L0.g, part.p);
    constexpr int32_t nm = 2 * (kRounds + 1);
    std::vector<std::pair<const int64_t*, int32_t>> segs = {
        {wt.p, nb}, {c.spread(SP_RATED), kSpreadWords}, {dmoves.p, nm}};
    if (!batch) segs.push_back({c.spread(SP_CUT), kSpreadWords});
    std::vector<int64_t> h((size_t)nb + kSpreadWords + nm + (batch ? 0 : kSpreadWords));
    read_segments(c, segs, h.data());
    const int64_t* hw = h.data();
    const int64_t* hr = hw + nb;
    const int64_t* hm = hr + kSpreadWords;
    for (int32_t b = 0; b < nb; ++b) jobs[bt.job[b]].maxw = std::max(jobs[bt.job[b]].maxw, hw[b]);
    if (!batch) {
        int64_t cut2 = 0;
        for (int q = 0; q < kSpreadWords; ++q) cut2 += hm[nm + q];
        jobs[0].cut = cut2 / 2;
    } else {
        std::vector<int64_t> cuts;
        edge_cut_jobs(c, L0.g, part.p, L0.gid.p, nj, cuts);
        for (int32_t j : L0.mem) jobs[j].cut = cuts[j];
    }
    for (int32_t j : L0.mem) jobs[j].status = jobs[j].maxw > jobs[j].lk ? KMP_IMBALANCED : KMP_OK;
    t.rated = 0;
    for (int q = 0; q < kSpreadWords; ++q) t.rated += hr[q];
    for (int r = 0; r < kRounds; ++r) {
        t.moves_cl += hm[r];
        t.moves_ref += hm[kRounds + 1 + r];
    }
}

// Derived integers of a job (Sec. 2 balance constraint, Sec. 5.1); k = 1 and
// n = 0 jobs are finished here.
void setup_job(Ctx& c, JobRun& jb)
{
    jb.e = eps_ppm(jb.eps);
    const int64_t W = (jb.cV + jb.k - 1) / jb.k;
    jb.lk = W * (kPPM + jb.e) / kPPM;
    jb.kc = (int32_t)std::min<int64_t>(jb.k, jb.g.n / kC);
    jb.run = jb.g.n > 0 && jb.k > 1;
    if (jb.g.n > 0 && jb.k == 1) {
        fill_i32(c, jb.out, 0, jb.g.n);
        jb.maxw = jb.cV;
        jb.level_n = {jb.g.n};
        jb.level_m = {jb.g.m};
        jb.L = 0;
        jb.status = jb.cV > jb.lk ? KMP_IMBALANCED : KMP_OK;
    }
    if (jb.g.n == 0) jb.status = KMP_OK;
}

void fill_stats(kmp_stats* st, const JobRun& jb, const Totals& t)
{
    st->cut = jb.cut;
    st->lk = jb.lk;
    st->max_block_weight = jb.maxw;
    st->levels = std::max(jb.L, 0);
    for (size_t l = 0; l < jb.level_n.size() && l <= (size_t)kMaxLevels; ++l) {
        st->level_n[l] = jb.level_n[l];
        st->level_m[l] = jb.level_m[l];
    }
    st->bipartitions = t.bip;
    st->balance_rounds = t.brounds;
    st->lp_exact_subrounds = t.exact;
    st->lp_cluster_moves = t.moves_cl;
    st->lp_refine_moves = t.moves_ref;
    st->lp_rated_edges = t.rated;
    st->contracted_edges = t.contracted;
    st->ms_coarsen_lp = t.ms_lp;
    st->ms_contract = t.ms_con;
    st->ms_initial = t.ms_ip;
    st->ms_refine = t.ms_ref;
}

int partition_impl(const DGraph& g0, int32_t k, double eps, uint64_t seed, int32_t* out_part, hipStream_t stream,
                   const kmp_options* opt, kmp_stats* st, void* arena, size_t arena_bytes)
{
    auto t_start = clk::now();
    if (!arena) init_pool_once();
    std::unique_ptr<Ctx> ctx(arena ? new Ctx(stream, arena, arena_bytes) : new Ctx(stream));
    Ctx& c = *ctx;
    std::unique_ptr<Prof> prof;
    if (opt && opt->profile) {
        prof.reset(new Prof());
        prof->mask = opt->profile_classes;
        c.prof = prof.get();
    }
    c.force_exact = opt && opt->force_exact;
    c.small_level_n = opt ? opt->small_level_n : 0;
    c.plain_loads = opt && opt->plain_loads;
    if (set_ip_options(c, opt) != KMP_OK) return KMP_EINVAL;
    std::vector<JobRun> jobs(1);
    JobRun& jb = jobs[0];
    jb.g = g0;
    jb.k = k;
    jb.eps = eps;
    jb.seed = seed;
    jb.out = out_part;
    jb.cV = prepare(c, g0, jb.maxdeg);
    if (opt && opt->validate) {
        int rc = validate_graph(c, g0);
        if (rc != KMP_OK) return rc;
    }
    setup_job(c, jb);
    Totals t;
    if (jb.run) run_jobs(c, jobs, false, DBuf<JobPtrs>(), opt, t);
    c.sync();
    if (st) {
        fill_stats(st, jb, t);
        st->ms_total = ms_since(t_start);
        if (prof) c.prof_collect(st->prof_launches, st->prof_ms, st->prof_bytes);
        st->workspace_bytes = (int64_t)c.workspace_taken();
    }
    c.prof = nullptr;
    return jb.status;
}

int partition_batch_impl(const kmp_graph_desc* gd, int32_t count, kmp_job_result* res, hipStream_t stream,
                         const kmp_options* opt, kmp_stats* st)
{
    auto t_start = clk::now();
    init_pool_once();
    Ctx c(stream);
    std::unique_ptr<Prof> prof;
    if (opt && opt->profile) {
        prof.reset(new Prof());
        prof->mask = opt->profile_classes;
        c.prof = prof.get();
    }
    c.force_exact = opt && opt->force_exact;
    c.small_level_n = opt ? opt->small_level_n : 0;
    c.plain_loads = opt && opt->plain_loads;
    if (set_ip_options(c, opt) != KMP_OK) return KMP_EINVAL;
    std::vector<JobRun> jobs(count);
    for (int32_t i = 0; i < count; ++i) {
        JobRun& jb = jobs[i];
        const kmp_graph_desc& d = gd[i];
        jb.g.n = d.n;
        jb.g.m = d.m;
        jb.g.xadj = d.xadj;
        jb.g.adjncy = d.adjncy;
        jb.g.vwgt = d.vwgt;
        jb.g.adjwgt = d.adjwgt;
        jb.k = d.k;
        jb.eps = d.epsilon;
        jb.seed = d.seed;
        jb.out = d.out_part;
        jb.status = check_args(d.xadj, d.n, d.m, d.k, d.epsilon, d.out_part);
        if (jb.status == KMP_OK && d.n == 0 && d.m != 0) jb.status = KMP_EINVAL;
        jb.run = jb.status == KMP_OK && d.n > 0;
    }
    if (opt && opt->validate)
        for (auto& jb : jobs)
            if (jb.run) {
                jb.status = validate_graph(c, jb.g);
                jb.run = jb.status == KMP_OK;
            }
    // m == xadj[n] and the weight sums, for the whole batch at once
    Totals t;
    DBuf<JobPtrs> dptr;
    check_batch(c, jobs, dptr);
    for (auto& jb : jobs)
        if (jb.run) setup_job(c, jb);
    bool any = false;
    for (auto& jb : jobs) any |= jb.run;
    if (any) run_jobs(c, jobs, true, dptr, opt, t);
    c.sync();
    if (res)
        for (int32_t i = 0; i < count; ++i) {
            kmp_job_result& r = res[i];
            memset(&r, 0, sizeof(r));
            r.status = jobs[i].status;
            r.levels = std::max(jobs[i].L, 0);
            r.cut = jobs[i].cut;
            r.max_block_weight = jobs[i].maxw;
            r.lk = jobs[i].lk;
            for (size_t l = 0; l < jobs[i].level_n.size() && l <= (size_t)kMaxLevels; ++l)
                r.level_n[l] = jobs[i].level_n[l];
        }
    if (st) {
        memset(st, 0, sizeof(*st));
        fill_stats(st, JobRun(), t);
        for (auto& jb : jobs) st->cut += jb.cut;
        st->ms_total = ms_since(t_start);
        st->workspace_bytes = (int64_t)c.workspace_taken();
        if (prof) c.prof_collect(st->prof_launches, st->prof_ms, st->prof_bytes);
    }
    c.prof = nullptr;
    return KMP_OK;
}

DGraph make_graph(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt, int32_t n,
                  int64_t m)
{
    DGraph g;
    g.n = n;
    g.m = m;
    g.xadj = xadj;
    g.adjncy = adjncy;
    g.vwgt = vwgt;
    g.adjwgt = adjwgt;
    return g;
}

template <typename F>
int64_t guarded(F&& f)
{
    try {
        return f();
    } catch (const Error& e) {
        return e.code;
    } catch (const std::bad_alloc&) {
        return KMP_ENOMEM;
    } catch (...) {
        return KMP_EHIP;
    }
}

// Coordinate search over output-invariant launch choices: time kmp_partition
// under each candidate (median of `reps` calls after an untimed one), keep a
// candidate only if it is at least 2% faster, and require every partition to
// equal the first one.
int64_t autotune_impl(const kmp_graph_desc& d, int32_t reps, hipStream_t stream, kmp_tuning* chosen,
                      kmp_autotune_report* report)
{
    const Tuning start = tuning_get();
    Tuning cur = start;
    std::vector<int32_t> ref((size_t)std::max(d.n, 1)), got((size_t)std::max(d.n, 1));
    int32_t configs = 0;
    bool have_ref = false;
    auto run = [&](const Tuning& t) -> double {
        tuning_set(t);
        std::vector<double> ms;
        for (int32_t r = 0; r <= reps; ++r) {
            const auto t0 = clk::now();
            const int rc = kmp_partition(d.xadj, d.adjncy, d.vwgt, d.adjwgt, d.n, d.m, d.k, d.epsilon, d.seed,
                                         d.out_part, stream);
            if (rc < 0) throw Error(rc, "partition failed while tuning");
            if (r > 0) ms.push_back(ms_since(t0));
        }
        if (d.n > 0) {
            KMP_HIP(hipMemcpyAsync(got.data(), d.out_part, sizeof(int32_t) * (size_t)d.n, hipMemcpyDeviceToHost,
                                   stream));
            KMP_HIP(hipStreamSynchronize(stream));
        }
        if (!have_ref) {
            ref = got;
            have_ref = true;
        } else if (ref != got) {
            throw Error(KMP_EHIP, "a tuning changed the partition");
        }
        ++configs;
        std::sort(ms.begin(), ms.end());
        return ms[ms.size() / 2];
    };
    try {
        const double ms_start = run(cur);
        double best = ms_start;
        auto consider = [&](const Tuning& t) {
            if (!tuning_valid(t)) return;
            const double ms = run(t);
            if (ms < 0.98 * best) {  // a clear gain, not timing noise
                best = ms;
                cur = t;
            }
        };
        for (int32_t v : {-1, 2048, 4096, 8192, 16384, 32768}) {
            if (v == cur.small_level_n) continue;
            Tuning t = cur;
            t.small_level_n = v;
            consider(t);
        }
        const Tuning dflt;
        for (int i = 0; i < 4; ++i)
            for (int32_t v : {dflt.cut[i], dflt.cut[i] / 2}) {
                if (v == cur.cut[i]) continue;
                Tuning t = cur;
                t.cut[i] = v;
                consider(t);
            }
        for (int32_t v : {2048, 8192}) {  // the hub tier's LDS tables (no effect without hubs)
            if (v == cur.hub_ts) continue;
            Tuning t = cur;
            t.hub_ts = v;
            consider(t);
        }
        tuning_set(cur);
        if (report) {
            report->configs = configs;
            report->reps = reps;
            report->ms_start = ms_start;
            report->ms_best = best;
        }
    } catch (...) {
        tuning_set(start);
        throw;
    }
    if (chosen) {
        memset(chosen, 0, sizeof(*chosen));
        chosen->small_level_n = cur.small_level_n;
        chosen->tier0_deg = cur.cut[0];
        chosen->tier1_deg = cur.cut[1];
        chosen->tier2_deg = cur.cut[2];
        chosen->tier3_deg = cur.cut[3];
        chosen->hub_lds_slots = cur.hub_ts;
    }
    return KMP_OK;
}

}  // namespace

int set_ip_options(Ctx& c, const kmp_options* opt)
{
    if (opt && (opt->fm_passes < 0 || opt->fm_passes > kFmMaxPasses)) return KMP_EINVAL;
    if (opt && opt->ip_pool != 0 && opt->ip_pool != 1) return KMP_EINVAL;
    if (opt && opt->adaptive_eps != 0 && opt->adaptive_eps != 1) return KMP_EINVAL;
    if (opt && opt->pq_balance != 0 && opt->pq_balance != 1) return KMP_EINVAL;
    if (opt && (opt->async_lp < 0 || opt->async_lp > 2)) return KMP_EINVAL;
    if (opt && opt->ip_multilevel != 0 && opt->ip_multilevel != 1) return KMP_EINVAL;
    c.fm_passes = opt ? opt->fm_passes : 0;
    c.ip_multilevel = opt && opt->ip_multilevel;
    c.async_lp = opt ? opt->async_lp : 0;
    c.ip_pool = opt && opt->ip_pool;
    c.adaptive_eps = opt && opt->adaptive_eps;
    c.pq_balance = opt && opt->pq_balance;
    return KMP_OK;
}

int run_batch(const kmp_graph_desc* graphs, int32_t count, kmp_job_result* results, hipStream_t stream,
              const kmp_options* opt, kmp_stats* stats)
{
    return (int)guarded([&]() -> int64_t {
        return partition_batch_impl(graphs, count, results, stream, opt, stats);
    });
}

}  // namespace kmp

using namespace kmp;

namespace {
std::mutex g_noalloc_mu[64];   // one call at a time per device: the scratch region is shared
void* g_noalloc_ptr[64] = {};  // device address of the scratch region per device, set at the first call
}  // namespace

extern "C" {

int kmp_partition_ex(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt,
                     int32_t n, int64_t m, int32_t k, double epsilon, uint64_t seed, int32_t* out_part, void* stream,
                     const kmp_options* opt, kmp_stats* stats)
{
    if (stats) memset(stats, 0, sizeof(*stats));
    int rc = check_args(xadj, n, m, k, epsilon, out_part);
    if (rc != KMP_OK) return rc;
    if (n == 0) return m == 0 ? KMP_OK : KMP_EINVAL;
    return (int)guarded([&]() -> int64_t {
        return partition_impl(make_graph(xadj, adjncy, vwgt, adjwgt, n, m), k, epsilon, seed, out_part,
                              (hipStream_t)stream, opt, stats, nullptr, 0);
    });
}

int kmp_partition(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt, int32_t n,
                  int64_t m, int32_t k, double epsilon, uint64_t seed, int32_t* out_part, void* stream)
{
    return kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, n, m, k, epsilon, seed, out_part, stream, nullptr, nullptr);
}

int kmp_partition_batch(const kmp_graph_desc* graphs, int32_t count, kmp_job_result* results, void* stream,
                        const kmp_options* opt, kmp_stats* stats)
{
    if (stats) memset(stats, 0, sizeof(*stats));
    if (count < 0 || (count > 0 && !graphs)) return KMP_EINVAL;
    if (count == 0) return KMP_OK;
    return run_batch(graphs, count, results, (hipStream_t)stream, opt, stats);
}

int kmp_set_tuning(const kmp_tuning* t)
{
    Tuning u;
    if (t) {
        u.small_level_n = t->small_level_n;
        u.cut[0] = t->tier0_deg;
        u.cut[1] = t->tier1_deg;
        u.cut[2] = t->tier2_deg;
        u.cut[3] = t->tier3_deg;
        u.hub_ts = t->hub_lds_slots ? t->hub_lds_slots : 4096;
        if (!tuning_valid(u)) return KMP_EINVAL;
    }
    tuning_set(u);
    return KMP_OK;
}

int kmp_get_tuning(kmp_tuning* t)
{
    if (!t) return KMP_EINVAL;
    const Tuning u = tuning_get();
    memset(t, 0, sizeof(*t));
    t->small_level_n = u.small_level_n;
    t->tier0_deg = u.cut[0];
    t->tier1_deg = u.cut[1];
    t->tier2_deg = u.cut[2];
    t->tier3_deg = u.cut[3];
    t->hub_lds_slots = u.hub_ts;
    return KMP_OK;
}

int kmp_autotune(const kmp_graph_desc* graph, int32_t reps, void* stream, kmp_tuning* chosen,
                 kmp_autotune_report* report)
{
    if (report) memset(report, 0, sizeof(*report));
    if (!graph || reps < 1 || reps > 50) return KMP_EINVAL;
    const int rc = check_args(graph->xadj, graph->n, graph->m, graph->k, graph->epsilon, graph->out_part);
    if (rc != KMP_OK) return rc;
    if (graph->n == 0) return KMP_EINVAL;
    return (int)guarded([&]() -> int64_t { return autotune_impl(*graph, reps, (hipStream_t)stream, chosen, report); });
}

const char* kmp_strerror(int code)
{
    switch (code) {
        case KMP_OK: return "ok";
        case KMP_IMBALANCED: return "partition written, but a block exceeds the balance bound";
        case KMP_EINVAL: return "invalid argument";
        case KMP_EGRAPH: return "invalid graph";
        case KMP_EOVERFLOW: return "weight sum exceeds int32";
        case KMP_ENOMEM: return "device memory allocation failed";
        case KMP_EHIP: return "HIP runtime error";
        case KMP_ETOOLARGE: return "input beyond the size limits of the allocation-free entry point";
        default: return "unknown status";
    }
}

const char* kmp_version(void) { return "0.1.0"; }

int kmp_lp_cluster(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt, int32_t n,
                   int32_t level, int64_t U, uint64_t seed, int32_t* label, int64_t* cw, uint32_t* fav,
                   int64_t* moves, void* stream)
{
    if (n < 0 || (n > 0 && (!xadj || !label || !cw || !fav))) return KMP_EINVAL;
    if (moves)
        for (int r = 0; r < kRounds; ++r) moves[r] = 0;
    if (n == 0) return 0;
    return (int)guarded([&]() -> int64_t {
        hipStream_t s = (hipStream_t)stream;
        init_pool_once();
        Ctx c(s);
        DGraph g = make_graph(xadj, adjncy, vwgt, adjwgt, n, 0);
        int32_t m32 = 0;
        c.read(&m32, xadj + n, sizeof(int32_t));
        g.m = m32;
        LPSchedule sched;
        lp_build_schedule(c, g, level, seed, sched);
        hipLaunchKernelGGL(k_iota_weights, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, vwgt, n, label, cw, fav);
        KMP_LAUNCH_CHECK();
        LPState ls{label, cw, n, nullptr, U, fav, TAG_CL};
        LPStats r = lp_run(c, g, level, seed, &sched, ls);
        c.sync();
        if (moves)
            for (int q = 0; q < kRounds; ++q) moves[q] = r.moves[q];
        return r.rounds;
    });
}

int64_t kmp_two_hop(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt, int32_t n,
                    int64_t U, int32_t* label, int64_t* cw, const uint32_t* fav, void* stream)
{
    if (n < 0 || (n > 0 && (!xadj || !label || !cw || !fav))) return KMP_EINVAL;
    if (n == 0) return 0;
    return guarded([&]() -> int64_t {
        init_pool_once();
        Ctx c((hipStream_t)stream);
        DGraph g = make_graph(xadj, adjncy, vwgt, adjwgt, n, 0);
        int64_t r = two_hop(c, g, U, label, cw, fav);
        c.sync();
        return r;
    });
}

int kmp_contract(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt, int32_t n,
                 const int32_t* label, int32_t* map, int32_t* cn, int64_t* cm, int32_t* cxadj, int32_t* cadjncy,
                 int32_t* cvwgt, int32_t* cadjwgt, void* stream)
{
    if (n < 0 || !cn || !cm || (n > 0 && (!xadj || !label || !map || !cxadj || !cvwgt))) return KMP_EINVAL;
    if (n == 0) {
        *cn = 0;
        *cm = 0;
        return KMP_OK;
    }
    return (int)guarded([&]() -> int64_t {
        init_pool_once();
        Ctx c((hipStream_t)stream);
        int32_t m32 = 0;
        c.read(&m32, xadj + n, sizeof(int32_t));
        DGraph g = make_graph(xadj, adjncy, vwgt, adjwgt, n, m32);
        // cluster weights from the labels
        DBuf<int64_t> cw(c, (size_t)n);
        DBuf<int32_t> lab(c, (size_t)n);
        KMP_HIP(hipMemcpyAsync(lab.p, label, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, c.stream));
        block_weights(c, g, lab.p, n, cw.p);
        OwnedGraph og;
        int32_t ncn = 0;
        int64_t ncm = 0;
        contract(c, g, lab.p, cw.p, map, og, ncn, ncm);
        KMP_HIP(hipMemcpyAsync(cxadj, og.xadj.p, sizeof(int32_t) * ((size_t)ncn + 1), hipMemcpyDeviceToDevice,
                               c.stream));
        KMP_HIP(hipMemcpyAsync(cvwgt, og.vwgt.p, sizeof(int32_t) * (size_t)ncn, hipMemcpyDeviceToDevice, c.stream));
        if (ncm > 0) {
            KMP_HIP(hipMemcpyAsync(cadjncy, og.adjncy.p, sizeof(int32_t) * ncm, hipMemcpyDeviceToDevice, c.stream));
            KMP_HIP(hipMemcpyAsync(cadjwgt, og.adjwgt.p, sizeof(int32_t) * ncm, hipMemcpyDeviceToDevice, c.stream));
        }
        c.sync();
        *cn = ncn;
        *cm = ncm;
        return KMP_OK;
    });
}

int kmp_bipartition_round(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt,
                          int32_t n, int32_t level, int32_t* part, int32_t* nblocks, int32_t* first, int32_t* fcount,
                          int64_t lk, uint64_t seed, void* stream)
{
    return kmp_bipartition_round_ex(xadj, adjncy, vwgt, adjwgt, n, level, part, nblocks, first, fcount, lk, seed, 0,
                                    0, stream);
}

int kmp_bipartition_round_ex(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt,
                             int32_t n, int32_t level, int32_t* part, int32_t* nblocks, int32_t* first,
                             int32_t* fcount, int64_t lk, uint64_t seed, int32_t fm_passes, int32_t ip_pool,
                             void* stream)
{
    if (n < 0 || !nblocks || *nblocks < 1 || !first || !fcount || (n > 0 && (!xadj || !part))) return KMP_EINVAL;
    if (fm_passes < 0 || fm_passes > kFmMaxPasses || (ip_pool != 0 && ip_pool != 1)) return KMP_EINVAL;
    return (int)guarded([&]() -> int64_t {
        init_pool_once();
        Ctx c((hipStream_t)stream);
        c.fm_passes = fm_passes;
        c.ip_pool = ip_pool != 0;
        int32_t m32 = 0;
        if (n > 0) c.read(&m32, xadj + n, sizeof(int32_t));
        DGraph g = make_graph(xadj, adjncy, vwgt, adjwgt, n, m32);
        BlockTab bt;
        bt.first.assign(first, first + *nblocks);
        bt.f.assign(fcount, fcount + *nblocks);
        bt.job.assign(*nblocks, 0);
        std::vector<uint8_t> split(*nblocks);
        for (int32_t b = 0; b < *nblocks; ++b) split[b] = bt.f[b] >= 2;
        bipartition_round(c, g, level, part, bt, split, std::vector<int64_t>{lk},
                          std::vector<uint32_t>{seed_hash(seed)});
        c.sync();
        for (int32_t i = 0; i < bt.size(); ++i) {
            first[i] = bt.first[i];
            fcount[i] = bt.f[i];
        }
        *nblocks = bt.size();
        return KMP_OK;
    });
}

int kmp_balance(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt, int32_t n,
                int32_t level, uint64_t seed, int32_t* part, int64_t* wt, int32_t nb, const int64_t* cap,
                void* stream)
{
    return kmp_balance_ex(xadj, adjncy, vwgt, adjwgt, n, level, seed, part, wt, nb, cap, 0, stream);
}

int kmp_balance_ex(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt,
                   int32_t n, int32_t level, uint64_t seed, int32_t* part, int64_t* wt, int32_t nb,
                   const int64_t* cap, int32_t pq, void* stream)
{
    if (n < 0 || nb < 1 || (n > 0 && (!xadj || !part || !wt || !cap)) || (pq != 0 && pq != 1)) return KMP_EINVAL;
    if (n == 0) return 0;
    return (int)guarded([&]() -> int64_t {
        init_pool_once();
        Ctx c((hipStream_t)stream);
        int32_t m32 = 0;
        c.read(&m32, xadj + n, sizeof(int32_t));
        DGraph g = make_graph(xadj, adjncy, vwgt, adjwgt, n, m32);
        LPSchedule sched;
        lp_build_schedule(c, g, level, seed, sched);
        BlockTab bt;
        bt.first.assign(nb, 0);
        bt.f.assign(nb, 1);
        bt.job.assign(nb, 0);
        int32_t r = (pq ? balance_pq : balance)(c, g, level, std::vector<uint64_t>{seed},
                                                [&]() -> const LPSchedule& { return sched; }, part, wt, bt, cap,
                                                JobTabs{}, nullptr, nullptr);
        c.sync();
        return r;
    });
}

int kmp_lp_refine(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt, int32_t n,
                  int32_t level, uint64_t seed, int32_t* part, int64_t* wt, int32_t nb, const int64_t* cap,
                  int64_t* moves, void* stream)
{
    if (n < 0 || nb < 1 || (n > 0 && (!xadj || !part || !wt || !cap))) return KMP_EINVAL;
    if (moves)
        for (int r = 0; r < kRounds; ++r) moves[r] = 0;
    if (n == 0) return 0;
    return (int)guarded([&]() -> int64_t {
        init_pool_once();
        Ctx c((hipStream_t)stream);
        int32_t m32 = 0;
        c.read(&m32, xadj + n, sizeof(int32_t));
        DGraph g = make_graph(xadj, adjncy, vwgt, adjwgt, n, m32);
        LPSchedule sched;
        lp_build_schedule(c, g, level, seed, sched);
        LPState ls{part, wt, nb, cap, 0, nullptr, TAG_REF};
        LPStats r = lp_run(c, g, level, seed, &sched, ls);
        c.sync();
        if (moves)
            for (int q = 0; q < kRounds; ++q) moves[q] = r.moves[q];
        return r.rounds;
    });
}

int64_t kmp_lp_subround(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt,
                        int32_t n, int32_t level, int32_t round, int32_t s, uint32_t tag, uint64_t seed,
                        int32_t* label, int64_t* wt, int32_t nlab, const int64_t* cap_vec, int64_t cap_scalar,
                        const uint8_t* active, uint32_t* fav, uint8_t* moved, void* stream)
{
    if (n < 0 || nlab < 1 || s < 0 || s >= kSub || (n > 0 && (!xadj || !label || !wt || !moved))) return KMP_EINVAL;
    if (n == 0) return 0;
    return guarded([&]() -> int64_t {
        init_pool_once();
        Ctx c((hipStream_t)stream);
        int32_t m32 = 0;
        c.read(&m32, xadj + n, sizeof(int32_t));
        DGraph g = make_graph(xadj, adjncy, vwgt, adjwgt, n, m32);
        LPSchedule sched;
        lp_build_schedule(c, g, level, seed, sched);
        LPState ls{label, wt, nlab, cap_vec, cap_scalar, fav, tag};
        int64_t r = lp_subround(c, g, level, round, s, seed, sched, ls, active, moved);
        c.sync();
        return r;
    });
}

int kmp_lp_async(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt, int32_t n,
                 int32_t level, uint32_t tag, uint64_t seed, int32_t* label, int64_t* wt, int32_t nlab,
                 const int64_t* cap_vec, int64_t cap_scalar, uint32_t* fav, int64_t* moves, int32_t serial,
                 void* stream)
{
    if (n < 0 || nlab < 1 || (tag != TAG_CL && tag != TAG_REF) || (serial != 0 && serial != 1) ||
        (n > 0 && (!xadj || !label || !wt)))
        return KMP_EINVAL;
    if (moves)
        for (int r = 0; r < kRounds; ++r) moves[r] = 0;
    if (n == 0) return 0;
    return (int)guarded([&]() -> int64_t {
        init_pool_once();
        Ctx c((hipStream_t)stream);
        c.async_lp = serial ? 2 : 1;
        int32_t m32 = 0;
        c.read(&m32, xadj + n, sizeof(int32_t));
        DGraph g = make_graph(xadj, adjncy, vwgt, adjwgt, n, m32);
        LPSchedule sched;
        lp_build_async_schedule(c, g, level, seed, sched);
        LPState ls{label, wt, nlab, cap_vec, cap_scalar, fav, tag};
        LPStats r = lp_run(c, g, level, seed, &sched, ls);
        c.sync();
        if (moves)
            for (int q = 0; q < kRounds; ++q) moves[q] = r.moves[q];
        return r.rounds;
    });
}

// ---------------------------------------------------------------- allocation-free entry point
// The scratch region of kmp_partition_noalloc: one copy per device, loaded
// with the code object.  Host code never passes this name to a kernel (on the
// host it is a stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[KMP_NOALLOC_SCRATCH_BYTES];

int kmp_partition_noalloc(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt,
                          int32_t n, int64_t m, int32_t k, double epsilon, uint64_t seed, int32_t* out_part,
                          void* stream, const kmp_options* opt, kmp_stats* stats)
{
    if (stats) memset(stats, 0, sizeof(*stats));
    int rc = check_args(xadj, n, m, k, epsilon, out_part);
    if (rc != KMP_OK) return rc;
    if (n > KMP_NOALLOC_MAX_N || m > KMP_NOALLOC_MAX_M) return KMP_ETOOLARGE;
    if (opt && opt->profile) return KMP_EINVAL;  // profiling records events, which the runtime allocates
    if (n == 0) return m == 0 ? KMP_OK : KMP_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return KMP_EHIP;
    std::lock_guard<std::mutex> lk(g_noalloc_mu[dev]);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return KMP_EHIP;
        }
        g_noalloc_ptr[dev] = p;
    }
    return (int)guarded([&]() -> int64_t {
        return partition_impl(make_graph(xadj, adjncy, vwgt, adjwgt, n, m), k, epsilon, seed, out_part,
                              (hipStream_t)stream, opt, stats, g_noalloc_ptr[dev], (size_t)KMP_NOALLOC_SCRATCH_BYTES);
    });
}

}  // extern "C"
