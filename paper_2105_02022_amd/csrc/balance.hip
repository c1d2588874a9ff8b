// k-way balancer (paper Sec. 5.3 "Balancing"): move just enough nodes out of
// every overloaded block, preferring high relative gain, into blocks that can
// take them.
//
// Deterministic reading, per round:
//   * target of a node v in an overloaded block b: the adjacent non-overloaded
//     block with the largest connection that still fits (ties by hash, then
//     index); otherwise the non-overloaded block with the most free capacity,
//     if it fits;
//   * d = conn(v, target) - conn(v, b); relative gain rg = d*c(v) if d >= 0,
//     d/c(v) otherwise;
//   * per overloaded block, candidates ordered by (rg desc, id asc); the
//     shortest prefix whose weight covers the overload is selected;
//   * selected moves into one target are admitted in ascending id while the
//     target stays within its cap.
// Sorting by rg is exact: d >= 0 sorts by the 62-bit integer d*c; d < 0 by
// (floor(|d|/c), floor(2^62 (|d| mod c) / c)); two distinct fractions with
// denominators below 2^31 differ by more than 2^-62, so the second word
// separates them.
//
// Queue balancer (kmp_options.pq_balance; the paper's own mechanics): per
// pass, for every overloaded block in ascending index, a queue of just enough
// of its nodes ordered by relative gain (larger first, then smaller id) is
// filled from the candidates of the pass start in ascending id (a node enters
// while the queue weighs less than the excess, later only if it beats the
// queue's lowest node, after which the lowest nodes leave while the queue
// weighs more than the excess plus the heaviest node weight); then the best
// node is taken while the block is overloaded: its target and gain are
// recomputed against the current weights; if the gain changed or its target
// can no longer take it, it is offered again if it is a border node, else it
// moves, and its neighbours still in the block that are neither queued nor
// offered before in this pass are offered in row order.  Jobs of a batch are
// independent: one workgroup per job; within a job the steps are sequential,
// with the workgroup's lanes over a node's row and over the queue.
#include "kmp_dev.h"
#include "pq_pass.h"

namespace kmp {

namespace {

// tstar: fallback block (one graph); batches: gtstar[bjob[b]] per job
__global__ void k_bal_candidates(const int32_t* __restrict__ part, const uint8_t* __restrict__ over,
                                 const int32_t* __restrict__ vwgt, int32_t n, int32_t tstar,
                                 const int32_t* __restrict__ bjob, const int32_t* __restrict__ gtstar,
                                 const int64_t* __restrict__ wt, const int64_t* __restrict__ cap,
                                 int32_t* __restrict__ bal_t, const int64_t* __restrict__ bal_d,
                                 int32_t* __restrict__ flag, uint32_t* __restrict__ kw0, uint32_t* __restrict__ kw1,
                                 uint32_t* __restrict__ kw2, uint32_t* __restrict__ kcls)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int32_t ok = 0;
    const int32_t b = part[v];
    if (over[b]) {
        const int64_t c = vwgt ? vwgt[v] : 1;
        int32_t t = bal_t[v];
        int64_t d = bal_d[v];  // -conn(own) when there is no adjacent target
        const int32_t ts = bjob ? gtstar[bjob[b]] : tstar;
        if (t < 0 && ts >= 0 && wt[ts] + c <= cap[ts]) t = ts;
        bal_t[v] = t;
        if (t >= 0) {
            ok = 1;
            uint32_t w0, w1, w2, cls;
            if (d >= 0) {
                const uint64_t key = ~((uint64_t)d * (uint64_t)c);  // descending d*c
                cls = 0;
                w0 = (uint32_t)(key >> 32);
                w1 = (uint32_t)key;
                w2 = 0;
            } else {
                const uint64_t ad = (uint64_t)(-d);
                const uint64_t q = ad / (uint64_t)c, r = ad % (uint64_t)c;
                const unsigned __int128 num = (unsigned __int128)r << 62;
                const uint64_t frac = (uint64_t)(num / (unsigned __int128)(uint64_t)c);
                cls = 1;
                w0 = (uint32_t)q;
                w1 = (uint32_t)(frac >> 32);
                w2 = (uint32_t)frac;
            }
            kw0[v] = w0;
            kw1[v] = w1;
            kw2[v] = w2;
            kcls[v] = cls;
        }
    }
    flag[v] = ok;
}

__global__ void k_compact_ids(const int32_t* __restrict__ flag, const int32_t* __restrict__ pos, int32_t n,
                              uint32_t* __restrict__ out)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && flag[v]) out[pos[v]] = (uint32_t)v;
}

__global__ void k_gather_key(const uint32_t* __restrict__ kw, const uint32_t* __restrict__ ids, int64_t nc,
                             uint32_t* __restrict__ keys)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nc) keys[i] = kw[ids[i]];
}

__global__ void k_gather_block(const int32_t* __restrict__ part, const uint32_t* __restrict__ ids, int64_t nc,
                               uint32_t* __restrict__ keys)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nc) keys[i] = (uint32_t)part[ids[i]];
}

__global__ void k_gather_weight(const uint32_t* __restrict__ ids, const int32_t* __restrict__ vwgt, int64_t nc,
                                int64_t* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nc) out[i] = vwgt ? vwgt[ids[i]] : 1;
}

// per block of the sorted list: weight before the element (exclusive)
__global__ void k_seg_base(const uint32_t* __restrict__ blk, const int64_t* __restrict__ pre,
                           const int64_t* __restrict__ cw, int64_t nc, int64_t* __restrict__ base)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nc && (i == 0 || blk[i] != blk[i - 1])) base[blk[i]] = pre[i] - cw[i];
}

__global__ void k_select(const uint32_t* __restrict__ ids, const uint32_t* __restrict__ blk,
                         const int64_t* __restrict__ pre, const int64_t* __restrict__ cw,
                         const int64_t* __restrict__ base, int64_t nc, const int64_t* __restrict__ wt,
                         const int64_t* __restrict__ cap, uint8_t* __restrict__ sel)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc) return;
    const uint32_t b = blk[i];
    const int64_t before = pre[i] - cw[i] - base[b];
    sel[ids[i]] = before < wt[b] - cap[b];
}

__global__ void k_sel_flags(const uint8_t* __restrict__ sel, int32_t n, int32_t* __restrict__ flag)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) flag[v] = sel[v];
}

__global__ void k_sel_compact(const uint8_t* __restrict__ sel, const int32_t* __restrict__ pos, int32_t n,
                              const int32_t* __restrict__ bal_t, uint32_t* __restrict__ keys,
                              uint32_t* __restrict__ vals)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && sel[v]) {
        keys[pos[v]] = (uint32_t)bal_t[v];
        vals[pos[v]] = (uint32_t)v;
    }
}

__global__ void k_admit_decide(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                               const int64_t* __restrict__ pre, const int64_t* __restrict__ base, int64_t ns,
                               const int64_t* __restrict__ wt, const int64_t* __restrict__ cap,
                               uint8_t* __restrict__ adm)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    const uint32_t t = keys[i];
    adm[i] = wt[t] + (pre[i] - base[t]) <= cap[t];
}

// moves are counted per block-of-threads into spread slots (one graph) or per
// job (batches: bjob != NULL)
__global__ __launch_bounds__(kBlock) void k_bal_apply(const uint32_t* __restrict__ keys,
                                                      const uint32_t* __restrict__ vals,
                                                      const uint8_t* __restrict__ adm, int64_t ns,
                                                      const int32_t* __restrict__ vwgt, int32_t* __restrict__ part,
                                                      int64_t* __restrict__ wt, const int32_t* __restrict__ bjob,
                                                      int64_t* counter)
{
    __shared__ int32_t bm;
    if (threadIdx.x == 0) bm = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t j = -1;
    if (i < ns && adm[i]) {
        const int32_t v = (int32_t)vals[i];
        const int32_t t = (int32_t)keys[i];
        const int64_t c = vwgt ? vwgt[v] : 1;
        const int32_t b = part[v];
        part[v] = t;
        atomicAdd((unsigned long long*)&wt[t], (unsigned long long)c);
        atomicAdd((unsigned long long*)&wt[b], (unsigned long long)(-c));
        j = bjob ? bjob[t] : 0;
        if (!bjob) atomicAdd(&bm, 1);
    }
    if (bjob) {
        job_add(counter, j, 1);
    } else {
        __syncthreads();
        if (threadIdx.x == 0 && bm) spread_add(counter, bm);
    }
}


// ---------------------------------------------------------------- queue balancer
// One thread per job runs the pass (pq_pass.h): the queues of a job depend on
// each other through the block weights, block by block, so a job's pass is
// sequential; the jobs of a batch run side by side.  The pass-start targets and
// gains come from the parallel balance-mode rating.
struct PQArgs {
    const int32_t* xadj;
    const int32_t* adjncy;
    const int32_t* vwgt;
    const int32_t* adjwgt;
    int32_t* part;
    int64_t* wt;
    const int64_t* cap;
    const int32_t* job_b0;     // [njobs + 1] first block of each job
    const uint32_t* hpre;      // [njobs] H prefix over (seed_job; T_BAL, level, pass)
    const uint8_t* job_on;     // [njobs] job takes part in this pass
    const int32_t* maxc;       // [njobs] heaviest node of the job
    const uint8_t* over;       // [nb] overloaded at the pass start
    const uint32_t* cand_blk;  // [ncand] candidates sorted by (block, id)
    const uint32_t* cand_id;
    int32_t ncand;
    const int32_t* bal_t;      // pass-start targets and gains of the candidates
    const int64_t* bal_d;
    PQItem* q;                 // queue storage, block b at qoff[b]
    const int32_t* qoff;       // [nb + 1]
    uint8_t* inq;              // [n] queued now
    uint8_t* tried;            // [n] offered as a neighbour in this pass (zeroed before the pass)
    int64_t* conn;             // [nb] zero between uses
    int32_t* touched;          // [nb] scratch list per job (its block range)
    int64_t* moved;            // [njobs] moves of the pass
    int32_t* full;             // set if a queue ran out of room (a broken invariant)
};

__global__ __launch_bounds__(64) void k_pq_pass_seq(PQArgs a)
{
    const int32_t j = blockIdx.x;
    if (threadIdx.x != 0 || !a.job_on[j]) return;
    PQJob J;
    J.xadj = a.xadj;
    J.adjncy = a.adjncy;
    J.vwgt = a.vwgt;
    J.adjwgt = a.adjwgt;
    J.part = a.part;
    J.wt = a.wt;
    J.cap = a.cap;
    J.b0 = a.job_b0[j];
    J.b1 = a.job_b0[j + 1];
    J.hpre = a.hpre[j];
    J.maxc = a.maxc[j];
    J.over = a.over;
    J.cand_blk = a.cand_blk;
    J.cand_id = a.cand_id;
    J.ncand = a.ncand;
    J.bal_t = a.bal_t;
    J.bal_d = a.bal_d;
    J.qs = a.q;
    J.qoff = a.qoff;
    J.inq = a.inq;
    J.tried = a.tried;
    J.conn = a.conn;
    J.touched = a.touched + J.b0;
    J.full = a.full;
    a.moved[j] = pq_pass_job(J);
}

__global__ void k_block_nodes(const int32_t* __restrict__ part, int32_t n, int32_t* __restrict__ cnt)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) atomicAdd(&cnt[part[v]], 1);
}

__global__ void k_job_maxc(const int32_t* __restrict__ vwgt, const int32_t* __restrict__ gid, int32_t n,
                           int32_t* __restrict__ maxc)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) atomicMax(&maxc[gid ? gid[v] : 0], vwgt ? vwgt[v] : 1);
}

}  // namespace

int32_t balance_pq(Ctx& c, const DGraph& g, int32_t level, const std::vector<uint64_t>& seeds,
                   const std::function<const LPSchedule&()>& sched, int32_t* part, int64_t* wt, const BlockTab& bt,
                   const int64_t* cap, const JobTabs& jt, const int32_t* boff, const std::vector<int64_t>* hcap_in)
{
    const int32_t n = g.n;
    const int32_t nb = bt.size();
    const int32_t njobs = (int32_t)seeds.size();
    const bool batch = jt.gid != nullptr;
    if (n == 0 || nb == 0) return 0;
    std::vector<int64_t> hcap, hwt(nb);
    if (hcap_in) {
        hcap = *hcap_in;
    } else {
        hcap.resize(nb);
        c.read(hcap.data(), cap, sizeof(int64_t) * nb);
    }
    // blocks of job j: [b0[j], b0[j + 1]) (a job's blocks are contiguous)
    std::vector<int32_t> hb0(njobs + 1, nb);
    for (int32_t b = nb - 1; b >= 0; --b) hb0[batch ? bt.job[b] : 0] = b;
    for (int32_t j = njobs - 1; j >= 0; --j)
        if (hb0[j] > hb0[j + 1]) hb0[j] = hb0[j + 1];  // jobs without blocks: empty range
    std::vector<uint8_t> hover(nb), active(njobs, 1), any(njobs), on(njobs);
    std::vector<int32_t> tstar(njobs);
    std::vector<int64_t> moved(njobs);
    std::vector<uint32_t> hpre(njobs);
    DBuf<uint8_t> over(c, (size_t)nb), don(c, (size_t)njobs), inq(c, (size_t)n), tried(c, (size_t)n);
    DBuf<int32_t> bal_t(c, (size_t)n), flag(c, (size_t)n + 1), pos(c, (size_t)n + 1), dbjob, dtstar;
    DBuf<int32_t> db0(c, (size_t)njobs + 1), maxc(c, (size_t)njobs), qoff(c, (size_t)nb + 1);
    DBuf<int32_t> touched(c, (size_t)nb);
    DBuf<int64_t> bal_d(c, (size_t)n), conn(c, (size_t)nb), dmoved(c, (size_t)njobs);
    DBuf<uint32_t> kw0(c, (size_t)n), kw1(c, (size_t)n), kw2(c, (size_t)n), kcls(c, (size_t)n), dhpre(c, (size_t)njobs);
    DBuf<PQItem> q(c, (size_t)std::max(n, 1));
    DBuf<int32_t> dfull(c, 1);
    c.write(db0.p, hb0.data(), sizeof(int32_t) * (njobs + 1));
    fill_bytes_many(c, {{inq.p, (int64_t)n, 0}, {conn.p, 8 * (int64_t)nb, 0}, {maxc.p, 4 * (int64_t)njobs, 0},
                        {dfull.p, 4, 0}});
    hipLaunchKernelGGL(k_job_maxc, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, g.vwgt, jt.gid, n, maxc.p);
    KMP_LAUNCH_CHECK();
    if (batch) {
        dbjob = DBuf<int32_t>(c, (size_t)nb);
        c.write(dbjob.p, bt.job.data(), sizeof(int32_t) * nb);
        dtstar = DBuf<int32_t>(c, (size_t)njobs);
    }
    int32_t pass = 0;
    for (;;) {
        c.read(hwt.data(), wt, sizeof(int64_t) * nb);
        std::fill(any.begin(), any.end(), 0);
        std::fill(tstar.begin(), tstar.end(), -1);
        for (int32_t b = 0; b < nb; ++b) {
            const int32_t j = batch ? bt.job[b] : 0;
            const bool ov = hwt[b] > hcap[b];
            any[j] |= ov;
            if (!ov && (tstar[j] < 0 || hcap[b] - hwt[b] > hcap[tstar[j]] - hwt[tstar[j]])) tstar[j] = b;
        }
        bool go = false;
        for (int32_t j = 0; j < njobs; ++j) {
            active[j] = active[j] && any[j];
            on[j] = active[j];
            go |= active[j] != 0;
            hpre[j] = hash_prefix(seeds[j], {TAG_BAL, (uint32_t)level, (uint32_t)pass});
        }
        if (!go) break;
        for (int32_t b = 0; b < nb; ++b) hover[b] = hwt[b] > hcap[b] && active[batch ? bt.job[b] : 0];
        c.write(over.p, hover.data(), (size_t)nb);
        c.write(don.p, on.data(), (size_t)njobs);
        c.write(dhpre.p, hpre.data(), sizeof(uint32_t) * njobs);
        if (batch) c.write(dtstar.p, tstar.data(), sizeof(int32_t) * njobs);
        // pass-start targets and gains of the nodes of overloaded blocks
        fill_i32(c, bal_t.p, -1, n);
        rate_for_balance(c, g, level, seeds[0], pass, sched(), part, wt, cap, over.p, bal_t.p, bal_d.p, jt, boff);
        hipLaunchKernelGGL(k_bal_candidates, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, part, over.p, g.vwgt, n,
                           tstar[0], dbjob.p, dtstar.p, wt, cap, bal_t.p, bal_d.p, flag.p, kw0.p, kw1.p, kw2.p, kcls.p);
        KMP_LAUNCH_CHECK();
        scan_excl_i32(c, flag.p, pos.p, n, pos.p + n);
        const int64_t ncand = c.read1(pos.p + n);
        // candidates by (block, id)
        DBuf<uint32_t> ids(c, (size_t)std::max<int64_t>(ncand, 1)), keys(c, (size_t)std::max<int64_t>(ncand, 1));
        DBuf<uint32_t> k2(c, (size_t)std::max<int64_t>(ncand, 1)), v2(c, (size_t)std::max<int64_t>(ncand, 1));
        uint32_t* sorted_ids = ids.p;
        uint32_t* sorted_keys = keys.p;
        if (ncand > 0) {
            hipLaunchKernelGGL(k_compact_ids, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, flag.p, pos.p, n, ids.p);
            KMP_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_gather_block, dim3(grid_for(ncand)), dim3(kBlock), 0, c.stream, part, ids.p, ncand,
                               keys.p);
            KMP_LAUNCH_CHECK();
            radix_sort_pairs(c, keys.p, ids.p, k2.p, v2.p, ncand, bits_for((uint64_t)(nb - 1)), &sorted_keys,
                             &sorted_ids);
        }
        // queue storage: block b holds at most its pass-start nodes
        fill_bytes_many(c, {{qoff.p, 4 * ((int64_t)nb + 1), 0}, {tried.p, (int64_t)n, 0},
                            {dmoved.p, 8 * (int64_t)njobs, 0}});
        hipLaunchKernelGGL(k_block_nodes, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, part, n, qoff.p);
        KMP_LAUNCH_CHECK();
        scan_excl_i32(c, qoff.p, qoff.p, nb, qoff.p + nb);
        PQArgs a;
        a.xadj = g.xadj;
        a.adjncy = g.adjncy;
        a.vwgt = g.vwgt;
        a.adjwgt = g.adjwgt;
        a.part = part;
        a.wt = wt;
        a.cap = cap;
        a.job_b0 = db0.p;
        a.hpre = dhpre.p;
        a.job_on = don.p;
        a.maxc = maxc.p;
        a.over = over.p;
        a.cand_blk = sorted_keys;
        a.cand_id = sorted_ids;
        a.ncand = (int32_t)ncand;
        a.bal_t = bal_t.p;
        a.bal_d = bal_d.p;
        a.q = q.p;
        a.qoff = qoff.p;
        a.inq = inq.p;
        a.tried = tried.p;
        a.conn = conn.p;
        a.touched = touched.p;
        a.moved = dmoved.p;
        a.full = dfull.p;
        {
            ProfScope ps(c, KMP_PROF_BALANCE);
            hipLaunchKernelGGL(k_pq_pass_seq, dim3(njobs), dim3(64), 0, c.stream, a);
            KMP_LAUNCH_CHECK();
        }
        c.read(moved.data(), dmoved.p, sizeof(int64_t) * njobs);
        for (int32_t j = 0; j < njobs; ++j) active[j] = active[j] && moved[j] > 0;
        ++pass;
    }
    if (pass > 0 && c.read1(dfull.p)) throw Error(KMP_EHIP, "queue balancer: a queue ran out of room");
    return pass;
}

int32_t balance(Ctx& c, const DGraph& g, int32_t level, const std::vector<uint64_t>& seeds,
                const std::function<const LPSchedule&()>& sched, int32_t* part, int64_t* wt, const BlockTab& bt,
                const int64_t* cap, const JobTabs& jt, const int32_t* boff, const std::vector<int64_t>* hcap_in)
{
    const int32_t n = g.n;
    const int32_t nb = bt.size();
    const int32_t njobs = (int32_t)seeds.size();
    const bool batch = jt.gid != nullptr;
    if (n == 0 || nb == 0) return 0;
    std::vector<int64_t> hcap, hwt(nb);
    if (hcap_in) {
        hcap = *hcap_in;
    } else {
        hcap.resize(nb);
        c.read(hcap.data(), cap, sizeof(int64_t) * nb);
    }
    std::vector<uint8_t> hover(nb), active(njobs, 1), any(njobs);
    std::vector<int32_t> tstar(njobs);
    std::vector<int64_t> moved(njobs);
    int32_t round = 0;
    DBuf<uint8_t> over, sel;
    DBuf<int32_t> bal_t, flag, dbjob, dtstar;
    DBuf<int64_t> bal_d, dmoved;
    DBuf<uint32_t> kw0, kw1, kw2, kcls;
    for (;;) {
        c.read(hwt.data(), wt, sizeof(int64_t) * nb);
        // per job: overloaded blocks, fallback block (most free capacity, smallest index)
        std::fill(any.begin(), any.end(), 0);
        std::fill(tstar.begin(), tstar.end(), -1);
        for (int32_t b = 0; b < nb; ++b) {
            const int32_t j = batch ? bt.job[b] : 0;
            const bool ov = hwt[b] > hcap[b];
            any[j] |= ov;
            if (!ov && (tstar[j] < 0 || hcap[b] - hwt[b] > hcap[tstar[j]] - hwt[tstar[j]])) tstar[j] = b;
        }
        bool go = false;
        for (int32_t j = 0; j < njobs; ++j) {
            active[j] = active[j] && any[j];  // a job stops for good: no overload, or no move last round
            go |= active[j] != 0;
        }
        if (!go) break;
        for (int32_t b = 0; b < nb; ++b) hover[b] = hwt[b] > hcap[b] && active[batch ? bt.job[b] : 0];
        if (!over.p) {
            over = DBuf<uint8_t>(c, (size_t)nb);
            sel = DBuf<uint8_t>(c, (size_t)n);
            bal_t = DBuf<int32_t>(c, (size_t)n);
            flag = DBuf<int32_t>(c, (size_t)n + 1);
            bal_d = DBuf<int64_t>(c, (size_t)n);
            kw0 = DBuf<uint32_t>(c, (size_t)n);
            kw1 = DBuf<uint32_t>(c, (size_t)n);
            kw2 = DBuf<uint32_t>(c, (size_t)n);
            kcls = DBuf<uint32_t>(c, (size_t)n);
            if (batch) {
                dbjob = DBuf<int32_t>(c, (size_t)nb);
                c.write(dbjob.p, bt.job.data(), sizeof(int32_t) * nb);
                dtstar = DBuf<int32_t>(c, (size_t)njobs);
                dmoved = DBuf<int64_t>(c, (size_t)njobs);
            }
        }
        c.write(over.p, hover.data(), (size_t)nb);
        if (batch) c.write(dtstar.p, tstar.data(), sizeof(int32_t) * njobs);
        fill_i32(c, bal_t.p, -1, n);
        rate_for_balance(c, g, level, seeds[0], round, sched(), part, wt, cap, over.p, bal_t.p, bal_d.p, jt, boff);
        hipLaunchKernelGGL(k_bal_candidates, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, part, over.p, g.vwgt, n,
                           tstar[0], dbjob.p, dtstar.p, wt, cap, bal_t.p, bal_d.p, flag.p, kw0.p, kw1.p, kw2.p, kcls.p);
        KMP_LAUNCH_CHECK();
        DBuf<int32_t> pos(c, (size_t)n + 1);
        scan_excl_i32(c, flag.p, pos.p, n, pos.p + n);
        const int64_t ncand = c.read1(pos.p + n);
        std::fill(moved.begin(), moved.end(), 0);
        if (ncand > 0) {
            // candidate ids in ascending order
            DBuf<uint32_t> ids(c, ncand), keys(c, ncand), k2(c, ncand), v2(c, ncand);
            hipLaunchKernelGGL(k_compact_ids, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, flag.p, pos.p, n, ids.p);
            KMP_LAUNCH_CHECK();
            // LSD: least significant key word first, block last
            const uint32_t* words[4] = {kw2.p, kw1.p, kw0.p, kcls.p};
            const int wbits[4] = {32, 32, 32, 1};
            for (int w = 0; w < 4; ++w) {
                hipLaunchKernelGGL(k_gather_key, dim3(grid_for(ncand)), dim3(kBlock), 0, c.stream, words[w], ids.p,
                                   ncand, keys.p);
                KMP_LAUNCH_CHECK();
                radix_sort_pairs(c, keys.p, ids.p, k2.p, v2.p, ncand, wbits[w]);
            }
            hipLaunchKernelGGL(k_gather_block, dim3(grid_for(ncand)), dim3(kBlock), 0, c.stream, part, ids.p, ncand,
                               keys.p);
            KMP_LAUNCH_CHECK();
            radix_sort_pairs(c, keys.p, ids.p, k2.p, v2.p, ncand, bits_for((uint64_t)(nb - 1)));
            // "just enough" prefix per overloaded block
            DBuf<int64_t> cw(c, ncand), pre(c, ncand), base(c, (size_t)nb);
            hipLaunchKernelGGL(k_gather_weight, dim3(grid_for(ncand)), dim3(kBlock), 0, c.stream, ids.p, g.vwgt,
                               ncand, cw.p);
            KMP_LAUNCH_CHECK();
            scan_incl_i64(c, cw.p, pre.p, ncand);
            hipLaunchKernelGGL(k_seg_base, dim3(grid_for(ncand)), dim3(kBlock), 0, c.stream, keys.p, pre.p, cw.p,
                               ncand, base.p);
            KMP_LAUNCH_CHECK();
            c.zero(sel.p, (size_t)n);
            hipLaunchKernelGGL(k_select, dim3(grid_for(ncand)), dim3(kBlock), 0, c.stream, ids.p, keys.p, pre.p, cw.p,
                               base.p, ncand, wt, cap, sel.p);
            KMP_LAUNCH_CHECK();
            // admission per target in ascending id
            hipLaunchKernelGGL(k_sel_flags, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, sel.p, n, flag.p);
            KMP_LAUNCH_CHECK();
            scan_excl_i32(c, flag.p, flag.p, n, flag.p + n);
            const int64_t ns = c.read1(flag.p + n);
            if (ns > 0) {
                DBuf<uint32_t> tk(c, ns), tv(c, ns), tk2(c, ns), tv2(c, ns);
                hipLaunchKernelGGL(k_sel_compact, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, sel.p, flag.p, n,
                                   bal_t.p, tk.p, tv.p);
                KMP_LAUNCH_CHECK();
                radix_sort_pairs(c, tk.p, tv.p, tk2.p, tv2.p, ns, bits_for((uint64_t)(nb - 1)));
                DBuf<int64_t> sc(c, ns), sp(c, ns), sb(c, (size_t)nb);
                DBuf<uint8_t> adm(c, ns);
                hipLaunchKernelGGL(k_gather_weight, dim3(grid_for(ns)), dim3(kBlock), 0, c.stream, tv.p, g.vwgt, ns,
                                   sc.p);
                KMP_LAUNCH_CHECK();
                scan_incl_i64(c, sc.p, sp.p, ns);
                hipLaunchKernelGGL(k_seg_base, dim3(grid_for(ns)), dim3(kBlock), 0, c.stream, tk.p, sp.p, sc.p, ns,
                                   sb.p);
                KMP_LAUNCH_CHECK();
                hipLaunchKernelGGL(k_admit_decide, dim3(grid_for(ns)), dim3(kBlock), 0, c.stream, tk.p, tv.p, sp.p,
                                   sb.p, ns, wt, cap, adm.p);
                KMP_LAUNCH_CHECK();
                int64_t* ctr;
                if (batch) {
                    c.zero(dmoved.p, sizeof(int64_t) * njobs);
                    ctr = dmoved.p;
                } else {
                    c.zero_spread(SP_BALMOVES);
                    ctr = c.spread(SP_BALMOVES);
                }
                hipLaunchKernelGGL(k_bal_apply, dim3(grid_for(ns)), dim3(kBlock), 0, c.stream, tk.p, tv.p, adm.p, ns,
                                   g.vwgt, part, wt, dbjob.p, ctr);
                KMP_LAUNCH_CHECK();
                if (batch) c.read(moved.data(), dmoved.p, sizeof(int64_t) * njobs);
                else moved[0] = c.read_spread(SP_BALMOVES);
            }
        }
        for (int32_t j = 0; j < njobs; ++j) active[j] = active[j] && moved[j] > 0;
        ++round;
    }
    return round;
}

}  // namespace kmp
