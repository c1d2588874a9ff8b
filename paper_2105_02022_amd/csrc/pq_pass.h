// One pass of the queue balancer for one job (paper Sec. 5.3 "Balancing"; the
// rule of kmp_options.pq_balance), written as plain sequential code so that the
// same routine runs in a GPU thread (one per job, k_pq_pass_seq) and in a host
// test built with AddressSanitizer.
//
// The overloaded blocks of the job are taken in ascending index.  A block's
// queue is filled from its pass-start candidates in ascending id (each with the
// target and gain it had at the pass start): a node enters while the queue
// weighs less than the block's excess, later only if it ranks above the
// queue's lowest node, after which the lowest nodes leave while the queue weighs
// more than the excess plus the job's heaviest node.  Then, while the block is
// overloaded, the best queued node (largest relative gain, then smallest id) is
// taken, its target and gain are recomputed against the current weights; if the
// gain changed or the target can no longer take it, it is offered again when it
// still has a neighbour in another block, else it moves, and its neighbours
// still in the block that are neither queued nor offered before in this pass
// are offered in row order.  Relative gain: d c(v) for d >= 0, d / c(v) for d < 0,
// compared exactly by cross-multiplication.  The target of a node is the
// adjacent block of the largest connection that can take it (ties by the pass's
// tie-break hash of the job-local block index, then index), else the block of
// the job with the most free room (smallest index on ties) if it can take it.
#pragma once
#include "kmp_dev.h"

#ifndef KMP_HD
#define KMP_HD __host__ __device__
#endif

namespace kmp {

struct PQItem {
    int64_t d;  // cut reduction of the move (may be negative)
    int32_t c;  // node weight
    int32_t v;  // node
    int32_t t;  // designated target block
    int32_t pad;
};

// A job's view for one pass: blocks [b0, b1); arrays indexed by node or by
// global block index; qs + qoff[b] has room for the nodes of block b.
struct PQJob {
    const int32_t* xadj;
    const int32_t* adjncy;
    const int32_t* vwgt;    // NULL: unit
    const int32_t* adjwgt;  // NULL: unit
    int32_t* part;
    int64_t* wt;
    const int64_t* cap;
    int32_t b0, b1;
    uint32_t hpre;  // H prefix over (seed; T_BAL, level, pass) of the job
    int64_t maxc;   // heaviest node of the job
    const uint8_t* over;       // overloaded at the pass start
    const uint32_t* cand_blk;  // pass-start candidates sorted by (block, id)
    const uint32_t* cand_id;
    int32_t ncand;
    const int32_t* bal_t;  // their pass-start targets and gains
    const int64_t* bal_d;
    PQItem* qs;
    const int32_t* qoff;
    uint8_t* inq;       // node is queued now
    uint8_t* tried;     // node was offered as a neighbour in this pass
    int64_t* conn;      // connection per block, zero between uses
    int32_t* touched;   // at least b1 - b0 entries
    int32_t* full;      // set if an entry did not fit its block's queue room (a broken invariant)
};

// sign of rg(d1, c1) - rg(d2, c2)
KMP_HD inline int pq_rg_cmp(int64_t d1, int64_t c1, int64_t d2, int64_t c2)
{
    if (d1 >= 0 && d2 >= 0) {
        const int64_t x = d1 * c1, y = d2 * c2;
        return (x > y) - (x < y);
    }
    if (d1 >= 0) return 1;
    if (d2 >= 0) return -1;
    const int64_t x = d1 * c2, y = d2 * c1;  // d1 / c1 against d2 / c2, both negative
    return (x > y) - (x < y);
}

// a ranks before b in a queue
KMP_HD inline bool pq_before(const PQItem& a, const PQItem& b)
{
    const int r = pq_rg_cmp(a.d, a.c, b.d, b.c);
    return r > 0 || (r == 0 && a.v < b.v);
}

struct PQQueue {
    PQItem* e;
    int32_t n, room;
    int64_t w;
};

KMP_HD inline int32_t pq_best(const PQQueue& q)
{
    int32_t b = 0;
    for (int32_t i = 1; i < q.n; ++i)
        if (pq_before(q.e[i], q.e[b])) b = i;
    return b;
}

KMP_HD inline int32_t pq_worst(const PQQueue& q)
{
    int32_t b = 0;
    for (int32_t i = 1; i < q.n; ++i)
        if (pq_before(q.e[b], q.e[i])) b = i;
    return b;
}

KMP_HD inline PQItem pq_remove(PQQueue& q, int32_t i, uint8_t* inq)
{
    const PQItem x = q.e[i];
    q.e[i] = q.e[q.n - 1];
    q.n -= 1;
    q.w -= x.c;
    inq[x.v] = 0;
    return x;
}

// A queue holds distinct nodes of its block (inq), so its pass-start node count
// is room enough; `full` records a broken invariant instead of writing past it.
KMP_HD inline void pq_add(PQQueue& q, const PQItem& x, uint8_t* inq, int32_t* full)
{
    if (q.n >= q.room) {
        *full = 1;
        return;
    }
    q.e[q.n] = x;
    q.n += 1;
    q.w += x.c;
    inq[x.v] = 1;
}

KMP_HD inline void pq_offer_item(PQQueue& q, const PQItem& x, int64_t excess, int64_t maxc, uint8_t* inq,
                                 int32_t* full)
{
    if (q.w < excess) {
        pq_add(q, x, inq, full);
        return;
    }
    if (q.n == 0 || !pq_before(x, q.e[pq_worst(q)])) return;
    pq_add(q, x, inq, full);
    while (q.n > 0 && q.w > excess + maxc) pq_remove(q, pq_worst(q), inq);
}

// target and gain of v against the current weights; false if no block takes it
KMP_HD inline bool pq_target_of(const PQJob& J, int32_t v, PQItem& out)
{
    const int32_t b = J.part[v];
    const int64_t cv = J.vwgt ? J.vwgt[v] : 1;
    int32_t nt = 0;
    for (int32_t e = J.xadj[v]; e < J.xadj[v + 1]; ++e) {
        const int32_t t = J.part[J.adjncy[e]];
        if (J.conn[t] == 0) J.touched[nt++] = t;
        J.conn[t] += J.adjwgt ? J.adjwgt[e] : 1;
    }
    int32_t best = -1;
    uint32_t hb = 0;
    for (int32_t i = 0; i < nt; ++i) {
        const int32_t t = J.touched[i];
        if (t == b || J.wt[t] + cv > J.cap[t]) continue;
        const uint32_t h = hash_step(J.hpre, (uint32_t)(t - J.b0), 4);  // H(seed; T_BAL, level, pass, t - b0)
        const bool take = best < 0 || J.conn[t] > J.conn[best] ||
                          (J.conn[t] == J.conn[best] && (h < hb || (h == hb && t < best)));
        if (take) {
            best = t;
            hb = h;
        }
    }
    if (best < 0) {
        int32_t tf = -1;
        for (int32_t t = J.b0; t < J.b1; ++t)
            if (t != b && (tf < 0 || J.cap[t] - J.wt[t] > J.cap[tf] - J.wt[tf])) tf = t;
        if (tf >= 0 && J.wt[tf] + cv <= J.cap[tf]) best = tf;
    }
    if (best >= 0) {
        out.v = v;
        out.t = best;
        out.c = (int32_t)cv;
        out.d = J.conn[best] - J.conn[b];
        out.pad = 0;
    }
    for (int32_t i = 0; i < nt; ++i) J.conn[J.touched[i]] = 0;
    return best >= 0;
}

KMP_HD inline bool pq_border(const PQJob& J, int32_t v)
{
    for (int32_t e = J.xadj[v]; e < J.xadj[v + 1]; ++e)
        if (J.part[J.adjncy[e]] != J.part[v]) return true;
    return false;
}

// first index of the sorted candidate blocks not below b
KMP_HD inline int32_t pq_lower(const uint32_t* blk, int32_t n, int32_t b)
{
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if ((int32_t)blk[mid] < b) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One pass over the job's overloaded blocks; returns the number of moves.
KMP_HD inline int64_t pq_pass_job(const PQJob& J)
{
    int64_t moves = 0;
    for (int32_t b = J.b0; b < J.b1; ++b) {
        if (!J.over[b]) continue;
        PQQueue q{J.qs + J.qoff[b], 0, J.qoff[b + 1] - J.qoff[b], 0};
        const int32_t c0 = pq_lower(J.cand_blk, J.ncand, b), c1 = pq_lower(J.cand_blk, J.ncand, b + 1);
        for (int32_t i = c0; i < c1; ++i) {
            const int32_t v = (int32_t)J.cand_id[i];
            PQItem x;
            x.v = v;
            x.t = J.bal_t[v];
            x.d = J.bal_d[v];
            x.c = J.vwgt ? J.vwgt[v] : 1;
            x.pad = 0;
            pq_offer_item(q, x, J.wt[b] - J.cap[b], J.maxc, J.inq, J.full);
        }
        while (J.wt[b] > J.cap[b] && q.n > 0) {
            const PQItem x = pq_remove(q, pq_best(q), J.inq);
            PQItem y;
            if (!pq_target_of(J, x.v, y)) continue;
            if (y.d != x.d || J.wt[x.t] + x.c > J.cap[x.t]) {
                if (pq_border(J, x.v)) pq_offer_item(q, y, J.wt[b] - J.cap[b], J.maxc, J.inq, J.full);
                continue;
            }
            J.wt[x.t] += x.c;
            J.wt[b] -= x.c;
            J.part[x.v] = x.t;
            ++moves;
            for (int32_t e = J.xadj[x.v]; e < J.xadj[x.v + 1]; ++e) {
                const int32_t u = J.adjncy[e];
                if (J.part[u] != b || J.tried[u] || J.inq[u]) continue;
                J.tried[u] = 1;
                PQItem z;
                if (pq_target_of(J, u, z)) pq_offer_item(q, z, J.wt[b] - J.cap[b], J.maxc, J.inq, J.full);
            }
        }
        for (int32_t i = 0; i < q.n; ++i) J.inq[q.e[i].v] = 0;  // what is left is not queued any more
    }
    return moves;
}

}  // namespace kmp
