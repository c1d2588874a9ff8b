// Host build of the GPU queue balancer's pass routine (paper_2105_02022_amd/
// csrc/pq_pass.h) for tests/test_pq_pass_host.py: the passes of one graph run
// on the CPU, every array allocated at its exact size so that AddressSanitizer
// reports any access outside it.  The pass-start targets and gains are the
// routine's own (the GPU takes them from its balance-mode rating).
//
// stdin (binary, little endian): n, m, nb, level (int32), seed (uint64), has_vw,
// has_ew (int32), xadj[n+1], adjncy[m], vwgt[n] if has_vw, adjwgt[m] if has_ew
// (int32), part[n] (int32), wt[nb], cap[nb] (int64).
// stdout: passes, queue-room flag (int32), part[n] (int32), wt[nb] (int64).
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <vector>

#include "pq_pass.h"

template <class T>
static T* exact(size_t n)
{
    return new T[n > 0 ? n : 1]();
}

template <class T>
static void rd(T* p, size_t n)
{
    if (n && fread(p, sizeof(T), n, stdin) != n) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
}

int main()
{
    int32_t hdr[4];
    uint64_t seed;
    int32_t flags[2];
    rd(hdr, 4);
    rd(&seed, 1);
    rd(flags, 2);
    const int32_t n = hdr[0], m = hdr[1], nb = hdr[2], level = hdr[3];
    int32_t* xadj = exact<int32_t>(n + 1);
    int32_t* adjncy = exact<int32_t>(m);
    int32_t* vwgt = flags[0] ? exact<int32_t>(n) : nullptr;
    int32_t* adjwgt = flags[1] ? exact<int32_t>(m) : nullptr;
    int32_t* part = exact<int32_t>(n);
    int64_t* wt = exact<int64_t>(nb);
    int64_t* cap = exact<int64_t>(nb);
    rd(xadj, n + 1);
    rd(adjncy, m);
    if (vwgt) rd(vwgt, n);
    if (adjwgt) rd(adjwgt, m);
    rd(part, n);
    rd(wt, nb);
    rd(cap, nb);

    uint8_t* over = exact<uint8_t>(nb);
    uint8_t* inq = exact<uint8_t>(n);
    uint8_t* tried = exact<uint8_t>(n);
    int64_t* conn = exact<int64_t>(nb);
    int32_t* touched = exact<int32_t>(nb);
    int32_t* bal_t = exact<int32_t>(n);
    int64_t* bal_d = exact<int64_t>(n);
    int32_t* qoff = exact<int32_t>(nb + 1);
    kmp::PQItem* qs = exact<kmp::PQItem>(n);
    int32_t full = 0;
    int64_t maxc = 0;
    for (int32_t v = 0; v < n; ++v) maxc = std::max<int64_t>(maxc, vwgt ? vwgt[v] : 1);

    kmp::PQJob J;
    J.xadj = xadj;
    J.adjncy = adjncy;
    J.vwgt = vwgt;
    J.adjwgt = adjwgt;
    J.part = part;
    J.wt = wt;
    J.cap = cap;
    J.b0 = 0;
    J.b1 = nb;
    J.maxc = maxc;
    J.over = over;
    J.bal_t = bal_t;
    J.bal_d = bal_d;
    J.qs = qs;
    J.qoff = qoff;
    J.inq = inq;
    J.tried = tried;
    J.conn = conn;
    J.touched = touched;
    J.full = &full;

    int32_t pass = 0;
    bool moved_prev = true;
    for (;;) {
        bool any = false;
        for (int32_t b = 0; b < nb; ++b) {
            over[b] = wt[b] > cap[b];
            any = any || over[b];
        }
        if (!any || !moved_prev) break;
        J.hpre = kmp::hash_prefix(seed, {kmp::TAG_BAL, (uint32_t)level, (uint32_t)pass});
        // pass-start candidates in (block, id) order with their targets and gains
        std::vector<std::pair<uint32_t, uint32_t>> cand;
        for (int32_t v = 0; v < n; ++v) {
            kmp::PQItem x;
            if (over[part[v]] && kmp::pq_target_of(J, v, x)) {
                bal_t[v] = x.t;
                bal_d[v] = x.d;
                cand.push_back({(uint32_t)part[v], (uint32_t)v});
            }
        }
        std::sort(cand.begin(), cand.end());
        uint32_t* cblk = exact<uint32_t>(cand.size());
        uint32_t* cid = exact<uint32_t>(cand.size());
        for (size_t i = 0; i < cand.size(); ++i) {
            cblk[i] = cand[i].first;
            cid[i] = cand[i].second;
        }
        J.cand_blk = cblk;
        J.cand_id = cid;
        J.ncand = (int32_t)cand.size();
        // queue room: the pass-start nodes of every block
        std::fill(qoff, qoff + nb + 1, 0);
        for (int32_t v = 0; v < n; ++v) qoff[part[v] + 1] += 1;
        for (int32_t b = 0; b < nb; ++b) qoff[b + 1] += qoff[b];
        std::fill(tried, tried + n, 0);
        const int64_t moves = kmp::pq_pass_job(J);
        delete[] cblk;
        delete[] cid;
        moved_prev = moves > 0;
        ++pass;
    }
    fwrite(&pass, sizeof(int32_t), 1, stdout);
    fwrite(&full, sizeof(int32_t), 1, stdout);
    fwrite(part, sizeof(int32_t), (size_t)n, stdout);
    fwrite(wt, sizeof(int64_t), (size_t)nb, stdout);
    delete[] xadj;
    delete[] adjncy;
    delete[] vwgt;
    delete[] adjwgt;
    delete[] part;
    delete[] wt;
    delete[] cap;
    delete[] over;
    delete[] inq;
    delete[] tried;
    delete[] conn;
    delete[] touched;
    delete[] bal_t;
    delete[] bal_d;
    delete[] qoff;
    delete[] qs;
    return 0;
}
