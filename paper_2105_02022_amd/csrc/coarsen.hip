// Coarsening steps after label propagation: two-hop merging of singleton
// clusters (paper Sec. 5.1 "Two-hop Clustering") and contraction (paper
// Sec. 2 "Multilevel Graph Partitioning").
//
// Contraction layout: coarse id = rank of the label among non-empty labels
// (prefix sum); members of every coarse node are bucketed; every coarse row
// aggregates (map[u], w) over its members' edges, dropping intra-cluster
// entries.  Rows whose members carry at most 4096 directed entries aggregate
// in an LDS hash table and sort it in LDS (bitonic); heavier rows go through
// an exact sort-reduce (stable radix by neighbour, then by row).
#include "kmp_dev.h"

namespace kmp {

namespace {

constexpr uint32_t EMPTY = 0xFFFFFFFFu;

// ---------------------------------------------------------------- two-hop
__global__ __launch_bounds__(kBlock) void k_count_nonempty(const int64_t* __restrict__ cw, int32_t n, int64_t* out)
{
    __shared__ int32_t cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int32_t local = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        local += cw[i] > 0;
    for (int d = 32; d > 0; d >>= 1) local += __shfl_xor(local, d, 64);
    if ((threadIdx.x & 63) == 0 && local) atomicAdd(&cnt, local);
    __syncthreads();
    if (threadIdx.x == 0 && cnt) spread_add(out, cnt);
}

// Batches: only jobs with glimit[job] > 0 take part.
__global__ void k_singleton_flags(const int32_t* __restrict__ label, const int64_t* __restrict__ cw,
                                  const int32_t* __restrict__ vwgt, int32_t n, const int32_t* __restrict__ gid,
                                  const int64_t* __restrict__ glimit, int32_t* __restrict__ flag)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int64_t c = vwgt ? vwgt[v] : 1;
    const bool takes_part = !gid || glimit[gid[v]] > 0;
    flag[v] = takes_part && cw[label[v]] == c;  // positive weights: the only member
}

// Group key 2 * fav; isolated nodes (fav NONE) form the last group of their
// job: key 2 * (end of the job's node range) - 1.
__global__ void k_singleton_compact(const int32_t* __restrict__ flag, const int32_t* __restrict__ flagpos,
                                    const uint32_t* __restrict__ fav, int32_t n, const int32_t* __restrict__ gid,
                                    const int32_t* __restrict__ gend, uint32_t* __restrict__ keys,
                                    uint32_t* __restrict__ vals)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n || !flag[v]) return;
    int32_t p = flagpos[v];
    uint32_t f = fav[v];
    const uint32_t end = gid ? (uint32_t)gend[gid[v]] : (uint32_t)n;
    keys[p] = f == kNone ? 2u * end - 1u : 2u * f;
    vals[p] = (uint32_t)v;
}

__global__ void k_group_heads(const uint32_t* __restrict__ keys, int64_t ns, int32_t* __restrict__ head)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    head[i] = (i == 0 || keys[i] != keys[i - 1]) ? (int32_t)i : 0;
}

__global__ void k_pair_eligible(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                const int32_t* __restrict__ gstart, int64_t ns, const int32_t* __restrict__ vwgt,
                                int64_t U, const int32_t* __restrict__ gid, const int64_t* __restrict__ gU,
                                int32_t* __restrict__ elig)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    int32_t e = 0;
    if (((i - gstart[i]) & 1) == 0 && i + 1 < ns && keys[i + 1] == keys[i]) {
        int64_t ca = vwgt ? vwgt[vals[i]] : 1;
        int64_t cb = vwgt ? vwgt[vals[i + 1]] : 1;
        e = ca + cb <= (gid ? gU[gid[vals[i]]] : U);
    }
    elig[i] = e;
}

// batches: eligible-pair rank at the first singleton of every job
__global__ void k_job_rank0(const uint32_t* __restrict__ vals, const int32_t* __restrict__ gid,
                            const int32_t* __restrict__ rank, int64_t ns, int32_t* __restrict__ grank0)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    const int32_t j = gid[vals[i]];
    if (i == 0 || gid[vals[i - 1]] != j) grank0[j] = rank[i];
}

__global__ void k_pair_apply(const uint32_t* __restrict__ vals, const int32_t* __restrict__ elig,
                             const int32_t* __restrict__ rank, int64_t ns, int64_t limit,
                             const int32_t* __restrict__ gid, const int64_t* __restrict__ glimit,
                             const int32_t* __restrict__ grank0, const int32_t* __restrict__ vwgt,
                             int32_t* __restrict__ label, int64_t* __restrict__ cw)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns || !elig[i]) return;
    if (gid) {
        const int32_t j = gid[vals[i]];
        if (rank[i] - grank0[j] >= glimit[j]) return;
    } else if (rank[i] >= limit) {
        return;
    }
    int32_t a = (int32_t)vals[i], b = (int32_t)vals[i + 1];
    int32_t la = label[a], lb = label[b];
    int64_t cb = vwgt ? vwgt[b] : 1;
    label[b] = la;
    atomicAdd((unsigned long long*)&cw[la], (unsigned long long)cb);
    atomicAdd((unsigned long long*)&cw[lb], (unsigned long long)(-cb));
}

// Per-job non-empty labels (label K of job j is node K of job j).
__global__ __launch_bounds__(kBlock) void k_count_nonempty_jobs(const int64_t* __restrict__ cw, int32_t n,
                                                                const int32_t* __restrict__ gid, int64_t* out)
{
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = base + threadIdx.x;
        int32_t j = -1;
        int64_t x = 0;
        if (i < n) {
            j = gid[i];
            x = cw[i] > 0;
        }
        job_add(out, j, x);
    }
}

// ---------------------------------------------------------------- contraction
// Batches: labels of jobs with gkeep[job] == 0 are not contracted.
__global__ void k_nonempty_flags(const int64_t* __restrict__ cw, int32_t n, const int32_t* __restrict__ gid,
                                 const uint8_t* __restrict__ gkeep, int32_t* __restrict__ flag)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = cw[i] > 0 && (!gkeep || gkeep[gid[i]]);
}

__global__ void k_map_and_weights(const int32_t* __restrict__ label, const int32_t* __restrict__ cid,
                                  const int64_t* __restrict__ cw, const int32_t* __restrict__ xadj, int32_t n,
                                  const int32_t* __restrict__ gid, const uint8_t* __restrict__ gkeep,
                                  int32_t* __restrict__ map, int32_t* __restrict__ cvwgt, int32_t* __restrict__ mcnt,
                                  int32_t* __restrict__ dsum)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    if (gkeep && !gkeep[gid[v]]) {
        map[v] = -1;
        return;
    }
    int32_t c = cid[label[v]];
    map[v] = c;
    if (cw[v] > 0) cvwgt[cid[v]] = (int32_t)cw[v];  // v read as a label here
    atomicAdd(&mcnt[c], 1);
    atomicAdd(&dsum[c], xadj[v + 1] - xadj[v]);
}

__global__ void k_place_members(const int32_t* __restrict__ map, int32_t n, const int32_t* __restrict__ mstart,
                                int32_t* __restrict__ cursor, int32_t* __restrict__ members)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int32_t c = map[v];
    if (c < 0) return;
    int32_t p = atomicAdd(&cursor[c], 1);
    members[mstart[c] + p] = (int32_t)v;
}

constexpr int R_T0 = 64, R_T1 = 512, R_T2 = 4096;

__global__ __launch_bounds__(kBlock) void k_row_tiers(const int32_t* __restrict__ dsum, int32_t nc,
                                                      uint32_t* __restrict__ key, uint32_t* __restrict__ val,
                                                      int32_t* __restrict__ cnt4)
{
    __shared__ int32_t h[4];
    if (threadIdx.x < 4) h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (int64_t)gridDim.x * blockDim.x) {
        int32_t d = dsum[c];
        uint32_t t = d <= R_T0 ? 0 : d <= R_T1 ? 1 : d <= R_T2 ? 2 : 3;
        key[c] = t;
        val[c] = (uint32_t)c;
        atomicAdd(&h[t], 1);
    }
    __syncthreads();
    if (threadIdx.x < 4 && h[threadIdx.x]) atomicAdd(&cnt4[threadIdx.x], h[threadIdx.x]);
}

struct RowArgs {
    const int32_t* xadj;
    const int32_t* adjncy;
    const int32_t* adjwgt;
    const int32_t* map;
    const int32_t* members;
    const int32_t* mstart;   // [nc+1]
    const int32_t* dstart;   // [nc+1] exclusive prefix of member degree sums
    int32_t* tmp_adj;
    int32_t* tmp_w;
    int32_t* cdeg;
    int64_t* bytes_ctr;
};

// G lanes per coarse row, 2^HB LDS slots per row; rows carry at most 2^(HB-1)
// fine entries, and a row of f fine entries uses the first 2^b >= 2 f slots.
// A lane loads four of its member's entries (and their coarse ids) before
// inserting any.  After aggregation the occupied slots are compacted to the
// front of the table (through registers) and only the next power of two above
// their count is sorted (bitonic).
template <int G, int HB>
__global__ __launch_bounds__(kBlock) void k_contract_rows(RowArgs a, const int32_t* __restrict__ rows, int32_t count)
{
    constexpr int GPB = kBlock / G;
    constexpr int HS = 1 << HB;
    constexpr int PER = HS / G;  // slots per lane
    __shared__ uint32_t s_keys[GPB * HS];
    __shared__ uint32_t s_vals[GPB * HS];
    __shared__ uint32_t s_u[GPB];
    __shared__ uint32_t s_pmax;
    const int tid = threadIdx.x, grp = tid / G, gl = tid % G;
    uint32_t* keys = s_keys + grp * HS;
    uint32_t* vals = s_vals + grp * HS;
    int64_t bytes = 0;
    for (int64_t base = (int64_t)xcd_block() * GPB; base < count; base += (int64_t)gridDim.x * GPB) {
        const int64_t i = base + grp;
        const int32_t row = i < count ? rows[i] : -1;
        int bits = 1;
        if (row >= 0) {
            const int32_t fine = a.dstart[row + 1] - a.dstart[row];
            while ((1 << bits) < 2 * fine && bits < HB) ++bits;
        }
        const int hsz = row >= 0 ? 1 << bits : 0;
        for (int j = gl; j < hsz; j += G) {
            keys[j] = EMPTY;
            vals[j] = 0;
        }
        if (tid < GPB) s_u[tid] = 0;
        if (tid == 0) s_pmax = 2;
        __syncthreads();
        if (row >= 0) {
            // the group's lanes split over the row's members (a power-of-two share
            // each, all G lanes for a single member), so the members' rows are
            // read side by side rather than one after another
            const int32_t m0 = a.mstart[row], m1 = a.mstart[row + 1];
            const int32_t nm = m1 - m0 < G ? m1 - m0 : G;
            int sw = G;  // lanes per member
            while (sw > 1 && (G / sw) < nm) sw >>= 1;
            const int sub = gl / sw, sl = gl % sw, par = G / sw;
            const uint32_t mask = (1u << bits) - 1u;
            constexpr int U = 4;
            for (int32_t mi = m0 + sub; mi < m1; mi += par) {
                const int32_t v = a.members[mi];
                const int32_t e1 = a.xadj[v + 1];
                for (int32_t e = a.xadj[v] + sl; e < e1; e += U * sw) {
                    // every load unconditional (indices clamped into the row), so all are in flight
                    int32_t u[U], cu[U];
                    uint32_t wq[U];
#pragma unroll
                    for (int q = 0; q < U; ++q) u[q] = a.adjncy[e + q * sw < e1 ? e + q * sw : e1 - 1];
#pragma unroll
                    for (int q = 0; q < U; ++q) {
                        cu[q] = a.map[u[q]];
                        wq[q] = a.adjwgt ? (uint32_t)a.adjwgt[e + q * sw < e1 ? e + q * sw : e1 - 1] : 1u;
                    }
#pragma unroll
                    for (int q = 0; q < U; ++q) {
                        if (e + q * sw >= e1 || cu[q] == row) continue;
                        const uint32_t w = wq[q];
                        // at most f distinct ids in at least 2 f slots: one sweep finds a slot
                        uint32_t h = slot_of((uint32_t)cu[q], bits);
                        for (uint32_t t = 0; t <= mask; ++t) {
                            const uint32_t old = atomicCAS(&keys[h], EMPTY, (uint32_t)cu[q]);
                            if (old == EMPTY || old == (uint32_t)cu[q]) {
                                atomicAdd(&vals[h], w);
                                break;
                            }
                            h = (h + 1) & mask;
                        }
                    }
                }
            }
        }
        __syncthreads();
        // compact the occupied slots (at most 2^(HB-1): one per fine entry)
        uint32_t rk[PER], rv[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const bool in = q * G + gl < hsz;
            rk[q] = in ? keys[q * G + gl] : EMPTY;
            rv[q] = in ? vals[q * G + gl] : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (rk[q] != EMPTY) {
                const uint32_t p = atomicAdd(&s_u[grp], 1u);
                keys[p] = rk[q];
                vals[p] = rv[q];
            }
        }
        __syncthreads();
        const uint32_t u = s_u[grp];
        uint32_t P = 2;
        while (P < u) P <<= 1;
        for (uint32_t j = u + gl; j < P; j += G) keys[j] = EMPTY;
        if (gl == 0) atomicMax(&s_pmax, P);
        __syncthreads();
        // bitonic sort of the first P entries, ascending key (padding last);
        // every group runs the block's largest P so the barriers stay uniform
        const uint32_t PM = s_pmax;
        for (uint32_t size = 2; size <= PM; size <<= 1) {
            for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                if (size <= P) {
                    for (uint32_t p = gl; p < P / 2; p += G) {
                        const uint32_t lo = 2 * stride * (p / stride) + (p % stride);
                        const uint32_t hi = lo + stride;
                        const bool up = (lo & size) == 0;
                        const uint32_t kl = keys[lo], kh = keys[hi];
                        if ((kl > kh) == up) {
                            keys[lo] = kh;
                            keys[hi] = kl;
                            const uint32_t t = vals[lo];
                            vals[lo] = vals[hi];
                            vals[hi] = t;
                        }
                    }
                }
                __syncthreads();
            }
        }
        if (row >= 0) {
            const int32_t o = a.dstart[row];
            for (uint32_t j = gl; j < u; j += G) {
                a.tmp_adj[o + j] = (int32_t)keys[j];
                a.tmp_w[o + j] = (int32_t)vals[j];
            }
            if (gl == 0) {
                a.cdeg[row] = (int32_t)u;
                const int64_t fine = a.dstart[row + 1] - a.dstart[row];
                const int64_t mem = a.mstart[row + 1] - a.mstart[row];
                bytes += 12 * fine + 12 * mem + 8 * (int64_t)u + 16;
            }
        }
        __syncthreads();
    }
    for (int d = 32; d > 0; d >>= 1) bytes += __shfl_xor(bytes, d, 64);
    if ((tid & 63) == 0 && bytes) spread_add(a.bytes_ctr, bytes);
}

// ---- heavy rows: expand, sort by (row, neighbour), reduce
__global__ __launch_bounds__(kBlock) void k_heavy_expand(RowArgs a, const int32_t* __restrict__ rows, int32_t nrows,
                                                         const int32_t* __restrict__ eoff, uint32_t nc,
                                                         uint32_t* __restrict__ nbr, uint32_t* __restrict__ rowq,
                                                         int32_t* __restrict__ w, int nbbits)
{
    // nbbits >= 0: one packed key (row << nbbits | neighbour) per entry in nbr, rowq unused
    for (int32_t q = blockIdx.x; q < nrows; q += gridDim.x) {
        const int32_t row = rows[q];
        int32_t pos = eoff[q];
        for (int32_t mi = a.mstart[row]; mi < a.mstart[row + 1]; ++mi) {
            const int32_t v = a.members[mi];
            const int32_t e0 = a.xadj[v], e1 = a.xadj[v + 1];
            for (int32_t e = e0 + threadIdx.x; e < e1; e += kBlock) {
                const int32_t cu = a.map[a.adjncy[e]];
                const int32_t p = pos + (e - e0);
                const uint32_t nb = cu == row ? nc : (uint32_t)cu;  // intra entries sort last in the row
                if (nbbits >= 0) {
                    nbr[p] = ((uint32_t)q << nbbits) | nb;
                } else {
                    nbr[p] = nb;
                    rowq[p] = (uint32_t)q;
                }
                w[p] = a.adjwgt ? a.adjwgt[e] : 1;
            }
            pos += e1 - e0;
        }
    }
}

__global__ void k_heavy_deg(const int32_t* __restrict__ rows, int32_t nrows, const int32_t* __restrict__ dsum,
                            int32_t* __restrict__ d)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nrows) d[q] = dsum[rows[q]];
}

__global__ void k_gather_u32(const uint32_t* __restrict__ src, const uint32_t* __restrict__ idx, int64_t n,
                             uint32_t* __restrict__ dst)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

__global__ void k_heavy_unpack(const uint32_t* __restrict__ key, int64_t n, int nbbits, uint32_t* __restrict__ rq,
                               uint32_t* __restrict__ nb)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const uint32_t k = key[i];
        rq[i] = nbbits < 32 ? k >> nbbits : 0u;
        nb[i] = k & (uint32_t)((1ull << nbbits) - 1);
    }
}

__global__ void k_heavy_heads(const uint32_t* __restrict__ rq, const uint32_t* __restrict__ nb,
                              const uint32_t* __restrict__ perm, const int32_t* __restrict__ w, int64_t ne,
                              int32_t* __restrict__ head, int64_t* __restrict__ wsorted)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    head[i] = (i == 0 || rq[i] != rq[i - 1] || nb[i] != nb[i - 1]);
    wsorted[i] = w[perm[i]];
}

// Row start: remember the run id of the row's first entry.
__global__ void k_heavy_rowfirst(const uint32_t* __restrict__ rq, const int32_t* __restrict__ head_excl, int64_t ne,
                                 int32_t* __restrict__ rowfirst)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ne && (i == 0 || rq[i] != rq[i - 1])) rowfirst[rq[i]] = head_excl[i];
}

__global__ void k_run_start(const int32_t* __restrict__ is_head, int64_t ne, int32_t* __restrict__ start_of_run,
                            const int32_t* __restrict__ head_excl)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ne && is_head[i]) start_of_run[head_excl[i]] = (int32_t)i;
}

// The last entry of every run writes the run (sum of its weights); the last
// entry of every row writes the row's distinct-neighbour count.  The intra-
// cluster run (neighbour id nc) sorts last in its row and is dropped.
__global__ void k_heavy_emit(const uint32_t* __restrict__ rq, const uint32_t* __restrict__ nb,
                             const int32_t* __restrict__ head_excl, const int32_t* __restrict__ is_head,
                             const int64_t* __restrict__ wpre, const int64_t* __restrict__ wsorted, int64_t ne,
                             uint32_t nc, const int32_t* __restrict__ rows, const int32_t* __restrict__ dstart,
                             const int32_t* __restrict__ start_of_run, const int32_t* __restrict__ rowfirst,
                             int32_t* __restrict__ tmp_adj, int32_t* __restrict__ tmp_w, int32_t* __restrict__ cdeg)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const bool run_last = (i + 1 == ne) || is_head[i + 1];
    if (!run_last) return;
    const uint32_t q = rq[i];
    const int32_t run = head_excl[i] + is_head[i] - 1;
    const int32_t pos = run - rowfirst[q];
    const int32_t row = rows[q];
    const uint32_t nbr = nb[i];
    if (nbr < nc) {
        const int32_t s = start_of_run[run];
        const int64_t sum = wpre[i] - wpre[s] + wsorted[s];
        tmp_adj[dstart[row] + pos] = (int32_t)nbr;
        tmp_w[dstart[row] + pos] = (int32_t)sum;
    }
    const bool row_last = (i + 1 == ne) || rq[i + 1] != q;
    if (row_last) cdeg[row] = nbr < nc ? pos + 1 : pos;
}

__global__ void k_copy_rows(const int32_t* __restrict__ cxadj, const int32_t* __restrict__ dstart, int32_t nc,
                            const int32_t* __restrict__ tmp_adj, const int32_t* __restrict__ tmp_w,
                            int32_t* __restrict__ cadj, int32_t* __restrict__ cw)
{
    // 16 lanes per row; rows of more than R_T2 fine entries are left to k_copy_heavy
    const int gl = threadIdx.x & 15;
    int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
    const int64_t stride = ((int64_t)gridDim.x * blockDim.x) >> 4;
    for (; r < nc; r += stride) {
        const int32_t s = dstart[r];
        if (dstart[r + 1] - s > R_T2) continue;
        const int32_t o = cxadj[r], len = cxadj[r + 1] - o;
        for (int32_t j = gl; j < len; j += 16) {
            cadj[o + j] = tmp_adj[s + j];
            cw[o + j] = tmp_w[s + j];
        }
    }
}

// The rows of more than R_T2 fine entries (the heavy path's; up to 10^5 coarse
// entries on power-law graphs), one workgroup each, eight entries per thread in
// flight (indices clamped into the row: the last entry is copied again).
__global__ __launch_bounds__(kBlock) void k_copy_heavy(const int32_t* __restrict__ hrows,
                                                       const int32_t* __restrict__ cxadj,
                                                       const int32_t* __restrict__ dstart,
                                                       const int32_t* __restrict__ tmp_adj,
                                                       const int32_t* __restrict__ tmp_w, int32_t* __restrict__ cadj,
                                                       int32_t* __restrict__ cw)
{
    const int32_t r = hrows[blockIdx.x];
    const int32_t o = cxadj[r], len = cxadj[r + 1] - o, s = dstart[r];
    if (len <= 0) return;
    for (int32_t j0 = threadIdx.x; j0 < len; j0 += 8 * kBlock) {
        int32_t x[8], w[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int32_t j = j0 + q * kBlock < len ? j0 + q * kBlock : len - 1;
            x[q] = tmp_adj[s + j];
            w[q] = tmp_w[s + j];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int32_t j = j0 + q * kBlock < len ? j0 + q * kBlock : len - 1;
            cadj[o + j] = x[q];
            cw[o + j] = w[q];
        }
    }
}

}  // namespace

// ================================================================ host side

int32_t count_nonempty(Ctx& c, const int64_t* cw, int32_t n)
{
    if (n <= 0) return 0;
    c.zero_spread(SP_NONEMPTY);
    hipLaunchKernelGGL(k_count_nonempty, dim3(grid_for(n, kBlock, 1024)), dim3(kBlock), 0, c.stream, cw, n,
                       c.spread(SP_NONEMPTY));
    KMP_LAUNCH_CHECK();
    return (int32_t)c.read_spread(SP_NONEMPTY);
}

void count_nonempty_jobs(Ctx& c, const int64_t* cw, int32_t n, const JobTabs& jt, int32_t njobs,
                         std::vector<int64_t>& out)
{
    out.assign(njobs, 0);
    if (n <= 0) return;
    if (!jt.gid) {
        out[0] = count_nonempty(c, cw, n);
        return;
    }
    DBuf<int64_t> d(c, (size_t)njobs);
    c.zero(d.p, sizeof(int64_t) * njobs);
    hipLaunchKernelGGL(k_count_nonempty_jobs, dim3(grid_for(n, kBlock, 1024)), dim3(kBlock), 0, c.stream, cw, n,
                       jt.gid, d.p);
    KMP_LAUNCH_CHECK();
    c.read(out.data(), d.p, sizeof(int64_t) * njobs);
}

namespace {

// Two-hop merging of singletons (Sec. 5.1): singletons sorted by (favoured
// cluster, id), paired (0,1), (2,3), ... inside a group; the first `limit`
// eligible pairs (c(a) + c(b) <= U) of every job merge.  One graph: scalar U
// and limit; batches: gU / glimit / gend by job.
int64_t two_hop_core(Ctx& c, const DGraph& g, const JobTabs& jt, int64_t U, int64_t limit, const int64_t* gU,
                     const int64_t* glimit, const int32_t* gend, int32_t njobs, int32_t* label, int64_t* cw,
                     const uint32_t* fav, bool count)
{
    const int32_t n = g.n;
    ProfScope ps(c, KMP_PROF_TWO_HOP);
    DBuf<int32_t> flag(c, (size_t)n), pos(c, (size_t)n + 1);
    hipLaunchKernelGGL(k_singleton_flags, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, label, cw, g.vwgt, n, jt.gid,
                       glimit, flag.p);
    KMP_LAUNCH_CHECK();
    scan_excl_i32(c, flag.p, pos.p, n, pos.p + n);
    const int32_t ns = c.read1(pos.p + n);
    if (ns < 2) return 0;
    DBuf<uint32_t> keys(c, ns), vals(c, ns), k2(c, ns), v2(c, ns);
    hipLaunchKernelGGL(k_singleton_compact, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, flag.p, pos.p, fav, n,
                       jt.gid, gend, keys.p, vals.p);
    KMP_LAUNCH_CHECK();
    uint32_t *skeys = nullptr, *svals = nullptr;  // the sorted pairs (first or alternate buffers)
    radix_sort_pairs(c, keys.p, vals.p, k2.p, v2.p, ns, bits_for(2 * (uint64_t)n), &skeys, &svals);
    DBuf<int32_t> gstart(c, ns), elig(c, (size_t)ns + 1);
    hipLaunchKernelGGL(k_group_heads, dim3(grid_for(ns)), dim3(kBlock), 0, c.stream, skeys, (int64_t)ns, gstart.p);
    KMP_LAUNCH_CHECK();
    scan_incl_max_i32(c, gstart.p, gstart.p, ns);
    hipLaunchKernelGGL(k_pair_eligible, dim3(grid_for(ns)), dim3(kBlock), 0, c.stream, skeys, svals, gstart.p,
                       (int64_t)ns, g.vwgt, U, jt.gid, gU, elig.p);
    KMP_LAUNCH_CHECK();
    DBuf<int32_t> rank(c, (size_t)ns + 1);
    scan_excl_i32(c, elig.p, rank.p, ns, rank.p + ns);
    DBuf<int32_t> grank0;
    if (jt.gid) {
        grank0 = DBuf<int32_t>(c, (size_t)njobs);
        hipLaunchKernelGGL(k_job_rank0, dim3(grid_for(ns)), dim3(kBlock), 0, c.stream, svals, jt.gid, rank.p,
                           (int64_t)ns, grank0.p);
        KMP_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_pair_apply, dim3(grid_for(ns)), dim3(kBlock), 0, c.stream, svals, elig.p, rank.p,
                       (int64_t)ns, limit, jt.gid, glimit, grank0.p, g.vwgt, label, cw);
    KMP_LAUNCH_CHECK();
    return count ? (int64_t)c.read1(rank.p + ns) : 0;
}

}  // namespace

int64_t two_hop(Ctx& c, const DGraph& g, int64_t U, int32_t* label, int64_t* cw, const uint32_t* fav, bool count,
                int32_t* nonempty_out)
{
    const int32_t n = g.n;
    const int32_t nc = count_nonempty(c, cw, n);
    const int64_t half = n / 2;
    if (nonempty_out) *nonempty_out = nc <= half ? nc : -1;
    if (nc <= half) return 0;
    const int64_t limit = (int64_t)nc - half;
    const int64_t E = two_hop_core(c, g, JobTabs{}, U, limit, nullptr, nullptr, nullptr, 1, label, cw, fav, count);
    return E < limit ? E : limit;
}

void two_hop_jobs(Ctx& c, const DGraph& g, const JobTabs& jt, const int64_t* gU, const int64_t* glimit,
                  const int32_t* gend, int32_t njobs, int32_t* label, int64_t* cw, const uint32_t* fav)
{
    two_hop_core(c, g, jt, 0, 0, gU, glimit, gend, njobs, label, cw, fav, false);
}

int32_t contract_ids(Ctx& c, const DGraph& g, const int64_t* cw, DBuf<int32_t>& cid, const JobTabs& jt,
                     const uint8_t* gkeep, int32_t known)
{
    const int32_t n = g.n;
    cid = DBuf<int32_t>(c, (size_t)n + 1);
    hipLaunchKernelGGL(k_nonempty_flags, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, cw, n, jt.gid, gkeep, cid.p);
    KMP_LAUNCH_CHECK();
    scan_excl_i32(c, cid.p, cid.p, n, cid.p + n);
    return known >= 0 ? known : c.read1(cid.p + n);
}

void contract(Ctx& c, const DGraph& g, const int32_t* label, const int64_t* cw, int32_t* map, OwnedGraph& out,
              int32_t& cn, int64_t& cm, const JobTabs& jt, const uint8_t* gkeep, DBuf<int32_t>* cid_in, int32_t nc_in,
              int32_t* maxdeg)
{
    const int32_t n = g.n;
    DBuf<int32_t> cid_own;
    int32_t nc;
    if (cid_in) {
        nc = nc_in;
    } else {
        nc = contract_ids(c, g, cw, cid_own, jt, gkeep);
    }
    DBuf<int32_t>& cid = cid_in ? *cid_in : cid_own;
    cn = nc;
    out.xadj = DBuf<int32_t>(c, (size_t)nc + 1);
    out.vwgt = DBuf<int32_t>(c, (size_t)nc);
    DBuf<int32_t> mstart(c, (size_t)nc + 1), dstart(c, (size_t)nc + 1), cursor(c, (size_t)nc);
    DBuf<int32_t> cnt4(c, 6);  // row tier counts; then the coarse entry count and largest degree
    fill_bytes_many(c, {{mstart.p, 4 * ((int64_t)nc + 1), 0},
                        {dstart.p, 4 * ((int64_t)nc + 1), 0},
                        {cursor.p, 4 * (int64_t)nc, 0},
                        {cnt4.p, 24, 0}});
    hipLaunchKernelGGL(k_map_and_weights, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, label, cid.p, cw, g.xadj, n,
                       jt.gid, gkeep, map, out.vwgt.p, mstart.p, dstart.p);
    KMP_LAUNCH_CHECK();
    // dsum keeps the per-row fine degree sums; dstart receives their offsets
    DBuf<int32_t> dsum = std::move(dstart);
    dstart = DBuf<int32_t>(c, (size_t)nc + 1);
    scan_excl_i32(c, mstart.p, mstart.p, nc, mstart.p + nc);
    scan_excl_i32(c, dsum.p, dstart.p, nc, dstart.p + nc);
    DBuf<int32_t> members(c, (size_t)n);
    hipLaunchKernelGGL(k_place_members, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, map, n, mstart.p, cursor.p,
                       members.p);
    KMP_LAUNCH_CHECK();
    // rows by tier of their fine entry count
    DBuf<uint32_t> rk(c, nc), rv(c, nc), rk2(c, nc), rv2(c, nc);
    hipLaunchKernelGGL(k_row_tiers, dim3(grid_for(nc, kBlock, 256)), dim3(kBlock), 0, c.stream, dsum.p, nc, rk.p, rv.p, cnt4.p);
    KMP_LAUNCH_CHECK();
    uint32_t* rsorted = nullptr;
    radix_sort_pairs(c, rk.p, rv.p, rk2.p, rv2.p, nc, 2, nullptr, &rsorted);
    int32_t tc[4];
    c.read(tc, cnt4.p, sizeof(tc));
    const int32_t* rows = reinterpret_cast<const int32_t*>(rsorted);
    DBuf<int32_t> tmp_adj(c, (size_t)(g.m > 0 ? g.m : 1)), tmp_w(c, (size_t)(g.m > 0 ? g.m : 1));
    DBuf<int32_t> cdeg(c, (size_t)nc + 1);
    RowArgs a;
    a.xadj = g.xadj;
    a.adjncy = g.adjncy;
    a.adjwgt = g.adjwgt;
    a.map = map;
    a.members = members.p;
    a.mstart = mstart.p;
    a.dstart = dstart.p;
    a.tmp_adj = tmp_adj.p;
    a.tmp_w = tmp_w.p;
    a.cdeg = cdeg.p;
    a.bytes_ctr = c.spread(SP_BYTES + KMP_PROF_CONTRACT_ROWS);
    int32_t off = 0;
    if (tc[0] > 0)
        KMP_LAUNCH_TIMED(c, KMP_PROF_CONTRACT_ROWS, (k_contract_rows<16, 7>), dim3(grid_for(tc[0], kBlock / 16, 65536)),
                         dim3(kBlock), 0, a, rows + off, tc[0]);
    off += tc[0];
    if (tc[1] > 0)
        KMP_LAUNCH_TIMED(c, KMP_PROF_CONTRACT_ROWS, (k_contract_rows<64, 10>),
                         dim3(grid_for(tc[1], kBlock / 64, 65536)), dim3(kBlock), 0, a, rows + off, tc[1]);
    off += tc[1];
    if (tc[2] > 0)
        KMP_LAUNCH_TIMED(c, KMP_PROF_CONTRACT_ROWS, (k_contract_rows<256, 13>), dim3(grid_for(tc[2], 1, 65536)),
                         dim3(kBlock), 0, a, rows + off, tc[2]);
    off += tc[2];
    const int32_t* heavy_rows = rows + off;  // the rows of more than R_T2 fine entries (tc[3] of them)
    if (tc[3] > 0) {
        const int32_t nh = tc[3];
        const int32_t* hrows = rows + off;
        DBuf<int32_t> eoff(c, (size_t)nh + 1);
        hipLaunchKernelGGL(k_heavy_deg, dim3(grid_for(nh)), dim3(kBlock), 0, c.stream, hrows, nh, dsum.p, eoff.p);
        KMP_LAUNCH_CHECK();
        scan_excl_i32(c, eoff.p, eoff.p, nh, eoff.p + nh);
        const int64_t ne = c.read1(eoff.p + nh);
        // (row, neighbour) fits one 32-bit key on most levels: one stable sort of
        // the packed key orders entries by (row, neighbour, entry id), as the two
        // stable sorts below do
        const int nbbits = bits_for((uint64_t)nc), rqbits = bits_for((uint64_t)(nh - 1));
        const bool packed = nbbits + rqbits <= 32;
        DBuf<uint32_t> nb(c, ne), rq(c, packed ? 1 : ne), perm(c, ne), t1(c, ne), t2(c, ne);
        DBuf<int32_t> w(c, ne);
        hipLaunchKernelGGL(k_heavy_expand, dim3(grid_for(nh, 1, 4096)), dim3(kBlock), 0, c.stream, a, hrows, nh,
                           eoff.p, (uint32_t)nc, nb.p, rq.p, w.p, packed ? nbbits : -1);
        KMP_LAUNCH_CHECK();
        DBuf<uint32_t> rqs(c, ne), nbs(c, ne), perm2;
        iota_i32(c, reinterpret_cast<int32_t*>(perm.p), ne);
        if (packed) {
            radix_sort_pairs(c, nb.p, perm.p, t1.p, t2.p, ne, nbbits + rqbits);
            hipLaunchKernelGGL(k_heavy_unpack, dim3(grid_for(ne)), dim3(kBlock), 0, c.stream, nb.p, ne, nbbits, rqs.p,
                               nbs.p);
            KMP_LAUNCH_CHECK();
            perm2 = std::move(perm);
        } else {
            // sort entry ids by neighbour, then stably by row
            radix_sort_pairs(c, nb.p, perm.p, t1.p, t2.p, ne, nbbits);
            hipLaunchKernelGGL(k_gather_u32, dim3(grid_for(ne)), dim3(kBlock), 0, c.stream, rq.p, perm.p, ne, rqs.p);
            KMP_LAUNCH_CHECK();
            // carry the neighbour along: sort (row, position) and gather both
            DBuf<uint32_t> pos(c, ne);
            iota_i32(c, reinterpret_cast<int32_t*>(pos.p), ne);
            radix_sort_pairs(c, rqs.p, pos.p, t1.p, t2.p, ne, rqbits);
            // final order: entry = perm[pos[i]]
            perm2 = DBuf<uint32_t>(c, ne);
            hipLaunchKernelGGL(k_gather_u32, dim3(grid_for(ne)), dim3(kBlock), 0, c.stream, perm.p, pos.p, ne,
                               perm2.p);
            KMP_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_gather_u32, dim3(grid_for(ne)), dim3(kBlock), 0, c.stream, nb.p, pos.p, ne, nbs.p);
            KMP_LAUNCH_CHECK();
        }
        DBuf<int32_t> head(c, (size_t)ne + 1), hexcl(c, (size_t)ne + 1), runstart(c, (size_t)ne + 1);
        DBuf<int64_t> ws(c, ne), wpre(c, ne);
        hipLaunchKernelGGL(k_heavy_heads, dim3(grid_for(ne)), dim3(kBlock), 0, c.stream, rqs.p, nbs.p, perm2.p, w.p,
                           ne, head.p, ws.p);
        KMP_LAUNCH_CHECK();
        scan_excl_i32(c, head.p, hexcl.p, ne, hexcl.p + ne);
        scan_incl_i64(c, ws.p, wpre.p, ne);
        hipLaunchKernelGGL(k_run_start, dim3(grid_for(ne)), dim3(kBlock), 0, c.stream, head.p, ne, runstart.p,
                           hexcl.p);
        KMP_LAUNCH_CHECK();
        DBuf<int32_t> rowfirst(c, (size_t)nh);
        hipLaunchKernelGGL(k_heavy_rowfirst, dim3(grid_for(ne)), dim3(kBlock), 0, c.stream, rqs.p, hexcl.p, ne,
                           rowfirst.p);
        KMP_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_heavy_emit, dim3(grid_for(ne)), dim3(kBlock), 0, c.stream, rqs.p, nbs.p, hexcl.p, head.p,
                           wpre.p, ws.p, ne, (uint32_t)nc, hrows, dstart.p, runstart.p, rowfirst.p, tmp_adj.p,
                           tmp_w.p, cdeg.p);
        KMP_LAUNCH_CHECK();
    }
    scan_excl_i32(c, cdeg.p, out.xadj.p, nc, out.xadj.p + nc);
    int32_t md = 0;
    entries_and_max_degree(c, out.xadj.p, nc, cm, md, cnt4.p + 4);
    if (maxdeg) *maxdeg = md;
    out.adjncy = DBuf<int32_t>(c, (size_t)(cm > 0 ? cm : 1));
    out.adjwgt = DBuf<int32_t>(c, (size_t)(cm > 0 ? cm : 1));
    if (nc > 0) {
        hipLaunchKernelGGL(k_copy_rows, dim3(grid_for((int64_t)nc * 16, kBlock, 16384)), dim3(kBlock), 0, c.stream,
                           out.xadj.p, dstart.p, nc, tmp_adj.p, tmp_w.p, out.adjncy.p, out.adjwgt.p);
        KMP_LAUNCH_CHECK();
        if (tc[3] > 0) {
            hipLaunchKernelGGL(k_copy_heavy, dim3((unsigned)tc[3]), dim3(kBlock), 0, c.stream, heavy_rows, out.xadj.p,
                               dstart.p, tmp_adj.p, tmp_w.p, out.adjncy.p, out.adjwgt.p);
            KMP_LAUNCH_CHECK();
        }
    }
}

}  // namespace kmp
