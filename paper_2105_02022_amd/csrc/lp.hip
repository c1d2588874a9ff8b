// Size-constrained label propagation on gfx950 (paper Sec. 2 "Size-
// Constrained Label Propagation", Sec. 5.1 coarsening, Sec. 5.3 refinement).
//
// Deterministic sub-round reading: a round visits the nodes in S = 4 hash
// classes; the nodes of one class are rated against the state at the start of
// the sub-round (rate kernels), then proposals into one target are admitted in
// ascending node id while the running weight fits (admission), then applied.
// After a round only nodes with a neighbour that moved stay active.
//
// Rate kernel tiers by degree (execution layout only; results identical):
//   tier 0  deg <= 16    one lane per node, neighbour labels in registers
//   tier 1  deg <= 64    16 lanes per node, 128-slot LDS hash per node
//   tier 2  deg <= 512   one wavefront per node, 1024-slot LDS hash
//   tier 3  deg <= 4096  one workgroup per node, 8192-slot LDS hash
//   tier 4  deg >  4096  global-memory hash table per hub, split into chunks
//                         of 8192 slots: many workgroups insert a hub's entries,
//                         many scan its table, one wave per hub picks the best
//
// Admission: proposals add their weight to demand[K]; targets whose whole
// demand fits are admitted at once.  The others ("contended") are appended to
// a list (with the target's weight at the start of the sub-round); the apply
// kernel decides each contended proposal by summing the weights of the
// proposals into its target with smaller ids, read from the list through LDS.
// Sub-rounds are enqueued speculatively: if the contended list of a sub-round
// is longer than kSmallCap, a device flag aborts the rest of the round and the
// host finishes it on the exact path (sort in global memory), one sub-round at
// a time.  Every round walks the same static class lists; a node is rated in a
// round after the first only if its stamp in that round's parity array says a
// neighbour moved (the apply kernel stamps the neighbours of moved nodes of
// tiers 0 and 1, a marking kernel those of the wider tiers).  Small levels and
// small batch jobs run the whole LP in one workgroup with its state in LDS.
#include <mutex>

#include "kmp_dev.h"

namespace kmp {

namespace {

constexpr int T0_DEG = 16, T1_DEG = 64, T2_DEG = 512, T3_DEG = 4096;
constexpr int T0_NARROW = 8;  // tier-0 nodes of at most this degree are listed first
constexpr uint32_t EMPTY = 0xFFFFFFFFu;
constexpr int kSmallCap = 4096;     // contended entries resolved on the device
constexpr int kCandChunk = 1024;    // contended entries staged in LDS per pass
constexpr int kWaveScanMax = 32;    // contended nodes of a wavefront scanned one by one by the whole wavefront

// ctl[] layout (int64, device): round control shared by the kernels (the
// contended-list length alternates between CTL_CONT and CTL_CONT + 1 by
// sub-round parity, so that each apply clears the next one's; an abort records
// its round stamp and sub-round), then the per-block move counts of every round
// as a spread counter whose slot lines hold one word per round (round r of slot
// q at CTL_MS + q * kSpreadStride + r), then the segment table of the lists
// without the skipped jobs (batches)
enum { CTL_ABORT = 0, CTL_ABORT_SUB = 1, CTL_ABORT_STAMP = 2, CTL_CONT = 3, CTL_N = 8, CTL_MS = CTL_N };
static_assert(kRounds <= kSpreadStride, "a round count per word of a slot line");
constexpr int kCtlWords = CTL_N + kSpreadWords + kSegs;  // int64 words (the table: 2 kSegs int32)

// Largest degree of tiers 0..3 (a tuning choice bounded by T0_DEG .. T3_DEG).
struct TierCuts {
    int32_t c[4];
};

__device__ inline int tier_of(int32_t d, const TierCuts& tc)
{
    return d <= tc.c[0] ? 0 : d <= tc.c[1] ? 1 : d <= tc.c[2] ? 2 : d <= tc.c[3] ? 3 : 4;
}

// ---------------------------------------------------------------- schedule
// segment = tier * S + class; nodes of jobs that do not take part get segment
// kSegs (sorted behind every segment).  The sort key is 2 * segment + (tier-0
// node of degree > T0_NARROW).
// For batches, jmax[j] receives the largest degree among job j's scheduled
// nodes (one atomic per wavefront when the wavefront's nodes share a job).
__global__ __launch_bounds__(kBlock) void k_sched_keys(const int32_t* __restrict__ xadj, int32_t n, uint32_t hsub,
                                                       JobTabs jt, const uint8_t* __restrict__ gpart, uint32_t level,
                                                       TierCuts tc, uint32_t* __restrict__ key,
                                                       uint32_t* __restrict__ val, int32_t* __restrict__ cnt,
                                                       int32_t* __restrict__ jmax)
{
    __shared__ int32_t h[kSegs + 1];
    if (threadIdx.x <= kSegs) h[threadIdx.x] = 0;
    __syncthreads();
    // grid-stride over a capped grid (uniform trip count: every lane reaches the
    // wavefront reductions); each block adds its kSegs + 1 counts once
    for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x; v0 < n; v0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = v0 + threadIdx.x;
        const bool in = v < n;
        int32_t j = -1, d = 0;
        if (in) {
            uint32_t hs = hsub, vl = (uint32_t)v;
            bool takes_part = true;
            if (jt.gid) {
                j = jt.gid[v];
                hs = hash_step(hash_step(jt.ghash[j], TAG_SUB, 1), level, 2);
                vl = (uint32_t)(v - jt.noff[j]);
                takes_part = !gpart || gpart[j];
            }
            const uint32_t s = hash_step(hs, vl, 3) % kSub;
            d = xadj[v + 1] - xadj[v];
            const uint32_t t = (uint32_t)tier_of(d, tc);
            const uint32_t k = takes_part ? t * kSub + s : (uint32_t)kSegs;
            key[v] = 2 * k + (t == 0 && d > T0_NARROW ? 1u : 0u);  // narrow tier-0 nodes first in their segment
            val[v] = (uint32_t)v;
            atomicAdd(&h[k], 1);
            if (!takes_part) j = -1;
        }
        if (jmax) {
            // lanes without a scheduled node carry j = -1
            const uint64_t live = ballot64(j >= 0);
            if (live) {
                const int32_t j0 = __shfl(j, __ffsll((unsigned long long)live) - 1, 64);
                if (ballot64(j >= 0 && j != j0) == 0) {
                    int32_t m = j >= 0 ? d : 0;
                    for (int q = 32; q > 0; q >>= 1) m = max(m, __shfl_xor(m, q, 64));
                    if ((threadIdx.x & 63) == 0) atomicMax(&jmax[j0], m);
                } else if (j >= 0) {
                    atomicMax(&jmax[j], d);
                }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x <= kSegs && h[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], h[threadIdx.x]);
}

// Hub sizing (the hub tier is described at k_hub_plan).
constexpr int kHubTS = 8192;        // slots of the LDS table of a partition, at most (kmp_tuning)
constexpr int kHubRun = 4096;       // entries of a run (k_hub_split)
constexpr int kHubPartAvg = 1024;   // entries per label partition, on average
constexpr int kHubMaxPart = 1024;   // label partitions of a hub, at most
constexpr int kHubPart = 8;
constexpr uint64_t kEmptySlot = 0xFFFFFFFF00000000ull;

__host__ __device__ inline int64_t hub_runs(int64_t d) { return (d + kHubRun - 1) / kHubRun; }

__host__ __device__ inline int32_t hub_parts(int64_t d)
{
    const int64_t p = (d + kHubPartAvg - 1) / kHubPartAvg;
    return (int32_t)(p < 1 ? 1 : p > kHubMaxPart ? kHubMaxPart : p);
}

__host__ __device__ inline int64_t hub_region(int64_t d)
{
    const int64_t words = hub_runs(d) * (hub_parts(d) + 1) + hub_parts(d);  // int32 words after the slots
    return 5 * d + (words + 1) / 2;
}

// Region size of every hub (8-byte slots).
__global__ void k_hub_slots(const int32_t* __restrict__ xadj, const int32_t* __restrict__ hubs, int32_t nh,
                            int64_t* __restrict__ slots)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nh) return;
    const int32_t v = hubs[i];
    slots[i] = hub_region(xadj[v + 1] - xadj[v]);
}

// The partition totals of every hub start at zero (the other parts of a region
// are written before they are read).
__global__ void k_hub_zero(const int32_t* __restrict__ xadj, const int32_t* __restrict__ hubs, int32_t nh,
                           const int64_t* __restrict__ off_by_node, uint64_t* __restrict__ tab)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nh) return;
    const int32_t v = hubs[i];
    const int64_t d = xadj[v + 1] - xadj[v];
    const int32_t P = hub_parts(d);
    uint32_t* ptot = reinterpret_cast<uint32_t*>(tab + off_by_node[v] + 5 * d) + hub_runs(d) * (P + 1);
    for (int32_t q = 0; q < P; ++q) ptot[q] = 0;
}

// region offset of every hub, indexed by node id (lists of later rounds are compacted)
__global__ void k_hub_scatter(const int32_t* __restrict__ hubs, const int64_t* __restrict__ slots,
                              const int64_t* __restrict__ incl, int32_t nh, int64_t* __restrict__ off_by_node)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nh) off_by_node[hubs[i]] = incl[i] - slots[i];
}

// Visit order of the asynchronous LP (paper Sec. 5.1 "Iteration Order"): the
// buckets' random chunks are the sub-round hash classes, taken one after
// another; inside a class the nodes go by degree bucket floor(log2 d) (degree
// 0 with bucket 0), then id.  A rating tier takes whole buckets (tier t the
// buckets up to blim[t]), so the class-s nodes of tier t are one contiguous
// segment (t, s) in (bucket, id) order.  The sort key is 32 * segment +
// bucket; nodes of jobs that do not take part get segment kSegs.
struct BucketCuts {
    int32_t blim[4];
};

__device__ inline int deg_bucket(int32_t d) { return d <= 1 ? 0 : 31 - __clz(d); }

__global__ __launch_bounds__(kBlock) void k_async_keys(const int32_t* __restrict__ xadj, int32_t n, uint32_t hsub,
                                                       JobTabs jt, const uint8_t* __restrict__ gpart, uint32_t level,
                                                       BucketCuts bc, uint32_t* __restrict__ key,
                                                       uint32_t* __restrict__ val, int32_t* __restrict__ cnt)
{
    __shared__ int32_t h[kSegs + 1];
    if (threadIdx.x <= kSegs) h[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        uint32_t hs = hsub, vl = (uint32_t)v;
        bool takes = true;
        if (jt.gid) {  // the class hash of the node's own job, on its job-local id
            const int32_t j = jt.gid[v];
            hs = hash_step(hash_step(jt.ghash[j], TAG_SUB, 1), level, 2);
            vl = (uint32_t)(v - jt.noff[j]);
            takes = !gpart || gpart[j];
        }
        const uint32_t cls = hash_step(hs, vl, 3) % kSub;
        const int b = deg_bucket(xadj[v + 1] - xadj[v]);
        int t = kTiers - 1;
        for (int q = kTiers - 2; q >= 0; --q)
            if (b <= bc.blim[q]) t = q;
        const uint32_t seg = takes ? (uint32_t)t * kSub + cls : (uint32_t)kSegs;
        key[v] = 32 * seg + (uint32_t)b;
        val[v] = (uint32_t)v;
        atomicAdd(&h[seg], 1);
    }
    __syncthreads();
    if (threadIdx.x <= kSegs && h[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], h[threadIdx.x]);
}

// ---------------------------------------------------------------- rating
struct Key3 {
    uint32_t r, h, k;  // rating (0 = none), hash, label
};

__device__ inline bool better(const Key3& a, const Key3& b)
{
    if (a.r != b.r) return a.r > b.r;
    if (a.h != b.h) return a.h < b.h;
    return a.k < b.k;
}

// One DPP step of the group argmax; lanes the step does not write see their own key.
template <int CTRL, int ROWS>
__device__ inline void best_step(Key3& a)
{
    Key3 b;
    b.r = (uint32_t)__builtin_amdgcn_update_dpp((int)a.r, (int)a.r, CTRL, ROWS, 0xF, false);
    b.h = (uint32_t)__builtin_amdgcn_update_dpp((int)a.h, (int)a.h, CTRL, ROWS, 0xF, false);
    b.k = (uint32_t)__builtin_amdgcn_update_dpp((int)a.k, (int)a.k, CTRL, ROWS, 0xF, false);
    if (better(b, a)) a = b;
}

// Best key of a group of WIDTH = 16 (one row) or 64 lanes, in every lane of the
// group: row butterflies, then for 64 lanes row_bcast:15 / row_bcast:31 and
// lane 63's result to every lane (`better` is a strict total order, so the
// order of the comparisons does not matter).  Every lane must be active.
template <int WIDTH>
__device__ inline Key3 group_best(Key3 a)
{
    static_assert(WIDTH == 16 || WIDTH == 64, "DPP groups are rows or the wavefront");
    best_step<0xB1, 0xF>(a);   // quad_perm [1,0,3,2]
    best_step<0x4E, 0xF>(a);   // quad_perm [2,3,0,1]
    best_step<0x141, 0xF>(a);  // row_half_mirror
    best_step<0x140, 0xF>(a);  // row_mirror
    if (WIDTH == 64) {
        best_step<0x142, 0xA>(a);  // row_bcast:15
        best_step<0x143, 0xC>(a);  // row_bcast:31
        a.r = (uint32_t)__builtin_amdgcn_readlane((int)a.r, 63);
        a.h = (uint32_t)__builtin_amdgcn_readlane((int)a.h, 63);
        a.k = (uint32_t)__builtin_amdgcn_readlane((int)a.k, 63);
    }
    return a;
}

struct RateArgs {
    const int32_t* xadj;
    const int32_t* adjncy;
    const int32_t* vwgt;
    const int32_t* adjwgt;
    const int32_t* label;
    const int64_t* wt;
    const int64_t* cap_vec;
    int64_t cap_scalar;
    const uint8_t* active;  // NULL = every listed node is rated; else nodes with active[v] == stamp
    uint8_t stamp;
    uint32_t hpre;          // H prefix over (seed; tag, level, round)
    int32_t* prop;          // [n], -1 = no proposal
    uint32_t* fav;          // [n] or NULL
    uint32_t* demand;       // [nlab]
    int64_t* counters;      // spread counter: rated edges
    int64_t* bytes_ctr;     // algorithmic bytes of this launch's class
    const int64_t* ctl;     // round control (abort flag) or NULL
    const int32_t* list;    // node lists, segments described by segtab
    const int32_t* segtab;  // [kSegs offsets][kSegs counts]
    int seg;
    // hubs
    uint64_t* hub_tab;       // per hub a region of hub_region(d) 8-byte slots (layout at k_hub_split)
    const int64_t* hub_off;  // by node id: first slot of the hub's region
    int32_t* hub_plan;       // [count + 1]: first run of each hub of the launch's segment, then the total
    int32_t* hub_pplan;      // [count + 1]: the same for the hubs' label partitions
    int32_t hub_ts;          // slots of a partition's LDS table (a power of two, at most kHubTS)
    uint32_t* hub_part;      // per label partition: its best keys and own rating (kHubPart words)
    // balance mode (over != NULL): rate the nodes of overloaded blocks only,
    // targets must be non-overloaded; write best target / gain
    const uint8_t* over;
    int32_t* bal_t;
    int64_t* bal_d;
    // batches (gid != NULL): per-job seed hash, label offset and scalar cap;
    // the per-node prefix is H(seed_job; tag, level, round)
    const int32_t* gid;
    const uint32_t* ghash;
    const int32_t* loff;
    const int64_t* gcap;
    uint32_t tag, level, round;
    // byte sizes of adjncy, label and wt for buffer loads (bufok: all below 2^31,
    // so every byte offset fits the 32-bit offset of a buffer load)
    uint32_t nr_adj, nr_lab, nr_wt;
    int32_t bufok;
    // asynchronous LP (amode != 0): a node that finds a better admissible label
    // moves at once.  1: fetch-and-add on the two weights (clustering: the bound
    // was checked against the weights the node read, so concurrent moves may
    // exceed it); 2: compare-and-swap on the target's weight keeps the bound
    // strictly (refinement).  label_w aliases label; a mover gets mflag[v] =
    // stamp and is counted in moved_ctr (spread counter).
    int32_t amode;
    int32_t* label_w;
    uint8_t* mflag;
    int64_t* moved_ctr;
};

// Buffer loads for gathers (gfx9 raw buffer descriptor): an offset at or past
// the buffer's size returns 0 without a memory access, so lanes with nothing
// to load take part in a gather without touching memory.
constexpr int kBufMiss = (int)0xFFFFFFF0u;
// the miss offset of 16-byte loads: at or past every buffer size here (below
// 2^31), and offset + 16 does not wrap
constexpr int kBufMiss16 = (int)0x80000000u;
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// Per-node part of the rating key: hash prefix, label offset, scalar cap.
struct NodeKey {
    uint32_t hp, lo;
    int64_t cap;
};

__device__ inline NodeKey node_key(const RateArgs& a, int32_t v)
{
    if (!a.gid) return NodeKey{a.hpre, 0u, a.cap_scalar};
    const int32_t j = a.gid[v];
    return NodeKey{hash3(a.ghash[j], a.tag, a.level, a.round), (uint32_t)a.loff[j],
                   a.gcap ? a.gcap[j] : a.cap_scalar};
}

__device__ inline bool aborted(const RateArgs& a) { return a.ctl && a.ctl[CTL_ABORT] != 0; }

__device__ inline bool node_selected(const RateArgs& a, int32_t v)
{
    if (a.over) return a.over[a.label[v]] != 0;
    return !a.active || a.active[v] == a.stamp;
}

// Asynchronous move of v from `own` to t (weight cv); returns 1 if it moved.
__device__ inline int async_move(const RateArgs& a, int32_t v, uint32_t own, uint32_t t, int64_t cv)
{
    unsigned long long* w = reinterpret_cast<unsigned long long*>(const_cast<int64_t*>(a.wt));
    if (a.amode == 2) {
        const int64_t cap = a.cap_vec ? a.cap_vec[t] : a.gcap ? a.gcap[a.gid[v]] : a.cap_scalar;
        unsigned long long old = w[t];
        // every failed exchange returns a weight another move wrote, and a launch
        // moves every node at most once, so the loop ends
        while ((int64_t)old + cv <= cap) {
            const unsigned long long seen = atomicCAS(&w[t], old, old + (unsigned long long)cv);
            if (seen == old) break;
            old = seen;
        }
        if ((int64_t)old + cv > cap) return 0;
    } else {
        atomicAdd(&w[t], (unsigned long long)cv);
    }
    atomicAdd(&w[own], (unsigned long long)(-cv));
    a.label_w[v] = (int32_t)t;
    a.mflag[v] = a.stamp;
    return 1;
}

// Returns 1 if the node moved (asynchronous mode), else 0.
__device__ inline int write_result(const RateArgs& a, int32_t v, uint32_t own, const Key3& fav, const Key3& adm,
                                   uint32_t rown, int64_t cv)
{
    if (a.over) {
        a.bal_t[v] = adm.r ? (int32_t)adm.k : -1;
        a.bal_d[v] = adm.r ? (int64_t)adm.r - (int64_t)rown : -(int64_t)rown;
        return 0;
    }
    if (a.fav) a.fav[v] = fav.r ? fav.k : kNone;
    if (adm.r > rown) {
        if (a.amode) return async_move(a, v, own, adm.k, cv);
        a.prop[v] = (int32_t)adm.k;
        atomicAdd(&a.demand[adm.k], (uint32_t)cv);
    }
    return 0;
}

// Rates a thread's slots of a node's label table, slot(j, K, V) giving the
// (label, rating) of slot j (K = EMPTY for none) for j = j0, j0 + step, ... <
// end: the own rating and the favoured label directly, the best admissible
// label with the weights (and caps, overload flags) of B slots gathered at
// once.  A label is weighed if it beats the admissible label found before its
// batch and taken if it is admissible and still beats it, so the result is
// that of weighing every label in slot order.  The gathers are unconditional
// (a slot that needs none reads the own label's weight), so the B loads of a
// batch are in flight together instead of one after another.
template <int B, bool CAPV, bool BAL, class Slot>
__device__ inline void rate_slots_t(const RateArgs& a, const NodeKey& nk, uint32_t own, int64_t cv, int64_t j0,
                                    int64_t end, int64_t step, Slot&& slot, Key3& fav, Key3& adm, uint32_t& rown)
{
    for (; j0 < end; j0 += B * step) {
        uint32_t K[B], V[B], Hs[B];
        bool need[B];
#pragma unroll
        for (int q = 0; q < B; ++q) {
            const int64_t j = j0 + q * step;
            K[q] = EMPTY;
            V[q] = 0;
            slot(j < end ? j : end - 1, K[q], V[q]);
            if (j >= end) K[q] = EMPTY;
        }
#pragma unroll
        for (int q = 0; q < B; ++q) {
            const bool cand = K[q] != EMPTY && K[q] != own;
            if (K[q] == own) rown = V[q];
            Hs[q] = hash_step(nk.hp, K[q] - nk.lo, 4);
            const Key3 c{V[q], Hs[q], K[q]};
            if (cand && better(c, fav)) fav = c;
            need[q] = cand && better(c, adm);
        }
        int64_t w[B], cap[B];
        bool ov[B];
#pragma unroll
        for (int q = 0; q < B; ++q) {
            const uint32_t l = need[q] ? K[q] : own;
            w[q] = a.wt[l];
            cap[q] = CAPV ? a.cap_vec[l] : nk.cap;
            ov[q] = BAL ? a.over[l] != 0 : false;
        }
#pragma unroll
        for (int q = 0; q < B; ++q) {
            const Key3 c{V[q], Hs[q], K[q]};
            if (need[q] && better(c, adm) && w[q] + cv <= cap[q] && !ov[q]) adm = c;
        }
    }
}

template <int B, class Slot>
__device__ inline void rate_slots(const RateArgs& a, const NodeKey& nk, uint32_t own, int64_t cv, int64_t j0,
                                  int64_t end, int64_t step, Slot&& slot, Key3& fav, Key3& adm, uint32_t& rown)
{
    if (a.cap_vec) {
        if (a.over) rate_slots_t<B, true, true>(a, nk, own, cv, j0, end, step, slot, fav, adm, rown);
        else rate_slots_t<B, true, false>(a, nk, own, cv, j0, end, step, slot, fav, adm, rown);
    } else {
        if (a.over) rate_slots_t<B, false, true>(a, nk, own, cv, j0, end, step, slot, fav, adm, rown);
        else rate_slots_t<B, false, false>(a, nk, own, cv, j0, end, step, slot, fav, adm, rown);
    }
}

// Per-block statistics: rated entries, algorithmic bytes and (asynchronous
// mode) moves, summed per wavefront, then per block in LDS, one atomic each per
// block (a wave rates fewer than 2^31 entries: a single graph has fewer,
// batches stay below 2^31).  Every thread of the block must call this.
__device__ inline void flush_stats(const RateArgs& a, int64_t nodes_in, int64_t edges_in, int64_t moves_in = 0)
{
    __shared__ unsigned long long s_stat[3];
    if (threadIdx.x == 0) s_stat[0] = s_stat[1] = s_stat[2] = 0;
    __syncthreads();
    const uint32_t edges = group_sum_u32<64>((uint32_t)edges_in);
    const uint32_t nodes = group_sum_u32<64>((uint32_t)nodes_in);
    const uint32_t moves = a.moved_ctr ? group_sum_u32<64>((uint32_t)moves_in) : 0u;  // uniform branch
    if ((threadIdx.x & 63) == 0 && (nodes | moves)) {
        atomicAdd(&s_stat[0], (unsigned long long)edges);
        atomicAdd(&s_stat[1], (unsigned long long)nodes);
        atomicAdd(&s_stat[2], (unsigned long long)moves);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t e = (int64_t)s_stat[0], nd = (int64_t)s_stat[1], mv = (int64_t)s_stat[2];
        if (nd) {
            spread_add(a.counters, e);
            spread_add(a.bytes_ctr, 25 * nd + (a.adjwgt ? 12 : 8) * e);
        }
        if (a.moved_ctr && mv) spread_add(a.moved_ctr, mv);
    }
}

// Branch-free best-key update.  A candidate's key is (rating << 32 | ~hash):
// a larger key is a larger rating, or an equal rating with a smaller hash;
// equal keys fall back to the smaller label.  Key 0 marks "no candidate" and
// never wins (a real rating is at least 1).
__device__ inline void take_best(uint64_t& bk, uint32_t& bl, uint64_t key, uint32_t lab)
{
    const bool t = key > bk || (key == bk && lab < bl);
    bk = t ? key : bk;
    bl = t ? lab : bl;
}

__device__ inline Key3 key3_of(uint64_t key, uint32_t lab)
{
    return Key3{(uint32_t)(key >> 32), ~(uint32_t)key, lab};
}

// Batcher's odd-even merge sort as a compare-exchange network over N register
// slots (19 exchanges for N = 8, 63 for N = 16): labels ascending, EMPTY last.
// W: the weights travel with their labels (else every weight is 1).  Slots
// that hold the constant EMPTY fold their exchanges away at compile time.
template <int N, bool W>
__device__ inline void sort_slots(uint32_t (&k)[N], uint32_t (&w)[N])
{
#pragma unroll
    for (int p = 1; p < N; p <<= 1) {
#pragma unroll
        for (int s = p; s >= 1; s >>= 1) {
#pragma unroll
            for (int j = s % p; j + s < N; j += 2 * s) {
#pragma unroll
                for (int i = 0; i < s; ++i) {
                    const int x = i + j, y = i + j + s;
                    if (y < N && x / (2 * p) == y / (2 * p)) {
                        const uint32_t kx = k[x], ky = k[y];
                        k[x] = kx < ky ? kx : ky;
                        k[y] = kx < ky ? ky : kx;
                        if constexpr (W) {
                            const uint32_t wx = w[x], wy = w[y];
                            w[x] = kx > ky ? wy : wx;
                            w[y] = kx > ky ? wx : wy;
                        }
                    }
                }
            }
        }
    }
}

// The rating of one node from its neighbours' labels and edge weights in the
// first L of N register slots (N = 4, 8 or 16 >= L; slots at or past the
// node's degree hold EMPTY): sort the slots by label, sum every run of equal
// labels into its last slot, then walk the run ends once for the own label's
// rating, the favoured label (FAV) and the best admissible label.
// wt_of(l), cap_of(l), over_of(l): label l's weight, cap and overload flag;
// the hash takes l - hoff.
template <int N, int L, bool W, bool FAV, class WT, class CAP, class OV>
__device__ inline void choose_slots(const uint32_t (&lab_in)[L], const uint32_t (&w_in)[L], uint32_t own,
                                    uint32_t hp, uint32_t hoff, int64_t cv, WT wt_of, CAP cap_of, OV over_of,
                                    Key3& fav, Key3& adm, uint32_t& rown)
{
    uint32_t lab[N], w[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        lab[j] = j < L ? lab_in[j] : EMPTY;
        w[j] = j < L ? w_in[j] : 1u;
    }
    sort_slots<N, W>(lab, w);
#pragma unroll
    for (int j = 1; j < L; ++j) w[j] += lab[j] == lab[j - 1] ? w[j - 1] : 0u;
    uint32_t cand[L];
    int64_t wk[L];
#pragma unroll
    for (int j = 0; j < L; ++j) {
        const uint32_t K = lab[j];
        const bool end = j == N - 1 || lab[j + 1] != K;
        const bool real = end && K != EMPTY;
        rown = real && K == own ? w[j] : rown;
        cand[j] = real && K != own ? K : EMPTY;
    }
    // weights of the candidates (wt_of sees EMPTY for the other slots)
#pragma unroll
    for (int j = 0; j < L; ++j) wk[j] = wt_of(cand[j]);
    uint64_t fk = 0, ak = 0;
    uint32_t fl = 0, al = 0;
#pragma unroll
    for (int j = 0; j < L; ++j) {
        const uint32_t K = lab[j];
        const bool c = cand[j] != EMPTY;
        const uint32_t h = hash_step(hp, K - hoff, 4);
        const uint64_t key = c ? ((uint64_t)w[j] << 32) | (uint64_t)(~h) : 0ull;
        if constexpr (FAV) take_best(fk, fl, key, K);
        const uint32_t l = c ? K : own;
        const bool fits = c && wk[j] + cv <= cap_of(l) && !over_of(l);
        take_best(ak, al, fits ? key : 0ull, K);
    }
    fav = key3_of(fk, fl);
    adm = key3_of(ak, al);
}

// Tier 0: one lane per node; the neighbours' labels and edge weights live in
// L registers (L >= the largest degree in the wavefront).  Gathers are
// unconditional (clamped indices, or buffer loads in which lanes past their
// degree miss), so each batch is issued back to back with one wait.  EW: edge
// weights present; CAPV: per-label caps; BAL: balance mode.
template <int L, bool EW, bool CAPV, bool BAL, bool BUF>
__device__ inline int rate_lane_node(const RateArgs& a, int32_t v, uint32_t own, int32_t e0, int32_t d, int64_t cv,
                                     const NodeKey& nk)
{
    constexpr int N = L <= 4 ? 4 : L <= 8 ? 8 : 16;
    static_assert(L % 4 == 0, "rows are loaded four entries at a time");
    uint32_t lab[L], w[L];
#pragma unroll
    for (int j = 0; j < L; ++j) {
        lab[j] = EMPTY;
        w[j] = 1u;
    }
    if (d > 0) {
        int32_t u[L];
        if constexpr (BUF) {
            // the row four entries per load (dword-aligned 16-byte loads); a load that
            // would reach past the end of adjncy misses and its entries are fetched one
            // by one below (only the last rows of the array); lanes past their degree miss
            const __amdgpu_buffer_rsrc_t radj = buf_rsrc(a.adjncy, a.nr_adj), rlab = buf_rsrc(a.label, a.nr_lab);
            const uint32_t m = a.nr_adj >> 2;
            bool tail = false;
#pragma unroll
            for (int q = 0; q < L / 4; ++q) {
                const bool inrow = 4 * q < d;
                const bool whole = (uint32_t)(e0 + 4 * q + 4) <= m;
                tail = tail || (inrow && !whole);
                const auto x = __builtin_amdgcn_raw_buffer_load_b128(radj, inrow && whole ? (e0 + 4 * q) * 4 : kBufMiss16,
                                                                     0, 0);
                u[4 * q] = (int32_t)x[0];
                u[4 * q + 1] = (int32_t)x[1];
                u[4 * q + 2] = (int32_t)x[2];
                u[4 * q + 3] = (int32_t)x[3];
            }
            if (tail) {
#pragma unroll
                for (int j = 0; j < L; ++j)
                    if (j < d && (uint32_t)(e0 + (j & ~3) + 4) > m)
                        u[j] = __builtin_amdgcn_raw_buffer_load_b32(radj, (e0 + j) * 4, 0, 0);
            }
#pragma unroll
            for (int j = 0; j < L; ++j) {
                const uint32_t l =
                    (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(rlab, j < d ? u[j] * 4 : kBufMiss, 0, 0);
                lab[j] = j < d ? l : EMPTY;
            }
            if constexpr (EW) {
                const __amdgpu_buffer_rsrc_t rew = buf_rsrc(a.adjwgt, a.nr_adj);
#pragma unroll
                for (int q = 0; q < L / 4; ++q) {
                    const bool inrow = 4 * q < d;
                    const bool whole = (uint32_t)(e0 + 4 * q + 4) <= m;
                    const auto x = __builtin_amdgcn_raw_buffer_load_b128(
                        rew, inrow && whole ? (e0 + 4 * q) * 4 : kBufMiss16, 0, 0);
                    w[4 * q] = x[0];
                    w[4 * q + 1] = x[1];
                    w[4 * q + 2] = x[2];
                    w[4 * q + 3] = x[3];
                }
                if (tail) {
#pragma unroll
                    for (int j = 0; j < L; ++j)
                        if (j < d && (uint32_t)(e0 + (j & ~3) + 4) > m)
                            w[j] = __builtin_amdgcn_raw_buffer_load_b32(rew, (e0 + j) * 4, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < L; ++j) u[j] = a.adjncy[e0 + (j < d ? j : d - 1)];
#pragma unroll
            for (int j = 0; j < L; ++j) {
                const uint32_t l = (uint32_t)a.label[u[j]];
                lab[j] = j < d ? l : EMPTY;
            }
            if constexpr (EW) {
#pragma unroll
                for (int j = 0; j < L; ++j) w[j] = (uint32_t)a.adjwgt[e0 + (j < d ? j : d - 1)];
            }
        }
    }
    // candidate weights: through a buffer in which EMPTY misses (no memory access),
    // else a plain load redirected to the own label
    auto wt_of = [&](uint32_t l) -> int64_t {
        if constexpr (BUF) {
            const auto x = __builtin_amdgcn_raw_buffer_load_b64(buf_rsrc(a.wt, a.nr_wt),
                                                                l != EMPTY ? (int)(l * 8u) : kBufMiss, 0, 0);
            return (int64_t)(((uint64_t)(uint32_t)x[1] << 32) | (uint32_t)x[0]);
        }
        return a.wt[l != EMPTY ? l : own];
    };
    auto cap_of = [&](uint32_t l) -> int64_t { return CAPV ? a.cap_vec[l] : nk.cap; };
    auto over_of = [&](uint32_t l) -> bool { return BAL ? a.over[l] != 0 : false; };
    Key3 fav, adm;
    uint32_t rown = 0;
    if (a.fav)  // clustering keeps the favoured cluster too (uniform branch)
        choose_slots<N, L, EW, true>(lab, w, own, nk.hp, nk.lo, cv, wt_of, cap_of, over_of, fav, adm, rown);
    else
        choose_slots<N, L, EW, false>(lab, w, own, nk.hp, nk.lo, cv, wt_of, cap_of, over_of, fav, adm, rown);
    return write_result(a, v, own, fav, adm, rown, cv);
}

// Rounds after the first (and balancing) rate only the selected nodes of a
// list: every tile of blockDim.x entries is compacted in LDS first, so the
// selected nodes fill the leading wavefronts and the others have no work.
template <bool EW, bool CAPV, bool BAL, bool BUF>
__global__ __launch_bounds__(kBlock) void k_rate_lane(RateArgs a)
{
    __shared__ int32_t s_v[kBlock];
    __shared__ uint32_t s_cnt[kBlock / 64];
    if (aborted(a)) return;
    const int32_t off = a.segtab[a.seg], count = a.segtab[kSegs + a.seg];
    const bool filter = BAL || a.active != nullptr;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = (int)(blockDim.x >> 6);
    int64_t edges = 0, nodes = 0, moves = 0;
    for (int64_t base = (int64_t)xcd_block() * blockDim.x; base < count; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = base + tid;
        int32_t v = i < count ? a.list[off + i] : -1;
        if (filter) {
            const bool sel = v >= 0 && node_selected(a, v);
            const uint64_t m = ballot64(sel);
            if (lane == 0) s_cnt[wv] = (uint32_t)__popcll(m);
            __syncthreads();
            uint32_t pre = 0, tot = 0;
            for (int q = 0; q < nw; ++q) {
                const uint32_t c = s_cnt[q];
                pre += q < wv ? c : 0u;
                tot += c;
            }
            if (sel)
                s_v[pre + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))] =
                    v;
            __syncthreads();
            v = (uint32_t)tid < tot ? s_v[tid] : -1;
            __syncthreads();  // the tables are rewritten by the next tile
        }
        if (!ballot64(v >= 0)) continue;  // uniform in the wavefront
        uint32_t own = 0;
        int32_t e0 = 0, d = 0;
        int64_t cv = 0;
        if (v >= 0) {
            own = (uint32_t)a.label[v];
            e0 = a.xadj[v];
            d = a.xadj[v + 1] - e0;
            cv = a.vwgt ? a.vwgt[v] : 1;
        }
        // register slots for the largest degree in the wavefront (every lane is active here)
        const uint32_t dmax = wave_max_u32_dpp((uint32_t)d);
        if (v >= 0) {
            const NodeKey nk = node_key(a, v);
            if (dmax <= 4) moves += rate_lane_node<4, EW, CAPV, BAL, BUF>(a, v, own, e0, d, cv, nk);
            else if (dmax <= 8) moves += rate_lane_node<8, EW, CAPV, BAL, BUF>(a, v, own, e0, d, cv, nk);
            else if (dmax <= 12) moves += rate_lane_node<12, EW, CAPV, BAL, BUF>(a, v, own, e0, d, cv, nk);
            else moves += rate_lane_node<T0_DEG, EW, CAPV, BAL, BUF>(a, v, own, e0, d, cv, nk);
            edges += d;
            nodes += 1;
        }
    }
    flush_stats(a, nodes, edges, moves);
}

// As lds_insert, but every slot is probed at most once: false if the table is
// full of other labels (the entry is then not inserted).
__device__ inline bool lds_try_insert(uint32_t* keys, uint32_t* vals, int bits, uint32_t K, uint32_t w)
{
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t h = slot_of(K, bits);
    for (uint32_t t = 0; t <= mask; ++t) {
        const uint32_t old = atomicCAS(&keys[h], EMPTY, K);
        if (old == EMPTY || old == K) {
            atomicAdd(&vals[h], w);
            return true;
        }
        h = (h + 1) & mask;
    }
    return false;
}

__device__ inline void lds_insert(uint32_t* keys, uint32_t* vals, int bits, uint32_t K, uint32_t w)
{
    const uint32_t mask = (1u << bits) - 1u;
    uint32_t h = slot_of(K, bits);
    while (true) {
        uint32_t old = atomicCAS(&keys[h], EMPTY, K);
        if (old == EMPTY || old == K) {
            atomicAdd(&vals[h], w);
            return;
        }
        h = (h + 1) & mask;
    }
}

// Orders the LDS accesses of a group of G lanes: a group of at most 64 lanes
// lies in one wavefront, whose LDS operations take effect in issue order, so
// only the compiler has to be kept from moving them across; a larger group
// spans the workgroup.
template <int G>
__device__ inline void group_sync()
{
    if constexpr (G <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    } else {
        __syncthreads();
    }
}

// Tiers 1-3: G lanes per node, 2^HB slots per node in LDS, 256 threads.  Groups
// of at most 64 lanes synchronise only within their wavefront, so the waves of
// a workgroup rate their nodes independently.  A lane loads four of its row's
// entries (and their labels) before inserting any, keeping four gathers in
// flight.
template <int G, int HB>
__global__ __launch_bounds__(kBlock) void k_rate_lds(RateArgs a)
{
    constexpr int GPB = kBlock / G;
    constexpr int HS = 1 << HB;
    __shared__ uint32_t s_keys[GPB * HS];
    __shared__ uint32_t s_vals[GPB * HS];
    __shared__ Key3 s_red[2][4];
    __shared__ uint32_t s_rown[4];
    // a workgroup per node: the occupied slots of its table are listed before they are
    // weighed (at most 2^(HB-1) labels), so the weighing visits labels, not slots
    constexpr bool kList = G == kBlock;
    __shared__ uint16_t s_occ[kList ? HS / 2 : 1];
    __shared__ int32_t s_nocc;
    if (aborted(a)) return;
    const int32_t off = a.segtab[a.seg], count = a.segtab[kSegs + a.seg];
    const int tid = threadIdx.x;
    const int grp = tid / G, gl = tid % G;
    uint32_t* keys = s_keys + grp * HS;
    uint32_t* vals = s_vals + grp * HS;
    int64_t edges = 0, nodes = 0, moves = 0;
    for (int64_t base = (int64_t)xcd_block() * GPB; base < count; base += (int64_t)gridDim.x * GPB) {
        const int64_t i = base + grp;
        int32_t v = -1;
        if (i < count) {
            v = a.list[off + i];
            if (!node_selected(a, v)) v = -1;
        }
        // the node's table: the smallest power of two of at least 2 d slots (at most
        // HS, which the tier's degree range guarantees); only those slots are cleared
        // and scanned
        int32_t e0 = 0, e1 = 0;
        if (v >= 0) {
            e0 = a.xadj[v];
            e1 = a.xadj[v + 1];
        }
        int bits = 1;
        while ((1 << bits) < 2 * (e1 - e0) && bits < HB) ++bits;
        const int hsn = v >= 0 ? 1 << bits : 0;
        for (int j = gl; j < hsn; j += G) {
            keys[j] = EMPTY;
            vals[j] = 0;
        }
        if (kList && tid == 0) s_nocc = 0;
        group_sync<G>();
        if (v >= 0) {
            // at most d distinct labels in at least 2 d slots: every insert finds its
            // slot within one sweep of the table
            // a lane's whole share of the row (the tier's largest degree / G entries) in one
            // batch, every load unconditional (indices clamped into the row)
            constexpr int U = (1 << (HB - 1)) / G;
            for (int32_t e = e0 + gl; e < e1; e += U * G) {
                int32_t u[U];
                uint32_t K[U], w[U];
#pragma unroll
                for (int q = 0; q < U; ++q) u[q] = a.adjncy[e + q * G < e1 ? e + q * G : e1 - 1];
#pragma unroll
                for (int q = 0; q < U; ++q) K[q] = (uint32_t)a.label[u[q]];
                if (a.adjwgt) {
#pragma unroll
                    for (int q = 0; q < U; ++q) w[q] = (uint32_t)a.adjwgt[e + q * G < e1 ? e + q * G : e1 - 1];
                } else {
#pragma unroll
                    for (int q = 0; q < U; ++q) w[q] = 1u;
                }
#pragma unroll
                for (int q = 0; q < U; ++q)
                    if (e + q * G < e1) lds_try_insert(keys, vals, bits, K[q], w[q]);
            }
            if (gl == 0) {
                edges += e1 - e0;
                nodes += 1;
            }
        }
        group_sync<G>();
        int32_t nocc = 0;
        if constexpr (kList) {
            for (int j = gl; j < hsn; j += G)
                if (keys[j] != EMPTY) s_occ[atomicAdd(&s_nocc, 1)] = (uint16_t)j;
            __syncthreads();
            nocc = s_nocc;
        }
        Key3 fav{0, 0, 0}, adm{0, 0, 0};
        uint32_t rown = 0, own = 0;
        int64_t cv = 0;
        if (v >= 0) {
            own = (uint32_t)a.label[v];
            const NodeKey nk = node_key(a, v);
            cv = a.vwgt ? a.vwgt[v] : 1;
            if constexpr (kList)
                rate_slots<4>(a, nk, own, cv, gl, nocc, G,
                              [&](int64_t q, uint32_t& K, uint32_t& V) {
                                  const int j = s_occ[q];
                                  K = keys[j];
                                  V = vals[j];
                              },
                              fav, adm, rown);
            else
                rate_slots<4>(a, nk, own, cv, gl, hsn, G,
                              [&](int64_t j, uint32_t& K, uint32_t& V) {
                                  K = keys[j];
                                  V = vals[j];
                              },
                              fav, adm, rown);
        }
        if constexpr (G <= 64) {
            fav = group_best<G>(fav);
            adm = group_best<G>(adm);
            rown = group_sum_u32<G>(rown);
        } else {
            fav = group_best<64>(fav);
            adm = group_best<64>(adm);
            rown = group_sum_u32<64>(rown);
            const int w = tid >> 6;
            if ((tid & 63) == 0) {
                s_red[0][w] = fav;
                s_red[1][w] = adm;
                s_rown[w] = rown;
            }
            __syncthreads();
            if (tid == 0) {
                for (int q = 1; q < 4; ++q) {
                    if (better(s_red[0][q], fav)) fav = s_red[0][q];
                    if (better(s_red[1][q], adm)) adm = s_red[1][q];
                    rown += s_rown[q];
                }
            }
        }
        if (v >= 0 && gl == 0) moves += write_result(a, v, own, fav, adm, rown, cv);
        group_sync<G>();  // the table is cleared for the next node only after every read
    }
    flush_stats(a, nodes, edges, moves);
}

// Tier 4: hubs (degree above the tier-3 cut-off).  A hub's entries are summed
// per label in two passes that touch no global hash table:
//   k_hub_plan    one workgroup: for the segment's rated hubs, the first run
//                 (kHubRun entries of the row) and the first label partition
//   k_hub_split   one workgroup per run: the run's labels and edge weights,
//                 counting-sorted in LDS by label partition (P partitions per
//                 hub, about kHubPartAvg entries each), written to the hub's
//                 staging array with the run's partition offsets; the
//                 partition totals are added to the hub's counters
//   k_hub_agg     one workgroup per label partition: its entries from every
//                 run summed per label in an LDS table (a partition of more
//                 entries than the table could hold uses a global table of its
//                 own, sized to never fill), rated, best keys per partition
//   k_hub_final   one wavefront per hub: the best over its partitions, result;
//                 the partition counters are cleared for the next use
// A label's entries all land in one partition, so every step follows the same
// rule as the other tiers (ratings summed per label, the best admissible and
// the favoured label by the strict key order) and the layout changes no result.
// A hub of degree d owns hub_region(d) 8-byte slots: d staging slots (label <<
// 32 | weight), 4 d slots for the overflow tables, then int32 arrays: the run
// offsets [runs][P + 1] and the partition totals [P] (zero between uses).
// Label partition of K among P: a mixing hash of its own (the LDS table slot
// takes the top bits of another multiplicative hash, which must not be constant
// within a partition), scaled to [0, P).
__device__ inline uint32_t hub_part_of(uint32_t K, int32_t P)
{
    return (uint32_t)(((uint64_t)fmix32(K ^ 0x5BD1E995u) * (uint64_t)P) >> 32);
}

__device__ inline int32_t hub_runs_of(const RateArgs& a, int32_t v)
{
    if (!node_selected(a, v)) return 0;
    return (int32_t)hub_runs(a.xadj[v + 1] - a.xadj[v]);
}

// Exclusive prefixes of the rated hubs' run and partition counts.
__global__ __launch_bounds__(kBlock) void k_hub_plan(RateArgs a)
{
    __shared__ int32_t s_wsum[2][kBlock / 64];
    __shared__ int32_t s_carry[2];
    if (aborted(a)) return;
    const int32_t off = a.segtab[a.seg], count = a.segtab[kSegs + a.seg];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid < 2) s_carry[tid] = 0;
    __syncthreads();
    for (int32_t base = 0; base < count; base += kBlock) {
        const int32_t i = base + tid;
        int32_t x[2] = {0, 0};
        if (i < count) {
            const int32_t v = a.list[off + i];
            x[0] = hub_runs_of(a, v);
            x[1] = x[0] ? hub_parts(a.xadj[v + 1] - a.xadj[v]) : 0;
        }
        int32_t incl[2] = {x[0], x[1]};  // inclusive scans within the wavefront
        for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int32_t y = __shfl_up(incl[q], d, 64);
                if (lane >= d) incl[q] += y;
            }
        }
        if (lane == 63) {
            s_wsum[0][wv] = incl[0];
            s_wsum[1][wv] = incl[1];
        }
        __syncthreads();
        int32_t before[2] = {s_carry[0], s_carry[1]};
        for (int q = 0; q < wv; ++q) {
            before[0] += s_wsum[0][q];
            before[1] += s_wsum[1][q];
        }
        if (i < count) {
            a.hub_plan[i] = before[0] + incl[0] - x[0];
            a.hub_pplan[i] = before[1] + incl[1] - x[1];
        }
        __syncthreads();
        if (tid == kBlock - 1) {
            s_carry[0] = before[0] + incl[0];
            s_carry[1] = before[1] + incl[1];
        }
        __syncthreads();
    }
    if (tid == 0) {
        a.hub_plan[count] = s_carry[0];
        a.hub_pplan[count] = s_carry[1];
    }
}

// The hub whose runs (or partitions) contain item ch: the last i with plan[i] <= ch.
__device__ inline int32_t hub_of_chunk(const int32_t* plan, int32_t count, int32_t ch)
{
    int32_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (plan[mid] <= ch) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_hub_split(RateArgs a)
{
    constexpr int PER = kHubRun / kBlock;
    __shared__ uint32_t s_cnt[kHubMaxPart];
    __shared__ uint32_t s_cur[kHubMaxPart];
    __shared__ uint32_t s_wsum[kBlock / 64];
    if (aborted(a)) return;
    const int32_t off = a.segtab[a.seg], count = a.segtab[kSegs + a.seg];
    const int32_t total = count > 0 ? a.hub_plan[count] : 0;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int32_t ch = xcd_block(); ch < total; ch += gridDim.x) {
        const int32_t i = hub_of_chunk(a.hub_plan, count, ch);
        const int32_t v = a.list[off + i];
        const int32_t r = ch - a.hub_plan[i];
        const int64_t e0 = a.xadj[v], d = a.xadj[v + 1] - e0;
        const int32_t P = hub_parts(d);
        const int64_t c0 = e0 + (int64_t)r * kHubRun, c1 = c0 + kHubRun < e0 + d ? c0 + kHubRun : e0 + d;
        uint64_t* reg = a.hub_tab + a.hub_off[v];
        uint32_t* roff = reinterpret_cast<uint32_t*>(reg + 5 * d) + (int64_t)r * (P + 1);
        uint32_t* ptot = reinterpret_cast<uint32_t*>(reg + 5 * d) + hub_runs(d) * (P + 1);
        for (int q = tid; q < P; q += kBlock) s_cnt[q] = 0;
        __syncthreads();
        // every load unconditional (indices clamped into the run), so all are in flight
        uint32_t K[PER], W[PER], pp[PER];
        int32_t u[PER];
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const int64_t e = c0 + (int64_t)t * kBlock + tid;
            u[t] = a.adjncy[e < c1 ? e : c1 - 1];
        }
#pragma unroll
        for (int t = 0; t < PER; ++t) K[t] = (uint32_t)a.label[u[t]];
        if (a.adjwgt) {
#pragma unroll
            for (int t = 0; t < PER; ++t) {
                const int64_t e = c0 + (int64_t)t * kBlock + tid;
                W[t] = (uint32_t)a.adjwgt[e < c1 ? e : c1 - 1];
            }
        } else {
#pragma unroll
            for (int t = 0; t < PER; ++t) W[t] = 1u;
        }
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            const bool in = c0 + (int64_t)t * kBlock + tid < c1;
            pp[t] = in ? hub_part_of(K[t], P) : 0xFFFFFFFFu;
        }
#pragma unroll
        for (int t = 0; t < PER; ++t)
            if (pp[t] != 0xFFFFFFFFu) atomicAdd(&s_cnt[pp[t]], 1u);
        __syncthreads();
        // exclusive prefix of the P counts: four per thread, wavefront scans, wave totals
        uint32_t loc[4], sum = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = 4 * tid + q;
            loc[q] = idx < P ? s_cnt[idx] : 0u;
            sum += loc[q];
        }
        uint32_t incl = sum;
        for (int dd = 1; dd < 64; dd <<= 1) {
            const uint32_t y = __shfl_up(incl, dd, 64);
            if (lane >= dd) incl += y;
        }
        if (lane == 63) s_wsum[wv] = incl;
        __syncthreads();
        uint32_t run = incl - sum;
        for (int q = 0; q < wv; ++q) run += s_wsum[q];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = 4 * tid + q;
            if (idx < P) {
                s_cur[idx] = run;
                roff[idx] = run;
                if (loc[q]) atomicAdd(&ptot[idx], loc[q]);
            }
            run += loc[q];
        }
        if (tid == 0) roff[P] = (uint32_t)(c1 - c0);
        __syncthreads();
        // entries to the staging slots of the run, grouped by partition
        uint64_t* st = reg + (c0 - e0);
#pragma unroll
        for (int t = 0; t < PER; ++t)
            if (pp[t] != 0xFFFFFFFFu) st[atomicAdd(&s_cur[pp[t]], 1u)] = ((uint64_t)K[t] << 32) | W[t];
        __syncthreads();  // the LDS counters are reset for the next run
    }
}

// The LDS table has a.hub_ts slots (keys, then sums), in the launch's dynamic
// shared memory: a smaller table lets more workgroups share a compute unit.
__global__ __launch_bounds__(kBlock) void k_hub_agg(RateArgs a)
{
    extern __shared__ __align__(16) uint32_t s_hub_lds[];
    __shared__ Key3 s_red[2][kBlock / 64];
    __shared__ uint32_t s_rown[kBlock / 64];
    __shared__ int64_t s_sum[2][kBlock / 64];
    __shared__ int32_t s_full;
    __shared__ uint32_t s_pre[kBlock + 1];  // a group of runs: exclusive prefix of their entries in the partition
    __shared__ uint32_t s_beg[kBlock];      // and where the partition starts in each run
    __shared__ uint32_t s_ws[kBlock / 64];
    if (aborted(a)) return;
    const int32_t off = a.segtab[a.seg], count = a.segtab[kSegs + a.seg];
    const int32_t total = count > 0 ? a.hub_pplan[count] : 0;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int32_t pc = xcd_block(); pc < total; pc += gridDim.x) {
        const int32_t i = hub_of_chunk(a.hub_pplan, count, pc);
        const int32_t v = a.list[off + i];
        const int32_t p = pc - a.hub_pplan[i];
        const int64_t d = a.xadj[v + 1] - a.xadj[v];
        const int32_t P = hub_parts(d);
        const int64_t nr = hub_runs(d);
        uint64_t* reg = a.hub_tab + a.hub_off[v];
        const uint32_t* roff = reinterpret_cast<const uint32_t*>(reg + 5 * d);
        const uint32_t* ptot = roff + nr * (P + 1);
        // the partition's entry count and the counts of the partitions before it
        int64_t e_own = 0, e_before = 0;
        for (int q = tid; q < P; q += kBlock) {
            const int64_t c = ptot[q];
            e_own += q == p ? c : 0;
            e_before += q < p ? c : 0;
        }
        for (int dd = 32; dd > 0; dd >>= 1) {
            e_own += __shfl_xor(e_own, dd, 64);
            e_before += __shfl_xor(e_before, dd, 64);
        }
        if (lane == 0) {
            s_sum[0][wv] = e_own;
            s_sum[1][wv] = e_before;
        }
        __syncthreads();
        int64_t E = 0, before = 0;
        for (int q = 0; q < kBlock / 64; ++q) {
            E += s_sum[0][q];
            before += s_sum[1][q];
        }
        const uint32_t own = (uint32_t)a.label[v];
        const int64_t cv = a.vwgt ? a.vwgt[v] : 1;
        const NodeKey nk = node_key(a, v);
        Key3 fav{0, 0, 0}, adm{0, 0, 0};
        uint32_t rown = 0;
        // every run's entries of partition p, in groups of up to kBlock runs: a thread reads
        // one run's offsets, a block scan numbers the group's entries, and thread t takes
        // entries t, t + kBlock, ... (four loads in flight), each found by a binary search
        // over the prefix, so no load waits for another
        auto each_entry = [&](auto&& f) {
            for (int64_t g0 = 0; g0 < nr; g0 += kBlock) {
                const int gn = nr - g0 < kBlock ? (int)(nr - g0) : kBlock;
                uint32_t s0 = 0, cnt = 0;
                if (tid < gn) {
                    const uint32_t* ro = roff + (g0 + tid) * (P + 1);
                    s0 = ro[p];
                    cnt = ro[p + 1] - s0;
                }
                uint32_t incl = cnt;
                for (int dd = 1; dd < 64; dd <<= 1) {
                    const uint32_t y = __shfl_up(incl, dd, 64);
                    if (lane >= dd) incl += y;
                }
                if (lane == 63) s_ws[wv] = incl;
                __syncthreads();
                uint32_t excl = incl - cnt;
                for (int q = 0; q < wv; ++q) excl += s_ws[q];
                s_pre[tid] = excl;
                s_beg[tid] = s0;
                if (tid == kBlock - 1) s_pre[kBlock] = excl + cnt;
                __syncthreads();
                const uint32_t tot = s_pre[kBlock];
                int top = 1;  // the largest power of two below gn (0: a single run)
                while (2 * top < gn) top *= 2;
                if (gn == 1) top = 0;
                constexpr int U = 4;
                for (uint32_t x0 = tid; x0 < tot; x0 += U * kBlock) {
                    int lo[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) lo[u] = 0;
                    // the last run whose prefix is at most x holds entry x
                    for (int step = top; step > 0; step >>= 1) {
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const int t = lo[u] + step;
                            if (t < gn && s_pre[t] <= x0 + u * kBlock) lo[u] = t;
                        }
                    }
                    uint64_t y[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const uint32_t x = x0 + u * kBlock;
                        y[u] = x < tot ? reg[(g0 + lo[u]) * kHubRun + s_beg[lo[u]] + (x - s_pre[lo[u]])] : 0;
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (x0 + u * kBlock < tot) f(y[u]);
                }
                __syncthreads();  // the group's prefix is rewritten by the next group
            }
        };
        // LDS table of at least 2 E slots, at most kts: a partition of fewer than kts entries
        // never fills it; a larger one may (more distinct labels than slots), and then takes a
        // global table of its own
        const int kts = a.hub_ts;
        uint32_t* const s_key = s_hub_lds;
        uint32_t* const s_val = s_hub_lds + kts;
        bool in_lds = E > 0;
        if (in_lds) {
            int lb = 1;
            while ((1ll << lb) < 2 * E && (1 << lb) < kts) ++lb;
            const int ls = 1 << lb;
            for (int q = tid; q < ls; q += kBlock) {
                s_key[q] = EMPTY;
                s_val[q] = 0;
            }
            if (tid == 0) s_full = 0;
            __syncthreads();
            if (E < kts) {
                each_entry([&](uint64_t x) { lds_insert(s_key, s_val, lb, (uint32_t)(x >> 32), (uint32_t)x); });
            } else {
                bool full = false;
                each_entry([&](uint64_t x) {
                    if (!full && !lds_try_insert(s_key, s_val, lb, (uint32_t)(x >> 32), (uint32_t)x)) full = true;
                });
                if (full) s_full = 1;
            }
            __syncthreads();
            in_lds = s_full == 0;
            if (in_lds)
                rate_slots<4>(a, nk, own, cv, tid, ls, kBlock,
                              [&](int64_t q, uint32_t& K, uint32_t& V) {
                                  K = s_key[q];
                                  V = s_val[q];
                              },
                              fav, adm, rown);
        }
        if (E > 0 && !in_lds) {
            // overflow table of 2^b >= 2 E slots at slot d + 4 * before (2^b < 4 E and the
            // partitions before it hold `before` entries, so the tables stay inside the 4 d slots)
            int gb = 1;
            while ((1ll << gb) < 2 * E) ++gb;
            const int64_t gs = 1ll << gb;
            const uint64_t mask = (uint64_t)gs - 1;
            unsigned long long* tab = reinterpret_cast<unsigned long long*>(reg + d + 4 * before);
            for (int64_t q = tid; q < gs; q += kBlock) tab[q] = kEmptySlot;
            __syncthreads();
            each_entry([&](uint64_t x) {
                const uint32_t K = (uint32_t)(x >> 32), w = (uint32_t)x;
                uint64_t h = slot_of(K, gb) & mask;
                while (true) {
                    const unsigned long long old = atomicCAS(&tab[h], kEmptySlot, (unsigned long long)x);
                    if (old == kEmptySlot) break;
                    if ((uint32_t)(old >> 32) == K) {
                        atomicAdd(&tab[h], (unsigned long long)w);
                        break;
                    }
                    h = (h + 1) & mask;
                }
            });
            __syncthreads();
            rate_slots<4>(a, nk, own, cv, tid, gs, kBlock,
                          [&](int64_t q, uint32_t& K, uint32_t& V) {
                              const uint64_t x = tab[q];
                              if (x != kEmptySlot) {
                                  K = (uint32_t)(x >> 32);
                                  V = (uint32_t)x;
                              }
                          },
                          fav, adm, rown);
        }
        fav = group_best<64>(fav);
        adm = group_best<64>(adm);
        rown = group_sum_u32<64>(rown);
        if (lane == 0) {
            s_red[0][wv] = fav;
            s_red[1][wv] = adm;
            s_rown[wv] = rown;
        }
        __syncthreads();
        if (tid == 0) {
            for (int q = 1; q < kBlock / 64; ++q) {
                if (better(s_red[0][q], fav)) fav = s_red[0][q];
                if (better(s_red[1][q], adm)) adm = s_red[1][q];
                rown += s_rown[q];
            }
            uint32_t* out = a.hub_part + (int64_t)pc * kHubPart;
            out[0] = fav.r;
            out[1] = fav.h;
            out[2] = fav.k;
            out[3] = adm.r;
            out[4] = adm.h;
            out[5] = adm.k;
            out[6] = rown;
        }
        __syncthreads();  // the LDS tables and sums are reused by the next partition
    }
}

__global__ __launch_bounds__(kBlock) void k_hub_final(RateArgs a)
{
    if (aborted(a)) return;
    const int32_t off = a.segtab[a.seg], count = a.segtab[kSegs + a.seg];
    const int lane = threadIdx.x & 63;
    constexpr int kWaves = kBlock / 64;
    int64_t edges = 0, nodes = 0, moves = 0;
    for (int64_t i = (int64_t)xcd_block() * kWaves + (threadIdx.x >> 6); i < count;
         i += (int64_t)gridDim.x * kWaves) {
        const int32_t c0 = a.hub_pplan[i], c1 = a.hub_pplan[i + 1];
        if (c1 == c0) continue;  // not rated in this round (uniform across the wavefront)
        const int32_t v = a.list[off + i];
        {
            // the partition totals start from zero at the hub's next use
            const int64_t d = a.xadj[v + 1] - a.xadj[v];
            const int32_t P = hub_parts(d);
            uint32_t* ptot = reinterpret_cast<uint32_t*>(a.hub_tab + a.hub_off[v] + 5 * d) + hub_runs(d) * (P + 1);
            for (int q = lane; q < P; q += 64) ptot[q] = 0;
        }
        Key3 fav{0, 0, 0}, adm{0, 0, 0};
        uint32_t rown = 0;
        for (int32_t ch = c0 + lane; ch < c1; ch += 64) {
            const uint32_t* p = a.hub_part + (int64_t)ch * kHubPart;
            const Key3 f{p[0], p[1], p[2]}, m{p[3], p[4], p[5]};
            if (better(f, fav)) fav = f;
            if (better(m, adm)) adm = m;
            rown += p[6];
        }
        fav = group_best<64>(fav);
        adm = group_best<64>(adm);
        rown = group_sum_u32<64>(rown);
        if (lane == 0) {
            moves += write_result(a, v, (uint32_t)a.label[v], fav, adm, rown, a.vwgt ? a.vwgt[v] : 1);
            edges += a.xadj[v + 1] - a.xadj[v];
            nodes += 1;
        }
    }
    flush_stats(a, nodes, edges, moves);
}

// ---------------------------------------------------------------- admission
// The class-s nodes of the current lists: segments (t, s) for all tiers t.
struct ClassSegs {
    int32_t off[kTiers];
    int32_t cnt[kTiers];
    int32_t total;
};

__device__ inline ClassSegs class_segs(const int32_t* segtab, int s)
{
    ClassSegs c;
    c.total = 0;
#pragma unroll
    for (int t = 0; t < kTiers; ++t) {
        c.off[t] = segtab[t * kSub + s];
        c.cnt[t] = segtab[kSegs + t * kSub + s];
        c.total += c.cnt[t];
    }
    return c;
}

__device__ inline int32_t class_pos(const ClassSegs& c, int64_t i)
{
#pragma unroll
    for (int t = 0; t < kTiers; ++t) {
        if (i < c.cnt[t]) return c.off[t] + (int32_t)i;
        i -= c.cnt[t];
    }
    return -1;
}

// Rating tier of position i of the class (see class_pos).
__device__ inline int class_tier(const ClassSegs& c, int64_t i)
{
#pragma unroll
    for (int t = 0; t < kTiers; ++t) {
        if (i < c.cnt[t]) return t;
        i -= c.cnt[t];
    }
    return kTiers;
}

// Wave-aggregated reservation of one slot per requesting lane of a device cursor.
__device__ inline int64_t reserve_slot(int64_t* cursor, bool want)
{
    const uint64_t b = ballot64(want);
    if (!b) return -1;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)b) - 1;
    int64_t base = 0;
    if (lane == leader) base = (int64_t)atomicAdd((unsigned long long*)cursor, (unsigned long long)__popcll(b));
    base = __shfl(base, leader, 64);
    return want ? base + __popcll(b & ((1ull << lane) - 1ull)) : -1;
}

// Cap of target K for a proposal of node v (v and K belong to one job).
struct CapArgs {
    const int64_t* vec;   // [nlab] or NULL
    int64_t scalar;
    const int32_t* gid;   // batches: per-job scalar caps
    const int64_t* gcap;
};

__device__ inline int64_t cap_for(const CapArgs& c, uint32_t K, uint32_t v)
{
    if (c.vec) return c.vec[K];
    if (c.gcap) return c.gcap[c.gid[v]];
    return c.scalar;
}

// acc[v]: 0 none, 1 admitted, 2 contended (decided by a contended path)
__global__ __launch_bounds__(kBlock) void k_admit_fast(int64_t* ctl, const int32_t* __restrict__ list,
                                                       const int32_t* __restrict__ segtab, int s,
                                                       const int32_t* __restrict__ prop,
                                                       const uint32_t* __restrict__ demand,
                                                       const int64_t* __restrict__ wt, CapArgs caps,
                                                       uint8_t* __restrict__ acc, uint32_t* __restrict__ ckeys,
                                                       uint32_t* __restrict__ cvals, int64_t* __restrict__ wsnap,
                                                       int cont_idx)
{
    if (ctl[CTL_ABORT]) return;
    const ClassSegs cs = class_segs(segtab, s);
    for (int64_t i0 = (int64_t)xcd_block() * blockDim.x; i0 < cs.total; i0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = i0 + threadIdx.x;
        bool cont = false;
        int32_t v = -1, K = -1;
        if (i < cs.total) {
            v = list[class_pos(cs, i)];
            K = prop[v];
            if (K >= 0) {
                const int64_t cap = cap_for(caps, (uint32_t)K, (uint32_t)v);
                const int64_t w = wt[K];
                if (w + (int64_t)demand[K] <= cap) {
                    acc[v] = 1;
                } else {
                    acc[v] = 2;
                    wsnap[K] = w;  // every proposal into K writes the same value
                    cont = true;
                }
            }
        }
        const int64_t slot = reserve_slot(&ctl[cont_idx], cont);
        if (cont) {
            ckeys[slot] = (uint32_t)K;
            cvals[slot] = (uint32_t)v;
        }
    }
}

// exact path (host synchronised): contended proposals in ascending id over all n
__global__ void k_contended_flags(const uint8_t* __restrict__ acc, int32_t n, int32_t* __restrict__ flag)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) flag[v] = acc[v] == 2;
}

__global__ void k_contended_compact(const uint8_t* __restrict__ acc, const int32_t* __restrict__ pos, int32_t n,
                                    const int32_t* __restrict__ prop, uint32_t* __restrict__ keys,
                                    uint32_t* __restrict__ vals)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && acc[v] == 2) {
        keys[pos[v]] = (uint32_t)prop[v];
        vals[pos[v]] = (uint32_t)v;
    }
}

__global__ void k_gather_cw(const uint32_t* __restrict__ vals, int64_t np, const int32_t* __restrict__ vwgt,
                            int64_t* __restrict__ out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) out[i] = vwgt ? vwgt[vals[i]] : 1;
}

__global__ void k_heads(const uint32_t* __restrict__ keys, const int64_t* __restrict__ pre, const uint32_t* __restrict__ vals,
                        const int32_t* __restrict__ vwgt, int64_t np, int64_t* __restrict__ base)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    if (i == 0 || keys[i] != keys[i - 1]) {
        int64_t c = vwgt ? vwgt[vals[i]] : 1;
        base[keys[i]] = pre[i] - c;
    }
}

__global__ void k_decide(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                         const int64_t* __restrict__ pre, const int64_t* __restrict__ base, int64_t np,
                         const int64_t* __restrict__ wt, CapArgs caps, uint8_t* __restrict__ acc)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    uint32_t K = keys[i];
    int64_t cap = cap_for(caps, K, vals[i]);
    acc[vals[i]] = wt[K] + (pre[i] - base[K]) <= cap ? 1 : 0;
}

// Apply the sub-round's moves.  Contended proposals (acc = 2) are decided
// here: v is admitted iff the weight of its target at the sub-round start plus
// the weights of all proposals into the target with id <= v fits the cap (the
// contended list is staged through LDS in chunks by the blocks that hold
// contended nodes).  A list longer than kSmallCap aborts the sub-round before
// any move is applied.  Moved nodes get mflag[v] = stamp (the round number + 1
// inside lp_run, so flags never need clearing); per-block move counts go to the
// spread slots ctl[ms + (block & 63)].  Block 0 clears the next sub-round's
// contended-list length.
__global__ __launch_bounds__(kBlock) void k_apply(int64_t* ctl, const int32_t* __restrict__ list,
                                                  const int32_t* __restrict__ segtab, int s,
                                                  int32_t* __restrict__ prop, uint8_t* __restrict__ acc,
                                                  uint32_t* __restrict__ demand, int32_t* __restrict__ label,
                                                  int64_t* __restrict__ wt, const int32_t* __restrict__ vwgt,
                                                  uint8_t* __restrict__ mflag, uint8_t stamp, int ms,
                                                  const uint32_t* __restrict__ ckeys,
                                                  const uint32_t* __restrict__ cvals,
                                                  const int64_t* __restrict__ wsnap, CapArgs caps, int cont_idx,
                                                  int64_t small_cap, const int32_t* __restrict__ xadj,
                                                  const int32_t* __restrict__ adjncy, uint8_t* __restrict__ act_next,
                                                  uint8_t stamp_next)
{
    __shared__ int32_t bm;
    __shared__ uint64_t s_kv[kCandChunk];  // (target << 32) | id
    __shared__ int32_t s_w[kCandChunk];
    if (ctl[CTL_ABORT]) return;
    const int64_t C = ctl[cont_idx];
    if (C > small_cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ctl[CTL_ABORT] = 1;
            ctl[CTL_ABORT_SUB] = s;
            ctl[CTL_ABORT_STAMP] = stamp;
        }
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl[CTL_CONT + ((cont_idx - CTL_CONT) ^ 1)] = 0;
    if (threadIdx.x == 0) bm = 0;
    __syncthreads();
    const ClassSegs cs = class_segs(segtab, s);
    int32_t mine = 0;
    for (int64_t i0 = (int64_t)xcd_block() * blockDim.x; i0 < cs.total; i0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = i0 + threadIdx.x;
        int32_t v = -1, K = -1, cw = 1, old = 0, e0 = 0, e1 = 0;
        uint8_t a = 0;
        const bool mark = act_next && i < cs.total && class_tier(cs, i) <= 1;
        if (i < cs.total) {
            v = list[class_pos(cs, i)];
            // everything a move needs, loaded together (acc[v] is 0 without a proposal)
            K = prop[v];
            a = acc[v];
            if (vwgt) cw = vwgt[v];
            old = label[v];
            if (mark) {
                e0 = xadj[v];
                e1 = xadj[v + 1];
            }
            asm volatile("" ::"v"(K), "v"((int32_t)a), "v"(cw), "v"(old), "v"(e0), "v"(e1));
        }
        const bool contended = K >= 0 && a == 2;
        if (__syncthreads_or(contended)) {
            const int lane = threadIdx.x & 63;
            int64_t pre = 0;
            for (int64_t c0 = 0; c0 < C; c0 += kCandChunk) {
                const int len = (int)(C - c0 < kCandChunk ? C - c0 : kCandChunk);
                for (int j = threadIdx.x; j < len; j += blockDim.x) {
                    const uint32_t u = cvals[c0 + j];
                    s_kv[j] = ((uint64_t)ckeys[c0 + j] << 32) | u;
                    if (vwgt) s_w[j] = vwgt[u];
                }
                __syncthreads();
                // entries of target K with id <= v: keys in [K << 32, (K << 32) | v].  A
                // wavefront with few contended nodes scans the chunk once per node with all its
                // lanes; with many, each contended lane scans the whole chunk
                const uint64_t lo = (uint64_t)(uint32_t)K << 32, hi = lo | (uint32_t)v;
                const uint64_t cmask = __ballot(contended);
                if (__popcll(cmask) <= kWaveScanMax) {
                    for (uint64_t m = cmask; m != 0; m &= m - 1) {
                        const int t = __ffsll((long long)m) - 1;
                        const uint64_t lt = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(lo >> 32), t) << 32);
                        const uint64_t ht = lt | (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)hi, t);
                        int64_t part = 0;
                        for (int j = lane; j < len; j += 64)
                            part += (s_kv[j] >= lt && s_kv[j] <= ht) ? (vwgt ? s_w[j] : 1) : 0;
                        for (int dd = 32; dd > 0; dd >>= 1) part += __shfl_xor(part, dd, 64);
                        if (lane == t) pre += part;
                    }
                } else if (contended) {
                    if (vwgt) {
#pragma unroll 8
                        for (int j = 0; j < len; ++j) pre += (s_kv[j] >= lo && s_kv[j] <= hi) ? s_w[j] : 0;
                    } else {
#pragma unroll 8
                        for (int j = 0; j < len; ++j) pre += (s_kv[j] >= lo && s_kv[j] <= hi) ? 1 : 0;
                    }
                }
                __syncthreads();
            }
            if (contended) a = wsnap[K] + pre <= cap_for(caps, (uint32_t)K, (uint32_t)v) ? 1 : 0;
        }
        if (K < 0) continue;
        if (a == 1) {
            const int64_t c = cw;
            label[v] = K;
            // 32-bit adds on the low words: a label's weight stays within [0, c(V)]
            // at every point of the sub-round (its leavers are among its members),
            // and c(V) < 2^31 is checked at the boundary, so the high word is 0
            atomicAdd(reinterpret_cast<uint32_t*>(&wt[K]), (uint32_t)c);
            atomicAdd(reinterpret_cast<uint32_t*>(&wt[old]), (uint32_t)(-c));
            mflag[v] = stamp;
            ++mine;
            // next round's active set: the neighbours of a moved node of degree
            // <= T1_DEG are marked here (larger ones by k_push_active)
            if (mark) {
                for (int32_t eb = e0; eb < e1; eb += 8) {
                    int32_t u[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) u[q] = adjncy[eb + q < e1 ? eb + q : e1 - 1];
#pragma unroll
                    for (int q = 0; q < 8; ++q) act_next[u[q]] = stamp_next;
                }
            }
        }
        prop[v] = -1;
        acc[v] = 0;
        demand[K] = 0;
    }
    mine = (int32_t)group_sum_u32<64>((uint32_t)mine);
    if ((threadIdx.x & 63) == 0 && mine) atomicAdd(&bm, mine);
    __syncthreads();
    if (threadIdx.x == 0 && bm)
        atomicAdd((unsigned long long*)&ctl[ms + (blockIdx.x & (kSpreadSlots - 1)) * kSpreadStride],
                  (unsigned long long)bm);
}

struct SegBounds {
    int32_t off[kSegs + 1];
};

// Mark the neighbours of the nodes moved in this round (mflag[v] == stamp)
// active for the next one (active[u] = mark; the stamps never need clearing).
// Segment seg0 + blockIdx.y of the lists; the segment's degree tier picks the
// width that walks a node's neighbours: one lane (tiers 0, 1), one wavefront
// (tiers 2, 3) or the whole workgroup (hubs).  k_apply marks the neighbours of
// moved nodes of tiers 0 and 1 itself, so this runs over tiers 2-4 only.
// Nothing happens after an abort (the host redoes this step once the round is
// finished).
__global__ __launch_bounds__(kBlock) void k_push_active(const int64_t* __restrict__ ctl,
                                                        const int32_t* __restrict__ list,
                                                        const int32_t* __restrict__ segtab,
                                                        const uint8_t* __restrict__ mflag, uint8_t stamp,
                                                        const int32_t* __restrict__ xadj,
                                                        const int32_t* __restrict__ adjncy,
                                                        uint8_t* __restrict__ active, uint8_t mark, int seg0)
{
    if (ctl[CTL_ABORT]) return;
    const int seg = seg0 + blockIdx.y;
    const int tier = seg / kSub;
    const int32_t off = segtab[seg], cnt = segtab[kSegs + seg];
    if (tier <= 1) {
        for (int64_t i = (int64_t)xcd_block() * blockDim.x + threadIdx.x; i < cnt;
             i += (int64_t)gridDim.x * blockDim.x) {
            const int32_t v = list[off + i];
            if (mflag[v] != stamp) continue;
            const int32_t e0 = xadj[v], e1 = xadj[v + 1];
            for (int32_t eb = e0; eb < e1; eb += 8) {  // 8 neighbour ids per batch of loads
                int32_t u[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) u[q] = adjncy[eb + q < e1 ? eb + q : e1 - 1];
#pragma unroll
                for (int q = 0; q < 8; ++q) active[u[q]] = mark;
            }
        }
        return;
    }
    // W lanes per node: a wavefront (tiers 2, 3) or the workgroup (hubs); the
    // loop bounds are uniform across the W lanes of a node
    const int W = tier == 4 ? kBlock : 64;
    const int per_block = kBlock / W;
    const int grp = threadIdx.x / W, gl = threadIdx.x % W;
    for (int64_t i = (int64_t)xcd_block() * per_block + grp; i < cnt; i += (int64_t)gridDim.x * per_block) {
        const int32_t v = list[off + i];
        if (mflag[v] != stamp) continue;
        const int32_t e1 = xadj[v + 1];
        // eight neighbour ids per lane in flight (indices clamped into the row: a repeated last
        // neighbour is marked twice)
        for (int32_t e0 = xadj[v] + gl; e0 < e1; e0 += 8 * W) {
            int32_t u[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) u[q] = adjncy[e0 + q * W < e1 ? e0 + q * W : e1 - 1];
#pragma unroll
            for (int q = 0; q < 8; ++q) active[u[q]] = mark;
        }
    }
}

// Lists without the nodes of skipped jobs: the nodes of `order` segment
// blockIdx.y whose job is not skipped, appended to the same segment region of
// `alist` (each block reserves its slots with one atomic; the order inside a
// segment is free); counts go to segtab[kSegs + seg] (zero before), the
// segment's start to segtab[seg].
__global__ __launch_bounds__(kBlock) void k_order_skip_jobs(const int32_t* __restrict__ order, SegBounds b,
                                                            const int32_t* __restrict__ gid,
                                                            const uint8_t* __restrict__ skip,
                                                            int32_t* __restrict__ alist, int32_t* __restrict__ segtab)
{
    __shared__ int32_t s_cnt, s_base;
    const int seg = blockIdx.y;
    const int32_t lo = b.off[seg], hi = b.off[seg + 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) segtab[seg] = lo;
    for (int64_t i0 = lo + (int64_t)xcd_block() * kBlock; i0 < hi; i0 += (int64_t)gridDim.x * kBlock) {
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        const int64_t i = i0 + threadIdx.x;
        int32_t v = -1, slot = -1;
        if (i < hi) {
            v = order[i];
            if (!skip[gid[v]]) slot = atomicAdd(&s_cnt, 1);
        }
        __syncthreads();
        if (threadIdx.x == 0 && s_cnt) s_base = atomicAdd(&segtab[kSegs + seg], s_cnt);
        __syncthreads();
        if (slot >= 0) alist[lo + s_base + slot] = v;
        __syncthreads();
    }
}

__global__ void k_ctl_set(int64_t* ctl, int idx, int64_t v)
{
    if (threadIdx.x == 0) ctl[idx] = v;
}

// ---------------------------------------------------------------- small levels
// Every round and sub-round of one LP call of a small job in a single
// workgroup (one workgroup per job).  The steps of a sub-round (rate, admit
// at the sub-round start weights, decide contended targets, apply) are
// separated by workgroup barriers instead of kernel launches, so the whole
// call costs one launch and one read-back.  The job's mutable state lives in
// LDS for the whole call (labels, proposals, admission flags, active stamps as
// local ids; label weights and demands as int32, which hold any weight since
// c(V) < 2^31); only the graph, the caps and the favoured clusters are in
// global memory, and labels and weights are written back at the end.  The
// next round's active set is marked while moves are applied, in the stamp
// array of the next round's parity (the marks never hide a node's stamp for
// the current round).  A job runs here only if every node sits in rating
// tiers 0 and 1 (degree <= T1_DEG): tier-0 nodes are rated one per lane,
// tier-1 nodes one per wavefront with a 2^7-slot LDS table.
constexpr int kSmallBlock = 1024;
// dynamic LDS of a job: 3 int32 per label (weight, demand, start weight of a
// contended target) + 3 int16 and 3 bytes per node (list, label, proposal;
// admission flag, two stamp arrays), within what the static tables leave
__host__ __device__ inline int64_t small_lds_bytes(int64_t nodes, int64_t labels)
{
    return (12 * labels + 9 * nodes + 15) & ~(int64_t)15;
}
constexpr int64_t kSmallLdsBudget = 128 * 1024;

struct SmallLP {
    RateArgs a;               // graph, caps, fav, counters, job tables; hpre / round set per round
    int32_t* label;           // [n] global labels (read at the start, written at the end)
    int64_t* wt;              // [nlab] global label weights (same)
    const int32_t* jstart;    // by workgroup: the job's first node, node count, first label, label count
    const int32_t* jcount;    // (all NULL for one job: then `one` holds the four values)
    const int32_t* jloff;
    const int32_t* jnlab;
    int32_t one[4];
    uint32_t hsub;            // one graph: H prefix over (seed; T_SUB, level) of the sub-round classes
    uint32_t hpre[kRounds];   // one graph: H prefix over (seed; tag, level, round) of every round
    int32_t cut0;             // largest degree rated one per lane (tier 0)
    uint32_t* cont;           // [n] contended (target << 16 | node), local ids, inside each job's node range
    int64_t* out;             // [kRounds] moves per round (summed over jobs), [kRounds] largest round count
};

// Tier-0 rating of local node li (global id v) against the LDS labels and
// weights; labels are local (global label - lo), which is also what the
// tie-break hash takes.
// nbr(e) gives entry e's neighbour as a local id, ewt(e) its weight.
template <int DEG, bool EW, bool CAPV, class NB, class EWT>
__device__ inline void rate_lane_local(const RateArgs& a, int32_t lo, uint32_t own, int32_t e0, int32_t d, int64_t cv,
                                       const NodeKey& nk, const int16_t* s_lab, const int32_t* s_wt, NB nbr, EWT ewt,
                                       Key3& fav, Key3& adm, uint32_t& rown)
{
    uint32_t lab[DEG], w[DEG];
#pragma unroll
    for (int j = 0; j < DEG; ++j) {
        lab[j] = EMPTY;
        w[j] = 1u;
    }
    if (d > 0) {
        int32_t u[DEG];
#pragma unroll
        for (int j = 0; j < DEG; ++j) u[j] = nbr(e0 + (j < d ? j : d - 1));
        if constexpr (EW) {
#pragma unroll
            for (int j = 0; j < DEG; ++j) w[j] = ewt(e0 + (j < d ? j : d - 1));
        }
#pragma unroll
        for (int j = 0; j < DEG; ++j) lab[j] = j < d ? (uint32_t)s_lab[u[j]] : EMPTY;
    }
    auto wt_of = [&](uint32_t l) -> int64_t { return l != EMPTY ? s_wt[l] : 0; };
    auto cap_of = [&](uint32_t l) -> int64_t { return CAPV ? a.cap_vec[lo + l] : nk.cap; };
    auto over_of = [](uint32_t) -> bool { return false; };
    if (a.fav)  // clustering keeps the favoured cluster too (uniform branch)
        choose_slots<DEG, DEG, EW, true>(lab, w, own, nk.hp, 0u, cv, wt_of, cap_of, over_of, fav, adm, rown);
    else
        choose_slots<DEG, DEG, EW, false>(lab, w, own, nk.hp, 0u, cv, wt_of, cap_of, over_of, fav, adm, rown);
}

// LCSR: the job's CSR is copied to LDS first (row starts relative to the job's
// first entry, node weights, edge weights, neighbours as local ids).
// Asynchronous move of local node li from label own to K inside the
// one-workgroup LP (weights and labels in LDS): strict (refinement) reserves
// K's weight with compare-and-swap, else fetch-and-add; the neighbours are
// marked for round r + 1.  Returns 1 if li moved.
template <class ROW, class NBR>
__device__ inline int32_t small_async_move(int32_t li, int32_t K, int32_t own, int32_t cv, int64_t cap, bool strict,
                                           int16_t* s_lab, int32_t* s_wt, uint8_t* act_next, uint8_t stamp_next,
                                           bool mark, ROW row0, NBR nbr)
{
    if (strict) {
        int32_t old = s_wt[K];
        // a failed exchange returns a weight another move wrote; every node moves at most once per class
        while ((int64_t)old + cv <= cap) {
            const int32_t seen = atomicCAS(&s_wt[K], old, old + cv);
            if (seen == old) break;
            old = seen;
        }
        if ((int64_t)old + cv > cap) return 0;
    } else {
        atomicAdd(&s_wt[K], cv);
    }
    atomicAdd(&s_wt[own], -cv);
    s_lab[li] = (int16_t)K;
    if (mark) {
        const int32_t e0 = row0(li), e1 = row0(li + 1);
        for (int32_t e = e0; e < e1; ++e) act_next[nbr(e)] = stamp_next;
    }
    return 1;
}

template <bool EW, bool CAPV, bool LCSR>
__global__ __launch_bounds__(kSmallBlock) void k_lp_small(SmallLP p)
{
    constexpr int HB = 7, HS = 1 << HB, NW = kSmallBlock / 64;
    __shared__ uint32_t s_keys[NW * HS];
    __shared__ uint32_t s_vals[NW * HS];
    __shared__ uint32_t s_kv[kCandChunk];  // (target << 16) | node, local ids
    __shared__ int32_t s_w[kCandChunk];
    __shared__ int32_t s_cont, s_moves;
    __shared__ int32_t s_cnt[3 * kSub], s_off[3 * kSub];
    extern __shared__ __align__(16) char s_dyn[];
    RateArgs a = p.a;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    uint32_t* keys = s_keys + wv * HS;
    uint32_t* vals = s_vals + wv * HS;
    const int32_t start = p.jstart ? p.jstart[blockIdx.x] : p.one[0];
    const int32_t nj = p.jstart ? p.jcount[blockIdx.x] : p.one[1];
    const int32_t lo = p.jstart ? p.jloff[blockIdx.x] : p.one[2];
    const int32_t nl = p.jstart ? p.jnlab[blockIdx.x] : p.one[3];
    int32_t* s_wt = reinterpret_cast<int32_t*>(s_dyn);
    int32_t* s_dem = s_wt + nl;
    int32_t* s_ws = s_dem + nl;
    int16_t* s_ord = reinterpret_cast<int16_t*>(s_ws + nl);
    int16_t* s_lab = s_ord + nj;
    int16_t* s_prop = s_lab + nj;
    uint8_t* s_acc = reinterpret_cast<uint8_t*>(s_prop + nj);
    uint8_t* s_act[2] = {s_acc + nj, s_acc + 2 * nj};
    int32_t *s_xa = nullptr, *s_vw = nullptr, *s_ew = nullptr;
    int16_t* s_adj = nullptr;
    if (LCSR) {
        const int32_t ebase = a.xadj[start], mj = a.xadj[start + nj] - ebase;
        char* q = reinterpret_cast<char*>(((uintptr_t)(s_act[1] + nj) + 15) & ~(uintptr_t)15);
        s_xa = reinterpret_cast<int32_t*>(q);
        s_vw = s_xa + (nj + 1);
        s_ew = s_vw + (a.vwgt ? nj : 0);
        s_adj = reinterpret_cast<int16_t*>(s_ew + (EW ? mj : 0));
        for (int32_t i = tid; i <= nj; i += kSmallBlock) s_xa[i] = a.xadj[start + i] - ebase;
        if (a.vwgt)
            for (int32_t i = tid; i < nj; i += kSmallBlock) s_vw[i] = a.vwgt[start + i];
        for (int32_t e = tid; e < mj; e += kSmallBlock) {
            s_adj[e] = (int16_t)(a.adjncy[ebase + e] - start);
            if (EW) s_ew[e] = a.adjwgt[ebase + e];
        }
    }
    // row start (entry index: local with LCSR, global without), neighbour (local id),
    // edge weight, node weight of local node li / entry e
    auto row0 = [&](int32_t li) -> int32_t { return LCSR ? s_xa[li] : a.xadj[start + li]; };
    auto nbr = [&](int32_t e) -> int32_t { return LCSR ? (int32_t)s_adj[e] : a.adjncy[e] - start; };
    auto ewt = [&](int32_t e) -> uint32_t { return !EW ? 1u : LCSR ? (uint32_t)s_ew[e] : (uint32_t)a.adjwgt[e]; };
    auto nwt = [&](int32_t li) -> int32_t { return !a.vwgt ? 1 : LCSR ? s_vw[li] : a.vwgt[start + li]; };
    for (int32_t i = tid; i < nj; i += kSmallBlock) {
        s_lab[i] = (int16_t)(p.label[start + i] - lo);
        s_prop[i] = -1;
        s_acc[i] = 0;
        s_act[0][i] = 0;
        s_act[1][i] = 0;
    }
    for (int32_t k = tid; k < nl; k += kSmallBlock) {
        s_wt[k] = (int32_t)p.wt[lo + k];
        s_dem[k] = 0;
    }
    uint32_t hs = p.hsub;
    if (a.gid) hs = hash_step(hash_step(a.ghash[a.gid[start]], TAG_SUB, 1), a.level, 2);
    // The job's class lists (local ids): for class s, tier-0 nodes of degree <=
    // T0_NARROW, the other tier-0 nodes, then tier-1 nodes (list 3 s + 0, 1, 2).
    // The order inside a list does not matter.
    auto list_of = [&](int32_t i) -> int {
        const int32_t d = row0(i + 1) - row0(i);
        const int t = d > p.cut0 ? 2 : d <= T0_NARROW ? 0 : 1;
        return 3 * (int)(hash_step(hs, (uint32_t)i, 3) % kSub) + t;
    };
    if (tid < 3 * kSub) s_cnt[tid] = 0;
    __syncthreads();
    for (int32_t i = tid; i < nj; i += kSmallBlock) atomicAdd(&s_cnt[list_of(i)], 1);
    __syncthreads();
    if (tid == 0) {
        int32_t o = 0;
        for (int q = 0; q < 3 * kSub; ++q) {
            s_off[q] = o;
            o += s_cnt[q];
            s_cnt[q] = 0;
        }
    }
    __syncthreads();
    for (int32_t i = tid; i < nj; i += kSmallBlock) {
        const int q = list_of(i);
        s_ord[s_off[q] + atomicAdd(&s_cnt[q], 1)] = (int16_t)i;
    }
    __syncthreads();
    int64_t edges = 0, nodes = 0;
    int32_t rounds = kRounds;
    for (int32_t r = 0; r < kRounds; ++r) {
        a.hpre = p.hpre[r];  // batches: node_key derives each job's prefix instead
        a.round = (uint32_t)r;
        const NodeKey nk = node_key(a, start);  // the same for every node of the job
        const uint8_t* act = s_act[r & 1];
        uint8_t* act_next = s_act[(r + 1) & 1];
        const uint8_t stamp = (uint8_t)(r + 1), stamp_next = (uint8_t)(r + 2);
        if (tid == 0) s_moves = 0;
        int32_t mine = 0;  // moves applied by this thread in round r
        for (int s = 0; s < kSub; ++s) {
            const int32_t o0 = s_off[3 * s], c0 = s_cnt[3 * s] + s_cnt[3 * s + 1], o1 = s_off[3 * s + 2],
                          c1 = s_cnt[3 * s + 2];
            const int32_t cn = s_cnt[3 * s], ow = o0 + cn, cw = s_cnt[3 * s + 1];
            // rate, tier 0 up to degree T0_NARROW: one lane per node, neighbours in registers
            for (int32_t i = tid; i < cn; i += kSmallBlock) {
                const int32_t li = s_ord[o0 + i];
                if (r > 0 && act[li] != stamp) continue;
                const int32_t v = start + li;
                const uint32_t own = (uint32_t)s_lab[li];
                const int32_t e0 = row0(li);
                const int32_t d = row0(li + 1) - e0;
                const int64_t cv = nwt(li);
                Key3 fav{0, 0, 0}, adm{0, 0, 0};
                uint32_t rown = 0;
                rate_lane_local<T0_NARROW, EW, CAPV>(a, lo, own, e0, d, cv, nk, s_lab, s_wt, nbr, ewt, fav, adm,
                                                     rown);
                if (a.fav) a.fav[v] = fav.r ? fav.k + (uint32_t)lo : kNone;
                if (adm.r > rown) {
                    if (a.amode) {
                        mine += small_async_move((int32_t)li, (int32_t)adm.k, (int32_t)own, (int32_t)cv,
                                                 CAPV ? a.cap_vec[lo + adm.k] : nk.cap, a.amode == 2, s_lab, s_wt,
                                                 act_next, stamp_next, r + 1 < kRounds, row0, nbr);
                    } else {
                        s_prop[li] = (int16_t)adm.k;
                        atomicAdd(&s_dem[adm.k], (int32_t)cv);
                    }
                }
                edges += d;
                nodes += 1;
            }
            // rate, the rest of tier 0 (degree <= cut0 <= 16): 16 lanes per node, one
            // neighbour per lane into a 32-slot LDS table of the group (the per-wave
            // tables below, split in four); the trip count is uniform in the block so
            // that the group reductions see whole wavefronts
            {
                constexpr int GW = 16, GS = 32, NG = kSmallBlock / GW;
                const int g = tid / GW, gl = tid % GW;
                uint32_t* gk = s_keys + g * GS;
                uint32_t* gv = s_vals + g * GS;
                for (int32_t i0 = 0; i0 < cw; i0 += NG) {
                    const int32_t i = i0 + g;
                    int32_t li = i < cw ? s_ord[ow + i] : -1;
                    if (li >= 0 && r > 0 && act[li] != stamp) li = -1;
                    gk[gl] = EMPTY;
                    gk[gl + GW] = EMPTY;
                    gv[gl] = 0;
                    gv[gl + GW] = 0;
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    int32_t v = 0, d = 0;
                    int64_t cv = 0;
                    uint32_t own = EMPTY;
                    if (li >= 0) {
                        v = start + li;
                        const int32_t e0 = row0(li);
                        d = row0(li + 1) - e0;
                        cv = nwt(li);
                        own = (uint32_t)s_lab[li];
                        if (gl < d) lds_insert(gk, gv, 5, (uint32_t)s_lab[nbr(e0 + gl)], ewt(e0 + gl));
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    Key3 fav{0, 0, 0}, adm{0, 0, 0};
                    uint32_t rown = 0;
                    if (li >= 0) {
                        for (int j = gl; j < GS; j += GW) {
                            const uint32_t key = gk[j], val = gv[j];
                            if (key == EMPTY) continue;
                            if (key == own) {
                                rown = val;
                                continue;
                            }
                            const Key3 c{val, hash_step(nk.hp, key, 4), key};
                            if (a.fav && better(c, fav)) fav = c;
                            if (better(c, adm)) {
                                const int64_t ck = CAPV ? a.cap_vec[lo + key] : nk.cap;
                                if (s_wt[key] + cv <= ck) adm = c;
                            }
                        }
                    }
                    fav = group_best<GW>(fav);
                    adm = group_best<GW>(adm);
                    rown = group_sum_u32<GW>(rown);
                    if (li >= 0 && gl == 0) {
                        if (a.fav) a.fav[v] = fav.r ? fav.k + (uint32_t)lo : kNone;
                        if (adm.r > rown) {
                            if (a.amode) {
                                mine += small_async_move(li, (int32_t)adm.k, (int32_t)own, (int32_t)cv,
                                                         CAPV ? a.cap_vec[lo + adm.k] : nk.cap, a.amode == 2, s_lab,
                                                         s_wt, act_next, stamp_next, r + 1 < kRounds, row0, nbr);
                            } else {
                                s_prop[li] = (int16_t)adm.k;
                                atomicAdd(&s_dem[adm.k], (int32_t)cv);
                            }
                        }
                        edges += d;
                        nodes += 1;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();  // the table is reused only after every read
                }
            }
            // rate, tier 1: one wavefront per node (the loop is uniform in the wave)
            for (int32_t i = wv; i < c1; i += NW) {
                const int32_t li = s_ord[o1 + i];
                if (r > 0 && act[li] != stamp) continue;
                const int32_t v = start + li;
                for (int j = lane; j < HS; j += 64) {
                    keys[j] = EMPTY;
                    vals[j] = 0;
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                __builtin_amdgcn_wave_barrier();
                const int32_t e0 = row0(li), e1 = row0(li + 1);
                for (int32_t e = e0 + lane; e < e1; e += 64) lds_insert(keys, vals, HB, (uint32_t)s_lab[nbr(e)], ewt(e));
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                __builtin_amdgcn_wave_barrier();
                const uint32_t own = (uint32_t)s_lab[li];
                const int64_t cv = nwt(li);
                Key3 fav{0, 0, 0}, adm{0, 0, 0};
                uint32_t rown = 0;
                for (int j = lane; j < HS; j += 64) {
                    const uint32_t key = keys[j], val = vals[j];
                    if (key == EMPTY) continue;
                    if (key == own) {
                        rown = val;
                        continue;
                    }
                    const Key3 c{val, hash_step(nk.hp, key, 4), key};
                    if (better(c, fav)) fav = c;
                    if (better(c, adm)) {
                        const int64_t ck = CAPV ? a.cap_vec[lo + key] : nk.cap;
                        if (s_wt[key] + cv <= ck) adm = c;
                    }
                }
                fav = group_best<64>(fav);
                adm = group_best<64>(adm);
                rown = group_sum_u32<64>(rown);
                if (lane == 0) {
                    if (a.fav) a.fav[v] = fav.r ? fav.k + (uint32_t)lo : kNone;
                    if (adm.r > rown) {
                        if (a.amode) {
                            mine += small_async_move(li, (int32_t)adm.k, (int32_t)own, (int32_t)cv,
                                                     CAPV ? a.cap_vec[lo + adm.k] : nk.cap, a.amode == 2, s_lab,
                                                     s_wt, act_next, stamp_next, r + 1 < kRounds, row0, nbr);
                        } else {
                            s_prop[li] = (int16_t)adm.k;
                            atomicAdd(&s_dem[adm.k], (int32_t)cv);
                        }
                    }
                    edges += e1 - e0;
                    nodes += 1;
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                __builtin_amdgcn_wave_barrier();  // the table is cleared for the next node only after every read
            }
            if (a.amode) {  // asynchronous: moves are already applied; the next class sees them
                __syncthreads();
                continue;
            }
            if (tid == 0) s_cont = 0;
            __syncthreads();
            // admission at the sub-round start weights (no weight changes until the apply step);
            // contended proposals are listed (target << 16 | node, local ids) with their weights
            const int32_t total = c0 + c1;
            for (int32_t i = tid; i < total; i += kSmallBlock) {
                const int32_t li = s_ord[i < c0 ? o0 + i : o1 + (i - c0)];
                const int32_t K = s_prop[li];
                if (K < 0) continue;
                const int64_t wK = s_wt[K];
                const int64_t cap = CAPV ? a.cap_vec[lo + K] : nk.cap;
                if (wK + (int64_t)s_dem[K] <= cap) {
                    s_acc[li] = 1;
                } else {
                    s_acc[li] = 2;
                    s_ws[K] = (int32_t)wK;  // every proposal into K writes the same value
                    const int32_t slot = atomicAdd(&s_cont, 1);
                    const uint32_t kv = ((uint32_t)K << 16) | (uint32_t)li;
                    const int32_t w = nwt(li);
                    if (slot < kCandChunk) {
                        s_kv[slot] = kv;
                        s_w[slot] = w;
                    }
                    p.cont[start + slot] = kv;
                }
            }
            __syncthreads();
            const int32_t C = s_cont;
            // contended targets: the longest prefix in id order that fits.  Up to
            // kCandChunk entries, every entry finds its prefix in the LDS list;
            // longer lists are staged through LDS in chunks per node.
            if (C > 0 && C <= kCandChunk) {
                for (int32_t t = tid; t < C; t += kSmallBlock) {
                    const uint32_t kv = s_kv[t];
                    const uint32_t klo = kv & 0xFFFF0000u;
                    int64_t pre = 0;
#pragma unroll 8
                    for (int j = 0; j < C; ++j) pre += (s_kv[j] >= klo && s_kv[j] <= kv) ? s_w[j] : 0;
                    const int32_t K = (int32_t)(kv >> 16);
                    const int64_t cap = CAPV ? a.cap_vec[lo + K] : nk.cap;
                    s_acc[kv & 0xFFFFu] = (int64_t)s_ws[K] + pre <= cap ? 1 : 0;
                }
                __syncthreads();
            }
            // apply the admitted moves and mark the neighbours of moved nodes for round r + 1
            for (int32_t i0 = 0; i0 < total; i0 += kSmallBlock) {
                const int32_t i = i0 + tid;
                int32_t li = -1, K = -1;
                uint8_t ac = 0;
                if (i < total) {
                    li = s_ord[i < c0 ? o0 + i : o1 + (i - c0)];
                    K = s_prop[li];
                    if (K >= 0) ac = s_acc[li];
                }
                const bool contended = ac == 2;  // only when C > kCandChunk
                if (C > kCandChunk && __syncthreads_or(contended)) {
                    int64_t pre = 0;
                    for (int32_t q0 = 0; q0 < C; q0 += kCandChunk) {
                        const int len = C - q0 < kCandChunk ? C - q0 : kCandChunk;
                        for (int j = tid; j < len; j += kSmallBlock) {
                            const uint32_t kv = p.cont[start + q0 + j];
                            s_kv[j] = kv;
                            s_w[j] = nwt((int32_t)(kv & 0xFFFFu));
                        }
                        __syncthreads();
                        if (contended) {
                            // entries of target K with local id <= li
                            const uint32_t klo = (uint32_t)K << 16, khi = klo | (uint32_t)li;
#pragma unroll 8
                            for (int j = 0; j < len; ++j) pre += (s_kv[j] >= klo && s_kv[j] <= khi) ? s_w[j] : 0;
                        }
                        __syncthreads();
                    }
                    if (contended) {
                        const int64_t cap = CAPV ? a.cap_vec[lo + K] : nk.cap;
                        ac = (int64_t)s_ws[K] + pre <= cap ? 1 : 0;
                    }
                }
                if (K < 0) continue;
                if (ac == 1) {
                    const int32_t c = nwt(li);
                    const int32_t old = s_lab[li];
                    s_lab[li] = (int16_t)K;
                    atomicAdd(&s_wt[K], c);
                    atomicAdd(&s_wt[old], -c);
                    if (r + 1 < kRounds) {
                        // neighbour ids in batches of 8 loads issued together
                        const int32_t e0 = row0(li), e1 = row0(li + 1);
                        for (int32_t eb = e0; eb < e1; eb += 8) {
                            int32_t u[8];
#pragma unroll
                            for (int q = 0; q < 8; ++q) u[q] = nbr(eb + q < e1 ? eb + q : e1 - 1);
#pragma unroll
                            for (int q = 0; q < 8; ++q) act_next[u[q]] = stamp_next;
                        }
                    }
                    ++mine;
                }
                s_prop[li] = -1;
                s_acc[li] = 0;
                s_dem[K] = 0;
            }
            __syncthreads();
        }
        mine = (int32_t)group_sum_u32<64>((uint32_t)mine);
        if (lane == 0 && mine) atomicAdd(&s_moves, mine);
        __syncthreads();
        const int32_t moved = s_moves;
        if (tid == 0 && moved) atomicAdd((unsigned long long*)&p.out[r], (unsigned long long)moved);
        __syncthreads();  // every thread has read s_moves before the next round clears it
        if (moved == 0) {
            rounds = r + 1;
            break;
        }
    }
    for (int32_t i = tid; i < nj; i += kSmallBlock) p.label[start + i] = lo + s_lab[i];
    for (int32_t k = tid; k < nl; k += kSmallBlock) p.wt[lo + k] = s_wt[k];
    if (tid == 0) atomicMax((unsigned long long*)&p.out[kRounds], (unsigned long long)rounds);
    flush_stats(a, nodes, edges);
}

}  // namespace

// ================================================================ host side

void hub_tables(Ctx& c, const DGraph& g, LPSchedule& sched);

void lp_build_schedule(Ctx& c, const DGraph& g, int32_t level, uint64_t seed, LPSchedule& sched, const JobTabs& jt,
                       const uint8_t* gpart, int32_t njobs)
{
    const int32_t n = g.n;
    sched.order = DBuf<int32_t>(c, (size_t)n);
    memset(sched.off, 0, sizeof(sched.off));
    memset(sched.cnt, 0, sizeof(sched.cnt));
    sched.hub_slots_total = 0;
    sched.hub_start = n;
    sched.segtab = DBuf<int32_t>(c, 2 * kSegs);
    if (n == 0) {
        c.zero(sched.segtab.p, sizeof(int32_t) * 2 * kSegs);
        return;
    }
    DBuf<uint32_t> key(c, n), key2(c, n);
    DBuf<int32_t> val(c, n), val2(c, n);
    const int32_t nj = jt.gid ? njobs : 0;
    DBuf<int32_t> cnt(c, (size_t)(kSegs + 1 + nj));  // segment sizes, then the jobs' largest degrees
    c.zero(cnt.p, (kSegs + 1 + nj) * sizeof(int32_t));
    const uint32_t hsub = hash_prefix(seed, {TAG_SUB, (uint32_t)level});
    {
        ProfScope ps(c, KMP_PROF_SCHEDULE);
        const TierCuts tc{{c.tune.cut[0], c.tune.cut[1], c.tune.cut[2], c.tune.cut[3]}};
        hipLaunchKernelGGL(k_sched_keys, dim3(grid_for(n, kBlock, 1024)), dim3(kBlock), 0, c.stream, g.xadj, n, hsub, jt, gpart,
                           (uint32_t)level, tc, key.p, reinterpret_cast<uint32_t*>(val.p), cnt.p,
                           nj ? cnt.p + kSegs + 1 : nullptr);
        KMP_LAUNCH_CHECK();
    }
    uint32_t* sorted = nullptr;
    radix_sort_pairs(c, key.p, reinterpret_cast<uint32_t*>(val.p), key2.p, reinterpret_cast<uint32_t*>(val2.p), n,
                     bits_for(2 * kSegs + 1), nullptr, &sorted);
    sched.order = reinterpret_cast<int32_t*>(sorted) == val.p ? std::move(val) : std::move(val2);
    std::vector<int32_t> hv((size_t)(kSegs + 1 + nj));
    c.read(hv.data(), cnt.p, sizeof(int32_t) * hv.size());
    const int32_t* h = hv.data();
    sched.job_maxdeg.assign(hv.begin() + kSegs + 1, hv.end());
    int32_t pos = 0;
    for (int j = 0; j < kSegs; ++j) {
        sched.off[j] = pos;
        sched.cnt[j] = h[j];
        pos += h[j];
    }
    sched.off[kSegs] = pos;  // nodes of jobs that do not take part follow
    int32_t tab[2 * kSegs];
    for (int j = 0; j < kSegs; ++j) {
        tab[j] = sched.off[j];
        tab[kSegs + j] = sched.cnt[j];
    }
    c.write(sched.segtab.p, tab, sizeof(tab));
    hub_tables(c, g, sched);
}

// Global hash tables of the hubs (the last tier, all classes contiguous).
void hub_tables(Ctx& c, const DGraph& g, LPSchedule& sched)
{
    const int32_t n = g.n;
    sched.hub_start = sched.off[(kTiers - 1) * kSub];
    const int32_t nh = sched.off[kSegs] - sched.hub_start;
    if (nh > 0) {
        DBuf<int64_t> slots(c, (size_t)nh), incl(c, (size_t)nh);
        const int32_t* hubs = sched.order.p + sched.hub_start;
        hipLaunchKernelGGL(k_hub_slots, dim3(grid_for(nh)), dim3(kBlock), 0, c.stream, g.xadj, hubs, nh, slots.p);
        KMP_LAUNCH_CHECK();
        scan_incl_i64(c, slots.p, incl.p, nh);
        sched.hub_slots_total = c.read1(incl.p + nh - 1);
        sched.hub_slot_off = DBuf<int64_t>(c, (size_t)n);
        hipLaunchKernelGGL(k_hub_scatter, dim3(grid_for(nh)), dim3(kBlock), 0, c.stream, hubs, slots.p, incl.p, nh,
                           sched.hub_slot_off.p);
        KMP_LAUNCH_CHECK();
    }
}

void lp_build_async_schedule(Ctx& c, const DGraph& g, int32_t level, uint64_t seed, LPSchedule& sched,
                             const JobTabs& jt, const uint8_t* gpart)
{
    const int32_t n = g.n;
    sched.order = DBuf<int32_t>(c, (size_t)n);
    memset(sched.off, 0, sizeof(sched.off));
    memset(sched.cnt, 0, sizeof(sched.cnt));
    sched.hub_slots_total = 0;
    sched.hub_start = n;
    sched.segtab = DBuf<int32_t>(c, 2 * kSegs);
    if (n == 0) {
        c.zero(sched.segtab.p, sizeof(int32_t) * 2 * kSegs);
        return;
    }
    DBuf<uint32_t> key(c, n), key2(c, n);
    DBuf<int32_t> val(c, n), val2(c, n);
    DBuf<int32_t> cnt(c, kSegs + 1);
    c.zero(cnt.p, (kSegs + 1) * sizeof(int32_t));
    // tier t takes the buckets b with 2^(b+1) - 1 <= its degree cut-off
    BucketCuts bc;
    for (int t = 0; t < 4; ++t) {
        int b = -1;
        while ((int64_t(2) << (b + 1)) - 1 <= c.tune.cut[t]) ++b;
        bc.blim[t] = b;
    }
    const uint32_t hsub = hash_prefix(seed, {TAG_SUB, (uint32_t)level});
    {
        ProfScope ps(c, KMP_PROF_SCHEDULE);
        hipLaunchKernelGGL(k_async_keys, dim3(grid_for(n, kBlock, 1024)), dim3(kBlock), 0, c.stream, g.xadj, n, hsub,
                           jt, gpart, (uint32_t)level, bc, key.p, reinterpret_cast<uint32_t*>(val.p), cnt.p);
        KMP_LAUNCH_CHECK();
    }
    uint32_t* sorted = nullptr;
    radix_sort_pairs(c, key.p, reinterpret_cast<uint32_t*>(val.p), key2.p, reinterpret_cast<uint32_t*>(val2.p), n,
                     bits_for(32 * kSegs + 31), nullptr, &sorted);
    sched.order = reinterpret_cast<int32_t*>(sorted) == val.p ? std::move(val) : std::move(val2);
    int32_t h[kSegs + 1];
    c.read(h, cnt.p, sizeof(h));
    int32_t pos = 0;
    for (int j = 0; j < kSegs; ++j) {
        sched.off[j] = pos;
        sched.cnt[j] = h[j];
        pos += h[j];
    }
    sched.off[kSegs] = pos;
    int32_t tab[2 * kSegs];
    for (int j = 0; j < kSegs; ++j) {
        tab[j] = sched.off[j];
        tab[kSegs + j] = sched.cnt[j];
    }
    c.write(sched.segtab.p, tab, sizeof(tab));
    hub_tables(c, g, sched);
}

namespace {

// Hub tables of a level (every slot free), the chunk plan of one launch and
// the per-chunk partial results; the tables return to free after every use.
struct HubBufs {
    DBuf<uint64_t> tab;
    DBuf<int32_t> plan, pplan;
    DBuf<uint32_t> part;
};

void hub_buffers(Ctx& c, const DGraph& g, const LPSchedule& sched, HubBufs& h)
{
    if (sched.hub_slots_total <= 0) return;
    const int32_t nh = sched.off[kSegs] - sched.hub_start;
    h.tab = DBuf<uint64_t>(c, (size_t)sched.hub_slots_total);
    h.plan = DBuf<int32_t>(c, (size_t)nh + 1);
    h.pplan = DBuf<int32_t>(c, (size_t)nh + 1);
    // label partitions of all hubs: a hub of degree d has at most d / kHubPartAvg + 1 and a
    // region of at least 5 d slots
    h.part = DBuf<uint32_t>(c, (size_t)(sched.hub_slots_total / (5 * kHubPartAvg) + nh) * kHubPart);
    hipLaunchKernelGGL(k_hub_zero, dim3(grid_for(nh)), dim3(kBlock), 0, c.stream, g.xadj,
                       sched.order.p + sched.hub_start, nh, sched.hub_slot_off.p, h.tab.p);
    KMP_LAUNCH_CHECK();
}

void set_hub_args(RateArgs& a, const HubBufs& h)
{
    a.hub_tab = h.tab.p;
    a.hub_plan = h.plan.p;
    a.hub_pplan = h.pplan.p;
    a.hub_part = h.part.p;
}

struct LPBuffers {
    DBuf<int32_t> prop;
    DBuf<uint8_t> acc;
    DBuf<uint32_t> demand;
    HubBufs hub;
    DBuf<uint8_t> mflag;           // round stamp of the last move of every node
    DBuf<uint32_t> ckeys, cvals;   // contended (target, id), unordered
    DBuf<int64_t> base;            // [nlab] weight before a target's first proposal
    DBuf<int64_t> ctl;
    DBuf<uint8_t> active;          // [2n] active stamps of the rounds, by round parity (lp_run)
    DBuf<int64_t> sout;            // one-workgroup LP: moves per round, round count
};

void lp_buffers(Ctx& c, const DGraph& g, const LPSchedule* sched, int32_t nlab, LPBuffers& b)
{
    b.prop = DBuf<int32_t>(c, (size_t)g.n);
    b.acc = DBuf<uint8_t>(c, (size_t)g.n);
    b.demand = DBuf<uint32_t>(c, (size_t)nlab);
    if (sched) hub_buffers(c, g, *sched, b.hub);
    b.mflag = DBuf<uint8_t>(c, (size_t)g.n);
    b.ckeys = DBuf<uint32_t>(c, (size_t)g.n);
    b.cvals = DBuf<uint32_t>(c, (size_t)g.n);
    b.base = DBuf<int64_t>(c, (size_t)nlab);
    b.ctl = DBuf<int64_t>(c, kCtlWords);
    b.active = DBuf<uint8_t>(c, 2 * (size_t)g.n);
    b.sout = DBuf<int64_t>(c, kRounds + 1);
    // prop = -1, everything else 0, in one launch
    fill_bytes_many(c, {{b.prop.p, 4 * (int64_t)g.n, 0xFF},
                        {b.acc.p, (int64_t)g.n, 0},
                        {b.demand.p, 4 * (int64_t)nlab, 0},
                        {b.mflag.p, (int64_t)g.n, 0},
                        {b.ctl.p, (int64_t)sizeof(int64_t) * kCtlWords, 0},
                        {b.active.p, 2 * (int64_t)g.n, 0},
                        {b.sout.p, (int64_t)sizeof(int64_t) * (kRounds + 1), 0}});
}

RateArgs make_rate_args(Ctx& c, const DGraph& g, const LPState& st, uint32_t hpre, LPBuffers* b)
{
    RateArgs a;
    memset(&a, 0, sizeof(a));
    a.xadj = g.xadj;
    a.adjncy = g.adjncy;
    a.vwgt = g.vwgt;
    a.adjwgt = g.adjwgt;
    a.label = st.label;
    a.wt = st.wt;
    a.cap_vec = st.cap_vec;
    a.cap_scalar = st.cap_scalar;
    a.hpre = hpre;
    a.fav = st.fav;
    a.counters = c.spread(SP_RATED);
    a.gid = st.jt.gid;
    a.ghash = st.jt.ghash;
    a.loff = st.loff;
    a.gcap = st.gcap;
    a.tag = st.tag;
    a.hub_ts = c.tune.hub_ts;
    const int64_t badj = 4 * g.m, blab = 4 * (int64_t)g.n, bwt = 8 * (int64_t)st.nlab;
    const int64_t lim = int64_t(1) << 31;
    if (!c.plain_loads && g.m > 0 && st.nlab > 0 && badj < lim && blab < lim && bwt < lim) {
        a.bufok = 1;
        a.nr_adj = (uint32_t)badj;
        a.nr_lab = (uint32_t)blab;
        a.nr_wt = (uint32_t)bwt;
    }
    if (b) {
        a.prop = b->prop.p;
        a.demand = b->demand.p;
        a.ctl = b->ctl.p;
        set_hub_args(a, b->hub);
    }
    return a;
}

// The LDS tables of tiers 1-3 hold at least twice as many slots as the largest
// degree a tier may take (the tuning may only lower the cut-offs).
static_assert((1 << 7) >= 2 * T1_DEG && (1 << 10) >= 2 * T2_DEG && (1 << 13) >= 2 * T3_DEG, "LDS table sizes");

// Launch the rating kernels of class s over the lists described by segtab;
// grids are sized by the level's segment sizes (upper bounds of the lists).
void launch_rate(Ctx& c, RateArgs a, const LPSchedule& sched, int32_t s, const int32_t* list, const int32_t* segtab,
                 const int32_t* ubs)
{
    int64_t* bytes = c.spread(SP_BYTES);
    a.list = list;
    a.segtab = segtab;
    a.hub_off = sched.hub_slot_off.p;
    for (int t = 0; t < kTiers; ++t) {
        const int seg = t * kSub + s;
        const int32_t ub = ubs[seg];
        if (ub == 0) continue;
        a.seg = seg;
        // LP launches count their algorithmic bytes per class (tier 3 joins tier 2); the
        // balancer's rating launches are timed under the balance class and count no LP bytes
        if (!a.over) a.bytes_ctr = bytes + kSpreadWords * (t < 3 ? t : t == 3 ? KMP_PROF_RATE_T2 : KMP_PROF_RATE_HUB);
        const int cls = a.over ? KMP_PROF_BALANCE
                               : t == 0 ? KMP_PROF_RATE_T0
                               : t == 1 ? KMP_PROF_RATE_T1
                               : t <= 3 ? KMP_PROF_RATE_T2
                                        : KMP_PROF_RATE_HUB;
        switch (t) {
            case 0: {
                const int bs = spread_block(ub);
                const dim3 grid(grid_for(ub, bs, 65536)), block(bs);
                const bool ew = a.adjwgt != nullptr;
                if (a.over) {
                    if (ew) KMP_LAUNCH_TIMED(c, cls, (k_rate_lane<true, true, true, false>), grid, block, 0, a);
                    else KMP_LAUNCH_TIMED(c, cls, (k_rate_lane<false, true, true, false>), grid, block, 0, a);
                } else if (a.bufok) {
                    if (a.cap_vec) {
                        if (ew) KMP_LAUNCH_TIMED(c, cls, (k_rate_lane<true, true, false, true>), grid, block, 0, a);
                        else KMP_LAUNCH_TIMED(c, cls, (k_rate_lane<false, true, false, true>), grid, block, 0, a);
                    } else {
                        if (ew) KMP_LAUNCH_TIMED(c, cls, (k_rate_lane<true, false, false, true>), grid, block, 0, a);
                        else KMP_LAUNCH_TIMED(c, cls, (k_rate_lane<false, false, false, true>), grid, block, 0, a);
                    }
                } else if (a.cap_vec) {
                    if (ew) KMP_LAUNCH_TIMED(c, cls, (k_rate_lane<true, true, false, false>), grid, block, 0, a);
                    else KMP_LAUNCH_TIMED(c, cls, (k_rate_lane<false, true, false, false>), grid, block, 0, a);
                } else {
                    if (ew) KMP_LAUNCH_TIMED(c, cls, (k_rate_lane<true, false, false, false>), grid, block, 0, a);
                    else KMP_LAUNCH_TIMED(c, cls, (k_rate_lane<false, false, false, false>), grid, block, 0, a);
                }
                break;
            }
            case 1:
                KMP_LAUNCH_TIMED(c, cls, (k_rate_lds<16, 7>), dim3(grid_for(ub, kBlock / 16, 65536)), dim3(kBlock), 0,
                                 a);
                break;
            case 2:
                KMP_LAUNCH_TIMED(c, cls, (k_rate_lds<64, 10>), dim3(grid_for(ub, kBlock / 64, 65536)), dim3(kBlock),
                                 0, a);
                break;
            case 3:
                KMP_LAUNCH_TIMED(c, cls, (k_rate_lds<256, 13>), dim3(grid_for(ub, 1, 65536)), dim3(kBlock), 0, a);
                break;
            default: {
                // runs and label partitions of the segment's hubs: a hub of degree d has at most
                // d / kHubRun + 1 runs and d / kHubPartAvg + 1 partitions, and a region of 5 d slots
                const int64_t runs = sched.hub_slots_total / (5 * kHubRun) + ub;
                const int64_t parts = sched.hub_slots_total / (5 * kHubPartAvg) + ub;
                // the partitions' LDS tables: the tuning's size (a power of two, 64 .. kHubTS)
                if (a.hub_ts < 64 || a.hub_ts > kHubTS || (a.hub_ts & (a.hub_ts - 1))) a.hub_ts = kHubTS / 2;
                KMP_LAUNCH_TIMED(c, cls, k_hub_plan, dim3(1), dim3(kBlock), 0, a);
                KMP_LAUNCH_TIMED(c, cls, k_hub_split, dim3(grid_for(runs, 1, 16384)), dim3(kBlock), 0, a);
                KMP_LAUNCH_TIMED(c, cls, k_hub_agg, dim3(grid_for(parts, 1, 16384)), dim3(kBlock),
                                 (size_t)8 * a.hub_ts, a);
                KMP_LAUNCH_TIMED(c, cls, k_hub_final, dim3(grid_for(ub, kBlock / 64, 65536)), dim3(kBlock), 0, a);
                break;
            }
        }
    }
}

int32_t class_ub(const int32_t* ubs, int32_t s)
{
    int32_t t = 0;
    for (int q = 0; q < kTiers; ++q) t += ubs[q * kSub + s];
    return t;
}

CapArgs cap_args(const LPState& st)
{
    return CapArgs{st.cap_vec, st.cap_scalar, st.jt.gid, st.gcap};
}

void launch_admit(Ctx& c, const int32_t* ubs, int32_t s, const int32_t* list, const int32_t* segtab, LPState& st,
                  LPBuffers& b)
{
    const int32_t ub = class_ub(ubs, s);
    if (ub == 0) return;
    ProfScope ps(c, KMP_PROF_ADMIT);
    const int bs = spread_block(ub);
    hipLaunchKernelGGL(k_admit_fast, dim3(grid_for(ub, bs, 8192)), dim3(bs), 0, c.stream, b.ctl.p, list,
                       segtab, s, b.prop.p, b.demand.p, st.wt, cap_args(st), b.acc.p, b.ckeys.p, b.cvals.p,
                       b.base.p, CTL_CONT + (s & 1));
    KMP_LAUNCH_CHECK();
}

void launch_apply(Ctx& c, const int32_t* ubs, int32_t s, const int32_t* list, const int32_t* segtab,
                  const DGraph& g, LPState& st, LPBuffers& b, uint8_t* mflag, uint8_t stamp, int ms,
                  uint8_t* act_next)
{
    const int32_t ub = class_ub(ubs, s);
    if (ub == 0) return;
    ProfScope ps(c, KMP_PROF_APPLY);
    const int bs = spread_block(ub);
    hipLaunchKernelGGL(k_apply, dim3(grid_for(ub, bs, 8192)), dim3(bs), 0, c.stream, b.ctl.p, list, segtab,
                       s, b.prop.p, b.acc.p, b.demand.p, st.label, st.wt, g.vwgt, mflag, stamp, ms, b.ckeys.p,
                       b.cvals.p, b.base.p, cap_args(st), CTL_CONT + (s & 1),
                       (int64_t)(c.force_exact ? 0 : kSmallCap), g.xadj, g.adjncy, act_next, (uint8_t)(stamp + 1));
    KMP_LAUNCH_CHECK();
}

void ctl_set(Ctx& c, LPBuffers& b, int idx, int64_t v)
{
    hipLaunchKernelGGL(k_ctl_set, dim3(1), dim3(64), 0, c.stream, b.ctl.p, idx, v);
    KMP_LAUNCH_CHECK();
}

// Exact admission of the contended proposals of sub-round s (host synchronised).
void resolve_exact(Ctx& c, const DGraph& g, LPState& st, LPBuffers& b, int32_t s)
{
    const int cont_idx = CTL_CONT + (s & 1);
    const int64_t ncont = c.read1(b.ctl.p + cont_idx);
    if (ncont == 0) return;
    const int32_t n = g.n;
    DBuf<int32_t> flag(c, (size_t)n), pos(c, (size_t)n + 1);
    hipLaunchKernelGGL(k_contended_flags, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, b.acc.p, n, flag.p);
    KMP_LAUNCH_CHECK();
    scan_excl_i32(c, flag.p, pos.p, n, pos.p + n);
    DBuf<uint32_t> keys(c, ncont), vals(c, ncont), keys2(c, ncont), vals2(c, ncont);
    hipLaunchKernelGGL(k_contended_compact, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, b.acc.p, pos.p, n, b.prop.p,
                       keys.p, vals.p);
    KMP_LAUNCH_CHECK();
    radix_sort_pairs(c, keys.p, vals.p, keys2.p, vals2.p, ncont, bits_for((uint64_t)(st.nlab - 1)));
    DBuf<int64_t> pre(c, ncont);
    hipLaunchKernelGGL(k_gather_cw, dim3(grid_for(ncont)), dim3(kBlock), 0, c.stream, vals.p, ncont, g.vwgt, pre.p);
    KMP_LAUNCH_CHECK();
    scan_incl_i64(c, pre.p, pre.p, ncont);
    hipLaunchKernelGGL(k_heads, dim3(grid_for(ncont)), dim3(kBlock), 0, c.stream, keys.p, pre.p, vals.p, g.vwgt, ncont,
                       b.base.p);
    KMP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_decide, dim3(grid_for(ncont)), dim3(kBlock), 0, c.stream, keys.p, vals.p, pre.p, b.base.p,
                       ncont, st.wt, cap_args(st), b.acc.p);
    KMP_LAUNCH_CHECK();
    ctl_set(c, b, cont_idx, 0);
}

// One sub-round on the exact path (host synchronised after admission).
void subround_exact(Ctx& c, const DGraph& g, const LPSchedule& sched, int32_t s, const int32_t* list,
                    const int32_t* segtab, const int32_t* ubs, LPState& st, LPBuffers& b, const RateArgs& a,
                    bool rate, uint8_t* mflag, uint8_t stamp, int ms, uint8_t* act_next)
{
    if (rate) {
        launch_rate(c, a, sched, s, list, segtab, ubs);
        launch_admit(c, ubs, s, list, segtab, st, b);
    }
    resolve_exact(c, g, st, b, s);
    launch_apply(c, ubs, s, list, segtab, g, st, b, mflag, stamp, ms, act_next);
}

}  // namespace

void rate_for_balance(Ctx& c, const DGraph& g, int32_t level, uint64_t seed, int32_t round,
                      const LPSchedule& sched, const int32_t* part, const int64_t* wt, const int64_t* cap,
                      const uint8_t* over, int32_t* bal_t, int64_t* bal_d, const JobTabs& jt, const int32_t* boff)
{
    if (g.n == 0) return;
    LPState st{const_cast<int32_t*>(part), const_cast<int64_t*>(wt), 0, cap, 0, nullptr, TAG_BAL, jt, boff};
    RateArgs a = make_rate_args(c, g, st, hash_prefix(seed, {TAG_BAL, (uint32_t)level, (uint32_t)round}), nullptr);
    a.level = (uint32_t)level;
    a.round = (uint32_t)round;
    a.counters = c.spread(SP_BYTES + KMP_PROF_OTHER);  // balancing reports no rated edges
    a.bytes_ctr = c.spread(SP_BYTES + KMP_PROF_OTHER);  // nor LP bytes
    a.over = over;
    a.bal_t = bal_t;
    a.bal_d = bal_d;
    HubBufs hb;
    hub_buffers(c, g, sched, hb);
    set_hub_args(a, hb);
    for (int32_t s = 0; s < kSub; ++s) launch_rate(c, a, sched, s, sched.order.p, sched.segtab.p, sched.cnt);
}

namespace {

// A graph's level runs the one-workgroup LP when it is small, its state fits in
// LDS and its nodes all sit in rating tiers 0 and 1 (degree <= T1_DEG), unless
// the exact admission path is forced.
bool small_level(const Ctx& c, const DGraph& g, const LPSchedule& sched, int32_t nlab)
{
    if (!small_job_fits(c, g.n, nlab)) return false;
    for (int j = 2 * kSub; j < kSegs; ++j)
        if (sched.cnt[j]) return false;
    return true;
}

template <bool EW, bool CAPV, bool LCSR>
void launch_small(Ctx& c, unsigned jobs, size_t lds, const SmallLP& p)
{
    allow_lds((const void*)k_lp_small<EW, CAPV, LCSR>, (int)kSmallLdsBudget);  // beyond the 64 KiB default
    KMP_LAUNCH_TIMED(c, KMP_PROF_LP_SMALL, (k_lp_small<EW, CAPV, LCSR>), dim3(jobs), dim3(kSmallBlock), lds, p);
}

// The LP of the given jobs (node ranges and label ranges), one workgroup each.
LPStats lp_run_small(Ctx& c, const DGraph& g, int32_t level, uint64_t seed, LPState& st, LPBuffers& b,
                     const std::vector<int32_t>& start, const std::vector<int32_t>& count,
                     const std::vector<int32_t>& loff, const std::vector<int32_t>& nlab)
{
    SmallLP p;
    memset(&p, 0, sizeof(p));
    p.a = make_rate_args(c, g, st, 0, &b);
    p.a.amode = c.async_lp == 1 ? (st.tag == TAG_REF ? 2 : 1) : 0;
    p.a.level = (uint32_t)level;
    p.a.ctl = nullptr;
    p.a.bytes_ctr = c.spread(SP_BYTES + KMP_PROF_LP_SMALL);
    p.label = st.label;
    p.wt = st.wt;
    const size_t nj = start.size();
    DBuf<int32_t> dt;
    if (nj == 1) {
        p.one[0] = start[0];
        p.one[1] = count[0];
        p.one[2] = loff[0];
        p.one[3] = nlab[0];
    } else {
        std::vector<int32_t> tab;
        tab.reserve(4 * nj);
        tab.insert(tab.end(), start.begin(), start.end());
        tab.insert(tab.end(), count.begin(), count.end());
        tab.insert(tab.end(), loff.begin(), loff.end());
        tab.insert(tab.end(), nlab.begin(), nlab.end());
        dt = DBuf<int32_t>(c, tab.size());
        c.write(dt.p, tab.data(), sizeof(int32_t) * tab.size());
        p.jstart = dt.p;
        p.jcount = dt.p + nj;
        p.jloff = dt.p + 2 * nj;
        p.jnlab = dt.p + 3 * nj;
    }
    p.hsub = hash_prefix(seed, {TAG_SUB, (uint32_t)level});
    for (int r = 0; r < kRounds; ++r) p.hpre[r] = hash_prefix(seed, {st.tag, (uint32_t)level, (uint32_t)r});
    p.cut0 = c.tune.cut[0];
    p.cont = b.ckeys.p;
    p.out = st.moves_out ? st.moves_out : b.sout.p;
    int64_t lds = 0;
    for (size_t q = 0; q < nj; ++q) lds = std::max(lds, small_lds_bytes(count[q], nlab[q]));
    const bool ew = g.adjwgt != nullptr, capv = st.cap_vec != nullptr;
    // one job over the whole graph: its CSR goes to LDS too when it fits
    bool lcsr = false;
    if (nj == 1 && start[0] == 0 && count[0] == g.n) {
        const int64_t csr = ((lds + 15) & ~(int64_t)15) + 4 * ((int64_t)g.n + 1) + (g.vwgt ? 4 * (int64_t)g.n : 0) +
                            (ew ? 4 * g.m : 0) + 2 * g.m;
        if (csr <= kSmallLdsBudget) {
            lds = csr;
            lcsr = true;
        }
    }
    const size_t L = (size_t)lds;
    if (lcsr) {
        if (ew && capv) launch_small<true, true, true>(c, 1, L, p);
        else if (ew) launch_small<true, false, true>(c, 1, L, p);
        else if (capv) launch_small<false, true, true>(c, 1, L, p);
        else launch_small<false, false, true>(c, 1, L, p);
    } else {
        if (ew && capv) launch_small<true, true, false>(c, (unsigned)nj, L, p);
        else if (ew) launch_small<true, false, false>(c, (unsigned)nj, L, p);
        else if (capv) launch_small<false, true, false>(c, (unsigned)nj, L, p);
        else launch_small<false, false, false>(c, (unsigned)nj, L, p);
    }
    LPStats out;
    if (st.moves_out) return out;  // the caller reads the accumulated counts later
    int64_t h[kRounds + 1];
    c.read(h, b.sout.p, sizeof(h));
    out.rounds = (int32_t)h[kRounds];
    for (int r = 0; r < kRounds; ++r) out.moves[r] = h[r];
    return out;
}

}  // namespace

int32_t small_limit(const Ctx& c)
{
    if (c.force_exact) return -1;
    return c.small_level_n != 0 ? c.small_level_n : c.tune.small_level_n;
}

bool small_job_fits(const Ctx& c, int32_t nodes, int32_t labels)
{
    const int32_t limit = small_limit(c);
    return limit >= 0 && nodes > 0 && nodes <= limit && small_lds_bytes(nodes, labels) <= kSmallLdsBudget;
}

namespace {

// The launch-per-step LP: kSub sub-rounds of rate / admit / apply launches per
// round, one read-back per round.  Nodes of the jobs in `skip` (already done
// by the one-workgroup LP) are left out of round 0 and are never activated.
LPStats lp_rounds(Ctx& c, const DGraph& g, int32_t level, uint64_t seed, const LPSchedule& sched, LPState& st,
                  LPBuffers& b, const std::vector<int32_t>& skip)
{
    LPStats out;
    const int32_t n = g.n;
    SegBounds bounds;
    for (int j = 0; j <= kSegs; ++j) bounds.off[j] = sched.off[j];
    int32_t ub[kSegs];
    memcpy(ub, sched.cnt, sizeof(ub));
    // Every round walks the same lists: round 0 rates all of them, later rounds
    // the nodes whose stamp in act[r & 1] is r + 1, set when a neighbour moved in
    // round r - 1 (by k_apply for moved nodes of tiers 0-1, k_push_active above).
    const int32_t* list = sched.order.p;
    const int32_t* segtab = sched.segtab.p;
    DBuf<int32_t> flist;
    if (!skip.empty()) {
        // batches: the lists without the skipped jobs' nodes
        int32_t* ftab = reinterpret_cast<int32_t*>(b.ctl.p + CTL_MS + kSpreadWords);
        flist = DBuf<int32_t>(c, (size_t)n);
        std::vector<uint8_t> flag((size_t)st.njobs, 0);
        for (int32_t j : skip) flag[j] = 1;
        DBuf<uint8_t> dflag(c, flag.size());
        c.write(dflag.p, flag.data(), flag.size());
        int32_t mseg = 1;
        for (int j = 0; j < kSegs; ++j) mseg = std::max(mseg, sched.cnt[j]);
        hipLaunchKernelGGL(k_order_skip_jobs, dim3(grid_for(mseg, kBlock, 1024), kSegs), dim3(kBlock), 0, c.stream,
                           sched.order.p, bounds, st.jt.gid, dflag.p, flist.p, ftab);
        KMP_LAUNCH_CHECK();
        int32_t tab[2 * kSegs];
        c.read(tab, ftab, sizeof(tab));
        for (int j = 0; j < kSegs; ++j) ub[j] = tab[kSegs + j];
        list = flist.p;
        segtab = ftab;
    }
    uint8_t* act[2] = {b.active.p, b.active.p + n};
    int32_t mbig = 0;  // largest segment of tiers 2-4 (their marking is a launch of its own)
    for (int j = 2 * kSub; j < kSegs; ++j) mbig = std::max(mbig, ub[j]);
    auto push_big = [&](int32_t r) {
        if (mbig == 0 || r + 1 >= kRounds) return;
        ProfScope ps(c, KMP_PROF_ACTIVE);
        hipLaunchKernelGGL(k_push_active, dim3(grid_for(mbig, kBlock, 1024), kSegs - 2 * kSub), dim3(kBlock), 0,
                           c.stream, b.ctl.p, list, segtab, b.mflag.p, (uint8_t)(r + 1), g.xadj, g.adjncy,
                           act[(r + 1) & 1], (uint8_t)(r + 2), 2 * kSub);
        KMP_LAUNCH_CHECK();
    };
    struct {
        int64_t ctl[CTL_N];
        int64_t moved[kSpreadWords];
    } h;
    static_assert(sizeof(h) <= sizeof(int64_t) * kCtlWords, "control block layout");
    auto args_of = [&](int32_t r) {
        RateArgs a = make_rate_args(c, g, st, hash_prefix(seed, {st.tag, (uint32_t)level, (uint32_t)r}), &b);
        a.level = (uint32_t)level;
        a.round = (uint32_t)r;
        a.active = r == 0 ? nullptr : act[r & 1];
        a.stamp = (uint8_t)(r + 1);
        return a;
    };
    auto next_of = [&](int32_t r) { return r + 1 < kRounds ? act[(r + 1) & 1] : nullptr; };
    // One round: S sub-rounds with no host synchronisation in between.
    auto launch_round = [&](int32_t r) {
        const RateArgs a = args_of(r);
        for (int32_t s = 0; s < kSub; ++s) {
            launch_rate(c, a, sched, s, list, segtab, ub);
            launch_admit(c, ub, s, list, segtab, st, b);
            launch_apply(c, ub, s, list, segtab, g, st, b, b.mflag.p, (uint8_t)(r + 1), CTL_MS + r,
                         next_of(r));
        }
        push_big(r);
    };
    // Clustering rarely converges before the last round, so its rounds are all
    // enqueued before the host reads the move counts once (a round after one
    // without moves has no active node and changes nothing).  Refinement usually
    // stops after a round or two: it reads the counts after every round.
    const bool ahead = st.tag == TAG_CL;
    int32_t r = 0;
    while (r < kRounds) {
        const int32_t last = ahead ? kRounds - 1 : r;
        for (int32_t q = r; q <= last; ++q) launch_round(q);
        c.read(&h, b.ctl.p, sizeof(h));
        int32_t done = last;  // rounds up to `done` are final
        if (h.ctl[CTL_ABORT]) {
            // round r0 stopped at sub-round s0 and every launch after it did
            // nothing: finish r0 on the exact path, then carry on from r0 + 1
            const int32_t s0 = (int32_t)h.ctl[CTL_ABORT_SUB];
            const int32_t r0 = (int32_t)h.ctl[CTL_ABORT_STAMP] - 1;
            if (r0 < r || r0 > last) throw Error(KMP_EHIP, "LP abort recorded for an unexpected round");
            const RateArgs a = args_of(r0);
            const uint8_t stamp = (uint8_t)(r0 + 1);
            const int ms = CTL_MS + r0;
            ctl_set(c, b, CTL_ABORT, 0);
            subround_exact(c, g, sched, s0, list, segtab, ub, st, b, a, false, b.mflag.p, stamp, ms, next_of(r0));
            for (int32_t s = s0 + 1; s < kSub; ++s)
                subround_exact(c, g, sched, s, list, segtab, ub, st, b, a, true, b.mflag.p, stamp, ms, next_of(r0));
            push_big(r0);
            c.read(&h, b.ctl.p, sizeof(h));
            out.exact_subrounds += kSub - s0;
            done = r0;
        }
        bool stop = false;
        for (int32_t q = r; q <= done && !stop; ++q) {
            int64_t nm = 0;
            for (int k = 0; k < kSpreadSlots; ++k) nm += h.moved[k * kSpreadStride + q];
            out.moves[q] = nm;
            out.rounds = q + 1;
            stop = nm == 0;
        }
        if (stop) break;
        r = done + 1;
    }
    return out;
}

// Asynchronous LP (paper Sec. 5.1 "Parallelization", Sec. 5.3 "Local
// Improvement") over an asynchronous schedule: per round and class one rating
// launch per tier, each rated node moving at once (clustering: fetch-and-add,
// refinement: compare-and-swap), so later classes see the moves of earlier
// ones; then the neighbours of the round's movers are marked for the next
// round.  Serial mode (c.async_lp == 2) launches the kernels once per node in
// visit order, which is the execution by one processing element.
LPStats lp_async_rounds(Ctx& c, const DGraph& g, int32_t level, uint64_t seed, const LPSchedule& sched, LPState& st)
{
    LPStats out;
    const int32_t n = g.n;
    HubBufs hub;
    hub_buffers(c, g, sched, hub);
    DBuf<uint8_t> mflag(c, (size_t)n), active(c, 2 * (size_t)n);
    DBuf<int64_t> ctl(c, kCtlWords);
    fill_bytes_many(c, {{mflag.p, (int64_t)n, 0},
                        {active.p, 2 * (int64_t)n, 0},
                        {ctl.p, (int64_t)sizeof(int64_t) * kCtlWords, 0}});
    const bool serial = c.async_lp == 2;
    DBuf<int32_t> one;  // serial mode: every segment starts at 0 and holds one node
    if (serial) {
        int32_t tab[2 * kSegs];
        for (int j = 0; j < kSegs; ++j) {
            tab[j] = 0;
            tab[kSegs + j] = 1;
        }
        one = DBuf<int32_t>(c, 2 * kSegs);
        c.write(one.p, tab, sizeof(tab));
    }
    uint8_t* act[2] = {active.p, active.p + n};
    int32_t mseg = 0;
    for (int j = 0; j < kSegs; ++j) mseg = std::max(mseg, sched.cnt[j]);
    auto launch_round = [&](int32_t r) {
        RateArgs a = make_rate_args(c, g, st, hash_prefix(seed, {st.tag, (uint32_t)level, (uint32_t)r}), nullptr);
        a.ctl = ctl.p;
        set_hub_args(a, hub);
        a.level = (uint32_t)level;
        a.round = (uint32_t)r;
        a.active = r == 0 ? nullptr : act[r & 1];
        a.stamp = (uint8_t)(r + 1);
        a.amode = st.tag == TAG_REF ? 2 : 1;
        a.label_w = st.label;
        a.mflag = mflag.p;
        a.moved_ctr = ctl.p + CTL_MS + r;
        for (int32_t s = 0; s < kSub; ++s) {
            if (!serial) {
                launch_rate(c, a, sched, s, sched.order.p, sched.segtab.p, sched.cnt);
                continue;
            }
            for (int t = 0; t < kTiers; ++t) {
                const int seg = t * kSub + s;
                int32_t u1[kSegs] = {};
                u1[seg] = 1;
                const int32_t* base = sched.order.p + sched.off[seg];
                for (int32_t p = 0; p < sched.cnt[seg]; ++p) launch_rate(c, a, sched, s, base + p, one.p, u1);
            }
        }
        if (r + 1 < kRounds && mseg > 0) {
            ProfScope ps(c, KMP_PROF_ACTIVE);
            hipLaunchKernelGGL(k_push_active, dim3(grid_for(mseg, kBlock, 1024), kSegs), dim3(kBlock), 0, c.stream,
                               ctl.p, sched.order.p, sched.segtab.p, mflag.p, (uint8_t)(r + 1), g.xadj, g.adjncy,
                               act[(r + 1) & 1], (uint8_t)(r + 2), 0);
            KMP_LAUNCH_CHECK();
        }
    };
    int64_t moved[kSpreadWords];
    // clustering enqueues every round before one read-back (a round after one
    // without moves rates nothing); refinement reads the count after each round
    const bool ahead = st.tag == TAG_CL;
    for (int32_t r = 0; r < kRounds;) {
        const int32_t last = ahead ? kRounds - 1 : r;
        for (int32_t q = r; q <= last; ++q) launch_round(q);
        c.read(moved, ctl.p + CTL_MS, sizeof(moved));
        bool stop = false;
        for (int32_t q = r; q <= last && !stop; ++q) {
            int64_t nm = 0;
            for (int k = 0; k < kSpreadSlots; ++k) nm += moved[k * kSpreadStride + q];
            out.moves[q] = nm;
            out.rounds = q + 1;
            stop = nm == 0;
        }
        if (stop) break;
        r = last + 1;
    }
    return out;
}

}  // namespace

LPStats lp_run(Ctx& c, const DGraph& g, int32_t level, uint64_t seed, const LPSchedule* sched_p, LPState& st)
{
    const int32_t n = g.n;
    if (n == 0) return LPStats();
    if (c.async_lp) {
        if (!sched_p) throw Error(KMP_EHIP, "the asynchronous LP needs its visit-order schedule");
        // a small single graph runs its whole call in one workgroup (not in serial mode, whose
        // one-node launches are the one-processing-element execution)
        if (c.async_lp == 1 && !st.jt.gid && small_level(c, g, *sched_p, st.nlab)) {
            LPBuffers b;
            lp_buffers(c, g, nullptr, st.nlab, b);
            return lp_run_small(c, g, level, seed, st, b, {0}, {n}, {0}, {st.nlab});
        }
        return lp_async_rounds(c, g, level, seed, *sched_p, st);
    }
    if (!sched_p) {  // a small single graph: no schedule needed
        LPBuffers b;
        lp_buffers(c, g, nullptr, st.nlab, b);
        return lp_run_small(c, g, level, seed, st, b, {0}, {n}, {0}, {st.nlab});
    }
    const LPSchedule& sched = *sched_p;
    // jobs that run the one-workgroup LP; the others take the launch-per-step path
    std::vector<int32_t> ss, sc, sl, sn;
    if (!st.jt.gid) {
        if (small_level(c, g, sched, st.nlab)) {
            ss.assign(1, 0);
            sc.assign(1, n);
            sl.assign(1, 0);
            sn.assign(1, st.nlab);
        }
    } else {
        ss = st.small_start;
        sc = st.small_count;
        sl = st.small_loff;
        sn = st.small_nlab;
    }
    int64_t small_nodes = 0;
    for (int32_t x : sc) small_nodes += x;
    const bool all_small = !ss.empty() && small_nodes == sched.off[kSegs];
    LPBuffers b;
    lp_buffers(c, g, &sched, st.nlab, b);
    LPStats small;
    if (!ss.empty()) {
        small = lp_run_small(c, g, level, seed, st, b, ss, sc, sl, sn);
        if (all_small) return small;
    }
    LPStats out = lp_rounds(c, g, level, seed, sched, st, b, st.small_jobs);
    for (int r = 0; r < kRounds; ++r) out.moves[r] += small.moves[r];
    out.rounds = std::max(out.rounds, small.rounds);
    return out;
}

int64_t lp_subround(Ctx& c, const DGraph& g, int32_t level, int32_t round, int32_t s, uint64_t seed,
                    const LPSchedule& sched, LPState& st, const uint8_t* active, uint8_t* moved)
{
    if (g.n == 0) return 0;
    LPBuffers b;
    lp_buffers(c, g, &sched, st.nlab, b);
    RateArgs a = make_rate_args(c, g, st, hash_prefix(seed, {st.tag, (uint32_t)level, (uint32_t)round}), &b);
    a.level = (uint32_t)level;
    a.round = (uint32_t)round;
    a.active = active;
    a.stamp = 1;  // the caller's active flags are 0 / 1
    subround_exact(c, g, sched, s, sched.order.p, sched.segtab.p, sched.cnt, st, b, a, true, moved, 1, CTL_MS,
                   nullptr);
    int64_t slots[kSpreadWords];
    c.read(slots, b.ctl.p + CTL_MS, sizeof(slots));
    int64_t nm = 0;
    for (int q = 0; q < kSpreadSlots; ++q) nm += slots[q * kSpreadStride];
    return nm;
}

}  // namespace kmp
