// Size-constrained label propagation on gfx950 (paper Sec. 2 "Size-
// Constrained Label Propagation", Sec. 5.1 coarsening, Sec. 5.3 refinement).
//
// Deterministic sub-round reading: a round visits the nodes in S = 4 hash
// classes; the nodes of one class are rated against the state at the start of
// the sub-round (rate kernel), then proposals into one target are admitted in
// ascending node id while the running weight fits (admission), then applied.
//
// Rate kernel tiers by degree (execution layout only; results identical):
//   tier 0  deg <= 16    8 lanes per node, 32-slot LDS hash per node
//   tier 1  deg <= 128   one wavefront per node, 256-slot LDS hash
//   tier 2  deg <= 2048  one workgroup per node, 4096-slot LDS hash
//   tier 3  deg >  2048  one workgroup per hub, global-memory hash table
// Admission: proposals add their weight to demand[K]; targets whose whole
// demand fits are admitted at once; the rest ("contended") are sorted by
// (target, id) and admitted by an inclusive prefix sum.
#include "kmp_dev.h"

namespace kmp {

namespace {

constexpr int T0_DEG = 16, T1_DEG = 128, T2_DEG = 2048;
constexpr uint32_t EMPTY = 0xFFFFFFFFu;

struct Seg4 {
    int32_t off[4];
    int32_t cnt[4];
};

__device__ inline int32_t seg_index(const Seg4& s, int64_t i)
{
    // map a flat index over the 4 segments to a position in `order`
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (i < s.cnt[t]) return s.off[t] + (int32_t)i;
        i -= s.cnt[t];
    }
    return -1;
}

// ---------------------------------------------------------------- schedule
__global__ __launch_bounds__(kBlock) void k_sched_keys(const int32_t* __restrict__ xadj, int32_t n, uint32_t hsub,
                                                       uint32_t* __restrict__ key, uint32_t* __restrict__ val,
                                                       int32_t* __restrict__ cnt16)
{
    __shared__ int32_t h[16];
    if (threadIdx.x < 16) h[threadIdx.x] = 0;
    __syncthreads();
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) {
        uint32_t s = hash_step(hsub, (uint32_t)v, 3) % kSub;
        int32_t d = xadj[v + 1] - xadj[v];
        uint32_t t = d <= T0_DEG ? 0 : d <= T1_DEG ? 1 : d <= T2_DEG ? 2 : 3;
        uint32_t k = t * kSub + s;
        key[v] = k;
        val[v] = (uint32_t)v;
        atomicAdd(&h[k], 1);
    }
    __syncthreads();
    if (threadIdx.x < 16 && h[threadIdx.x]) atomicAdd(&cnt16[threadIdx.x], h[threadIdx.x]);
}

__global__ void k_hub_slots(const int32_t* __restrict__ xadj, const int32_t* __restrict__ hubs, int32_t nh,
                            int64_t* __restrict__ slots)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nh) return;
    int32_t v = hubs[i];
    int64_t d = xadj[v + 1] - xadj[v];
    int64_t s = 1;
    while (s < 2 * d) s <<= 1;
    slots[i] = s;
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

template <int WIDTH>
__device__ inline Key3 group_best(Key3 a)
{
#pragma unroll
    for (int d = WIDTH / 2; d > 0; d >>= 1) {
        Key3 b;
        b.r = __shfl_xor(a.r, d, WIDTH);
        b.h = __shfl_xor(a.h, d, WIDTH);
        b.k = __shfl_xor(a.k, d, WIDTH);
        if (better(b, a)) a = b;
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
    const uint8_t* active;  // NULL = all
    uint32_t hpre;          // H prefix over (seed; tag, level, round)
    int32_t* prop;          // [n], -1 = no proposal
    uint32_t* fav;          // [n] or NULL
    uint32_t* demand;       // [nlab]
    int64_t* counters;      // [0] rated edges
    int64_t* bytes_ctr;     // algorithmic bytes of this launch's class
    // hubs (tier 3)
    uint32_t* hub_keys;
    uint32_t* hub_vals;
    const int64_t* hub_off;
    // balance mode (over != NULL): rate the nodes of overloaded blocks only,
    // targets must be non-overloaded; write best target / gain / own rating
    const uint8_t* over;
    int32_t* bal_t;
    int64_t* bal_d;
};

__device__ inline bool node_selected(const RateArgs& a, int32_t v)
{
    if (a.over) return a.over[a.label[v]] != 0;
    return !a.active || a.active[v];
}

__device__ inline void write_result(const RateArgs& a, int32_t v, const Key3& fav, const Key3& adm, uint32_t rown,
                                    int64_t cv)
{
    if (a.over) {
        a.bal_t[v] = adm.r ? (int32_t)adm.k : -1;
        a.bal_d[v] = adm.r ? (int64_t)adm.r - (int64_t)rown : -(int64_t)rown;
        return;
    }
    if (a.fav) a.fav[v] = fav.r ? fav.k : kNone;
    if (adm.r > rown) {
        a.prop[v] = (int32_t)adm.k;
        atomicAdd(&a.demand[adm.k], (uint32_t)cv);
    }
}

__device__ inline int64_t cap_of(const RateArgs& a, uint32_t K) { return a.cap_vec ? a.cap_vec[K] : a.cap_scalar; }

// Evaluate one table entry for the lane-local bests.
__device__ inline void consider(const RateArgs& a, uint32_t key, uint32_t val, uint32_t own, int64_t cv, Key3& fav,
                                Key3& adm, uint32_t& rown)
{
    if (key == EMPTY) return;
    if (key == own) {
        rown = val;
        return;
    }
    Key3 c{val, hash_step(a.hpre, key, 4), key};
    if (better(c, fav)) fav = c;
    if (better(c, adm)) {
        if (a.wt[key] + cv <= cap_of(a, key) && !(a.over && a.over[key])) adm = c;
    }
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

// G lanes per node, 2^HB slots per node in LDS.  256 threads per block.
template <int G, int HB>
__global__ __launch_bounds__(kBlock) void k_rate_lds(RateArgs a, const int32_t* __restrict__ order, int32_t count)
{
    constexpr int GPB = kBlock / G;
    constexpr int HS = 1 << HB;
    __shared__ uint32_t s_keys[GPB * HS];
    __shared__ uint32_t s_vals[GPB * HS];
    __shared__ Key3 s_red[2][4];
    __shared__ uint32_t s_rown[4];
    const int tid = threadIdx.x;
    const int grp = tid / G, gl = tid % G;
    uint32_t* keys = s_keys + grp * HS;
    uint32_t* vals = s_vals + grp * HS;
    int64_t edges = 0, nodes = 0;
    for (int64_t base = (int64_t)blockIdx.x * GPB; base < count; base += (int64_t)gridDim.x * GPB) {
        const int64_t i = base + grp;
        int32_t v = -1;
        if (i < count) {
            v = order[i];
            if (!node_selected(a, v)) v = -1;
        }
        for (int j = gl; j < HS; j += G) {
            keys[j] = EMPTY;
            vals[j] = 0;
        }
        __syncthreads();
        int32_t e0 = 0, e1 = 0;
        if (v >= 0) {
            e0 = a.xadj[v];
            e1 = a.xadj[v + 1];
            for (int32_t e = e0 + gl; e < e1; e += G) {
                uint32_t K = (uint32_t)a.label[a.adjncy[e]];
                uint32_t w = a.adjwgt ? (uint32_t)a.adjwgt[e] : 1u;
                lds_insert(keys, vals, HB, K, w);
            }
            if (gl == 0) {
                edges += e1 - e0;
                nodes += 1;
            }
        }
        __syncthreads();
        Key3 fav{0, 0, 0}, adm{0, 0, 0};
        uint32_t rown = 0;
        uint32_t own = 0;
        int64_t cv = 0;
        if (v >= 0) {
            own = (uint32_t)a.label[v];
            cv = a.vwgt ? a.vwgt[v] : 1;
            for (int j = gl; j < HS; j += G) consider(a, keys[j], vals[j], own, cv, fav, adm, rown);
        }
        if (G <= 64) {
            fav = group_best<G>(fav);
            adm = group_best<G>(adm);
#pragma unroll
            for (int d = G / 2; d > 0; d >>= 1) rown += __shfl_xor(rown, d, G);
        } else {
            // G == 256: wave reduce, then across the 4 waves through LDS
            fav = group_best<64>(fav);
            adm = group_best<64>(adm);
#pragma unroll
            for (int d = 32; d > 0; d >>= 1) rown += __shfl_xor(rown, d, 64);
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
        if (v >= 0 && gl == 0) write_result(a, v, fav, adm, rown, cv);
        __syncthreads();
    }
    // rated edge statistic and algorithmic bytes (per wave leader)
    for (int d = 32; d > 0; d >>= 1) {
        edges += __shfl_xor(edges, d, 64);
        nodes += __shfl_xor(nodes, d, 64);
    }
    if ((tid & 63) == 0 && edges) {
        atomicAdd((unsigned long long*)&a.counters[0], (unsigned long long)edges);
        const int64_t bytes = 25 * nodes + (a.adjwgt ? 12 : 8) * edges;
        atomicAdd((unsigned long long*)a.bytes_ctr, (unsigned long long)bytes);
    } else if ((tid & 63) == 0 && nodes) {
        atomicAdd((unsigned long long*)a.bytes_ctr, (unsigned long long)(25 * nodes));
    }
}

// One workgroup per hub node, hash table in global memory.
__global__ __launch_bounds__(kBlock) void k_rate_hub(RateArgs a, const int32_t* __restrict__ order, int32_t count)
{
    __shared__ Key3 s_red[2][4];
    __shared__ uint32_t s_rown[4];
    const int tid = threadIdx.x;
    for (int64_t i = blockIdx.x; i < count; i += gridDim.x) {
        int32_t v = order[i];
        if (!node_selected(a, v)) continue;  // uniform across the block
        const int32_t e0 = a.xadj[v], e1 = a.xadj[v + 1];
        const int64_t d = e1 - e0;
        int bits = 1;
        while ((1ll << bits) < 2 * d) ++bits;
        const int64_t hs = 1ll << bits;
        uint32_t* keys = a.hub_keys + a.hub_off[i];
        uint32_t* vals = a.hub_vals + a.hub_off[i];
        for (int64_t j = tid; j < hs; j += kBlock) {
            keys[j] = EMPTY;
            vals[j] = 0;
        }
        __threadfence_block();
        __syncthreads();
        for (int32_t e = e0 + tid; e < e1; e += kBlock) {
            uint32_t K = (uint32_t)a.label[a.adjncy[e]];
            uint32_t w = a.adjwgt ? (uint32_t)a.adjwgt[e] : 1u;
            const uint32_t mask = (uint32_t)(hs - 1);
            uint32_t h = slot_of(K, bits) & mask;
            while (true) {
                uint32_t old = atomicCAS(&keys[h], EMPTY, K);
                if (old == EMPTY || old == K) {
                    atomicAdd(&vals[h], w);
                    break;
                }
                h = (h + 1) & mask;
            }
        }
        __threadfence_block();
        __syncthreads();
        const uint32_t own = (uint32_t)a.label[v];
        const int64_t cv = a.vwgt ? a.vwgt[v] : 1;
        Key3 fav{0, 0, 0}, adm{0, 0, 0};
        uint32_t rown = 0;
        for (int64_t j = tid; j < hs; j += kBlock) {
            uint32_t key = __hip_atomic_load(&keys[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t val = __hip_atomic_load(&vals[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            consider(a, key, val, own, cv, fav, adm, rown);
        }
        fav = group_best<64>(fav);
        adm = group_best<64>(adm);
        for (int dd = 32; dd > 0; dd >>= 1) rown += __shfl_xor(rown, dd, 64);
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
            write_result(a, v, fav, adm, rown, cv);
            atomicAdd((unsigned long long*)&a.counters[0], (unsigned long long)d);
            atomicAdd((unsigned long long*)a.bytes_ctr, (unsigned long long)(25 + (a.adjwgt ? 12 : 8) * d));
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- admission
// acc[v]: 0 none, 1 admitted, 2 contended (decided by the exact path)
__global__ void k_admit_fast(Seg4 seg, int64_t total, const int32_t* __restrict__ order,
                             const int32_t* __restrict__ prop, const uint32_t* __restrict__ demand,
                             const int64_t* __restrict__ wt, const int64_t* __restrict__ cap_vec, int64_t cap_scalar,
                             uint8_t* __restrict__ acc, int64_t* counters)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int contended = 0;
    if (i < total) {
        int32_t v = order[seg_index(seg, i)];
        int32_t K = prop[v];
        if (K >= 0) {
            int64_t cap = cap_vec ? cap_vec[K] : cap_scalar;
            if (wt[K] + (int64_t)demand[K] <= cap) {
                acc[v] = 1;
            } else {
                acc[v] = 2;
                contended = 1;
            }
        }
    }
    uint64_t b = ballot64(contended);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd((unsigned long long*)&counters[1], (unsigned long long)__popcll(b));
}

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
                         const int64_t* __restrict__ wt, const int64_t* __restrict__ cap_vec, int64_t cap_scalar,
                         uint8_t* __restrict__ acc)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    uint32_t K = keys[i];
    int64_t cap = cap_vec ? cap_vec[K] : cap_scalar;
    acc[vals[i]] = wt[K] + (pre[i] - base[K]) <= cap ? 1 : 0;
}

__global__ void k_apply(Seg4 seg, int64_t total, const int32_t* __restrict__ order, int32_t* __restrict__ prop,
                        uint8_t* __restrict__ acc, uint32_t* __restrict__ demand, int32_t* __restrict__ label,
                        int64_t* __restrict__ wt, const int32_t* __restrict__ vwgt, uint8_t* __restrict__ moved,
                        int32_t* __restrict__ moved_list, int64_t* counters)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    int32_t v = order[seg_index(seg, i)];
    int32_t K = prop[v];
    if (K < 0) return;
    if (acc[v] == 1) {
        int64_t c = vwgt ? vwgt[v] : 1;
        int32_t old = label[v];
        label[v] = K;
        atomicAdd((unsigned long long*)&wt[K], (unsigned long long)c);
        atomicAdd((unsigned long long*)&wt[old], (unsigned long long)(-c));
        if (moved) moved[v] = 1;
        unsigned long long slot = atomicAdd((unsigned long long*)&counters[2], 1ull);
        if (moved_list) moved_list[slot] = v;
    }
    prop[v] = -1;
    acc[v] = 0;
    demand[K] = 0;
}

// mark the neighbours of moved nodes active for the next round
__global__ void k_push_active(const int32_t* __restrict__ moved_list, int64_t nm, const int32_t* __restrict__ xadj,
                              const int32_t* __restrict__ adjncy, uint8_t* __restrict__ active)
{
    // one wavefront per moved node
    const int lane = threadIdx.x & 63;
    int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (; w < nm; w += nw) {
        int32_t v = moved_list[w];
        for (int32_t e = xadj[v] + lane; e < xadj[v + 1]; e += 64) active[adjncy[e]] = 1;
    }
}

}  // namespace

// ================================================================ host side

void lp_build_schedule(Ctx& c, const DGraph& g, int32_t level, uint64_t seed, LPSchedule& sched)
{
    const int32_t n = g.n;
    sched.order = DBuf<int32_t>(c, (size_t)n);
    memset(sched.off, 0, sizeof(sched.off));
    memset(sched.cnt, 0, sizeof(sched.cnt));
    sched.hub_slots_total = 0;
    sched.hub_start = n;
    if (n == 0) return;
    DBuf<uint32_t> key(c, n), val(c, n), key2(c, n), val2(c, n);
    DBuf<int32_t> cnt(c, 16);
    c.zero(cnt.p, 16 * sizeof(int32_t));
    const uint32_t hsub = hash_prefix(seed, {TAG_SUB, (uint32_t)level});
    ProfScope ps(c, KMP_PROF_SCHEDULE);
    hipLaunchKernelGGL(k_sched_keys, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, g.xadj, n, hsub, key.p, val.p,
                       cnt.p);
    KMP_LAUNCH_CHECK();
    radix_sort_pairs(c, key.p, val.p, key2.p, val2.p, n, 4);
    KMP_HIP(hipMemcpyAsync(sched.order.p, val.p, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, c.stream));
    int32_t h[16];
    c.read(h, cnt.p, sizeof(h));
    // key = tier * 4 + class: the segments follow in that order
    int32_t pos = 0;
    int32_t segoff[4][4];
    for (int t = 0; t < 4; ++t)
        for (int s = 0; s < kSub; ++s) {
            segoff[t][s] = pos;
            sched.off[s][t] = pos;
            sched.cnt[s][t] = h[t * kSub + s];
            pos += h[t * kSub + s];
        }
    sched.hub_start = segoff[3][0];
    // hub hash tables: hubs of all classes are contiguous from segoff[3][0]
    int32_t nh = n - segoff[3][0];
    if (nh > 0) {
        sched.hub_slot_off = DBuf<int64_t>(c, (size_t)nh + 1);
        DBuf<int64_t> slots(c, (size_t)nh);
        hipLaunchKernelGGL(k_hub_slots, dim3(grid_for(nh)), dim3(kBlock), 0, c.stream, g.xadj,
                           sched.order.p + segoff[3][0], nh, slots.p);
        KMP_LAUNCH_CHECK();
        scan_incl_i64(c, slots.p, sched.hub_slot_off.p + 1, nh);
        c.zero(sched.hub_slot_off.p, sizeof(int64_t));
        sched.hub_slots_total = c.read1(sched.hub_slot_off.p + nh);
    }
}

namespace {

struct LPBuffers {
    DBuf<int32_t> prop;
    DBuf<uint8_t> acc;
    DBuf<uint32_t> demand;
    DBuf<uint32_t> hub_keys, hub_vals;
    DBuf<int32_t> moved_list;
};

void lp_buffers(Ctx& c, const DGraph& g, const LPSchedule& sched, int32_t nlab, LPBuffers& b)
{
    b.prop = DBuf<int32_t>(c, (size_t)g.n);
    fill_i32(c, b.prop.p, -1, g.n);
    b.acc = DBuf<uint8_t>(c, (size_t)g.n);
    c.zero(b.acc.p, (size_t)g.n);
    b.demand = DBuf<uint32_t>(c, (size_t)nlab);
    c.zero(b.demand.p, sizeof(uint32_t) * (size_t)nlab);
    if (sched.hub_slots_total > 0) {
        b.hub_keys = DBuf<uint32_t>(c, (size_t)sched.hub_slots_total);
        b.hub_vals = DBuf<uint32_t>(c, (size_t)sched.hub_slots_total);
    }
    b.moved_list = DBuf<int32_t>(c, (size_t)g.n);
}

void launch_rate(Ctx& c, RateArgs a, const LPSchedule& sched, int32_t s, uint32_t* hub_keys, uint32_t* hub_vals)
{
    const int32_t* order = sched.order.p;
    int32_t cnt[4];
    for (int t = 0; t < 4; ++t) cnt[t] = sched.cnt[s][t];
    a.hub_keys = hub_keys;
    a.hub_vals = hub_vals;
    int64_t* bytes = c.counters() + kBytesSlot;
    if (cnt[0] > 0) {
        constexpr int G = 8, GPB = kBlock / G;
        ProfScope ps(c, KMP_PROF_RATE_T0);
        a.bytes_ctr = bytes + KMP_PROF_RATE_T0;
        hipLaunchKernelGGL((k_rate_lds<G, 5>), dim3(grid_for(cnt[0], GPB, 65536)), dim3(kBlock), 0, c.stream, a,
                           order + sched.off[s][0], cnt[0]);
        KMP_LAUNCH_CHECK();
    }
    if (cnt[1] > 0) {
        constexpr int G = 64, GPB = kBlock / G;
        ProfScope ps(c, KMP_PROF_RATE_T1);
        a.bytes_ctr = bytes + KMP_PROF_RATE_T1;
        hipLaunchKernelGGL((k_rate_lds<G, 8>), dim3(grid_for(cnt[1], GPB, 65536)), dim3(kBlock), 0, c.stream, a,
                           order + sched.off[s][1], cnt[1]);
        KMP_LAUNCH_CHECK();
    }
    if (cnt[2] > 0) {
        ProfScope ps(c, KMP_PROF_RATE_T2);
        a.bytes_ctr = bytes + KMP_PROF_RATE_T2;
        hipLaunchKernelGGL((k_rate_lds<256, 12>), dim3(grid_for(cnt[2], 1, 65536)), dim3(kBlock), 0, c.stream, a,
                           order + sched.off[s][2], cnt[2]);
        KMP_LAUNCH_CHECK();
    }
    if (cnt[3] > 0) {
        // hub tables are indexed by position in the hub range (all classes contiguous)
        a.hub_off = sched.hub_slot_off.p + (sched.off[s][3] - sched.hub_start);
        ProfScope ps(c, KMP_PROF_RATE_HUB);
        a.bytes_ctr = bytes + KMP_PROF_RATE_HUB;
        hipLaunchKernelGGL(k_rate_hub, dim3(grid_for(cnt[3], 1, 4096)), dim3(kBlock), 0, c.stream, a,
                           order + sched.off[s][3], cnt[3]);
        KMP_LAUNCH_CHECK();
    }
}

// Returns moves of this sub-round; appends moved ids after `moved_base`.
int64_t subround_impl(Ctx& c, const DGraph& g, int32_t level, int32_t round, int32_t s, uint64_t seed,
                      const LPSchedule& sched, LPState& st, const uint8_t* active, uint8_t* moved, LPBuffers& b,
                      int64_t moved_base)
{
    int64_t* ctr = c.counters();
    // counters[1] contended count; counters[2] = moved-list cursor
    c.zero(ctr + 1, sizeof(int64_t));
    set_i64(c, ctr + 2, moved_base);
    RateArgs a;
    a.xadj = g.xadj;
    a.adjncy = g.adjncy;
    a.vwgt = g.vwgt;
    a.adjwgt = g.adjwgt;
    a.label = st.label;
    a.wt = st.wt;
    a.cap_vec = st.cap_vec;
    a.cap_scalar = st.cap_scalar;
    a.active = active;
    a.hpre = hash_prefix(seed, {st.tag, (uint32_t)level, (uint32_t)round});
    a.prop = b.prop.p;
    a.fav = st.fav;
    a.demand = b.demand.p;
    a.counters = ctr;
    a.hub_off = nullptr;
    a.over = nullptr;
    a.bal_t = nullptr;
    a.bal_d = nullptr;

    const int32_t* order = sched.order.p;
    int32_t cnt[4];
    for (int t = 0; t < 4; ++t) cnt[t] = sched.cnt[s][t];
    launch_rate(c, a, sched, s, b.hub_keys.p, b.hub_vals.p);
    Seg4 seg;
    int64_t total = 0;
    for (int t = 0; t < 4; ++t) {
        seg.off[t] = sched.off[s][t];
        seg.cnt[t] = cnt[t];
        total += cnt[t];
    }
    if (total == 0) return 0;
    {
        ProfScope ps(c, KMP_PROF_ADMIT);
        hipLaunchKernelGGL(k_admit_fast, dim3(grid_for(total)), dim3(kBlock), 0, c.stream, seg, total, order, b.prop.p,
                           b.demand.p, st.wt, st.cap_vec, st.cap_scalar, b.acc.p, ctr);
        KMP_LAUNCH_CHECK();
    }
    int64_t ncont = c.read1(ctr + 1);
    if (ncont > 0) {
        const int32_t n = g.n;
        DBuf<int32_t> flag(c, (size_t)n + 1);
        hipLaunchKernelGGL(k_contended_flags, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, b.acc.p, n, flag.p);
        KMP_LAUNCH_CHECK();
        scan_excl_i32(c, flag.p, flag.p, n, nullptr);
        DBuf<uint32_t> keys(c, ncont), vals(c, ncont), keys2(c, ncont), vals2(c, ncont);
        hipLaunchKernelGGL(k_contended_compact, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, b.acc.p, flag.p, n,
                           b.prop.p, keys.p, vals.p);
        KMP_LAUNCH_CHECK();
        radix_sort_pairs(c, keys.p, vals.p, keys2.p, vals2.p, ncont, bits_for((uint64_t)(st.nlab - 1)));
        DBuf<int64_t> pre(c, ncont), base(c, (size_t)st.nlab);
        hipLaunchKernelGGL(k_gather_cw, dim3(grid_for(ncont)), dim3(kBlock), 0, c.stream, vals.p, ncont, g.vwgt,
                           pre.p);
        KMP_LAUNCH_CHECK();
        scan_incl_i64(c, pre.p, pre.p, ncont);
        hipLaunchKernelGGL(k_heads, dim3(grid_for(ncont)), dim3(kBlock), 0, c.stream, keys.p, pre.p, vals.p, g.vwgt,
                           ncont, base.p);
        KMP_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_decide, dim3(grid_for(ncont)), dim3(kBlock), 0, c.stream, keys.p, vals.p, pre.p, base.p,
                           ncont, st.wt, st.cap_vec, st.cap_scalar, b.acc.p);
        KMP_LAUNCH_CHECK();
    }
    {
        ProfScope ps(c, KMP_PROF_APPLY);
        hipLaunchKernelGGL(k_apply, dim3(grid_for(total)), dim3(kBlock), 0, c.stream, seg, total, order, b.prop.p,
                           b.acc.p, b.demand.p, st.label, st.wt, g.vwgt, moved, b.moved_list.p, ctr);
        KMP_LAUNCH_CHECK();
    }
    int64_t cursor = c.read1(ctr + 2);
    return cursor - moved_base;
}

}  // namespace

void rate_for_balance(Ctx& c, const DGraph& g, int32_t level, uint64_t seed, int32_t round,
                      const LPSchedule& sched, const int32_t* part, const int64_t* wt, const int64_t* cap,
                      const uint8_t* over, int32_t* bal_t, int64_t* bal_d)
{
    if (g.n == 0) return;
    RateArgs a;
    memset(&a, 0, sizeof(a));
    a.xadj = g.xadj;
    a.adjncy = g.adjncy;
    a.vwgt = g.vwgt;
    a.adjwgt = g.adjwgt;
    a.label = part;
    a.wt = wt;
    a.cap_vec = cap;
    a.hpre = hash_prefix(seed, {TAG_BAL, (uint32_t)level, (uint32_t)round});
    a.counters = c.counters() + 10;  // statistic slot not reported for balancing
    a.over = over;
    a.bal_t = bal_t;
    a.bal_d = bal_d;
    DBuf<uint32_t> hk, hv;
    if (sched.hub_slots_total > 0) {
        hk = DBuf<uint32_t>(c, (size_t)sched.hub_slots_total);
        hv = DBuf<uint32_t>(c, (size_t)sched.hub_slots_total);
    }
    for (int32_t s = 0; s < kSub; ++s) launch_rate(c, a, sched, s, hk.p, hv.p);
}

LPStats lp_run(Ctx& c, const DGraph& g, int32_t level, uint64_t seed, const LPSchedule& sched, LPState& st)
{
    LPStats out;
    if (g.n == 0) return out;
    LPBuffers b;
    lp_buffers(c, g, sched, st.nlab, b);
    DBuf<uint8_t> active(c, (size_t)g.n);
    int64_t* ctr = c.counters();
    c.zero(ctr, sizeof(int64_t));  // rated edges
    for (int32_t r = 0; r < kRounds; ++r) {
        out.rounds = r + 1;
        int64_t nm = 0;
        for (int32_t s = 0; s < kSub; ++s)
            nm += subround_impl(c, g, level, r, s, seed, sched, st, r == 0 ? nullptr : active.p, nullptr, b, nm);
        out.moves[r] = nm;
        if (nm == 0) break;
        if (r + 1 < kRounds) {
            c.zero(active.p, (size_t)g.n);
            ProfScope ps(c, KMP_PROF_ACTIVE);
            hipLaunchKernelGGL(k_push_active, dim3(grid_for(nm * 64, kBlock, 8192)), dim3(kBlock), 0, c.stream,
                               b.moved_list.p, nm, g.xadj, g.adjncy, active.p);
            KMP_LAUNCH_CHECK();
        }
    }
    out.rated_edges = c.read1(ctr);
    return out;
}

int64_t lp_subround(Ctx& c, const DGraph& g, int32_t level, int32_t round, int32_t s, uint64_t seed,
                    const LPSchedule& sched, LPState& st, const uint8_t* active, uint8_t* moved)
{
    if (g.n == 0) return 0;
    LPBuffers b;
    lp_buffers(c, g, sched, st.nlab, b);
    return subround_impl(c, g, level, round, s, seed, sched, st, active, moved, b, 0);
}

}  // namespace kmp
