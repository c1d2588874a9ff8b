// Initial bipartitioning during uncoarsening (paper Alg. 2 "bipartitionBlocks",
// Sec. 4 "Handling General k", Sec. 5.2), projection (Alg. 1) and block
// statistics.
//
// Every block with final count f >= 2 is split by greedy graph growing (GGG,
// Sec. 5.2): one workgroup per block builds the block's induced subgraph in
// local ids (rank of the node id inside the block) and runs R = 8 growths,
// one per wavefront; the growth with the lexicographically smallest
// (infeasible?, overload, cut, seed index) is kept.  Growth j adds, while the
// grown side weighs less than floor(c(B) f0 / f), the frontier node with the
// largest gain (smallest local id on ties) that fits under f0 * L_k, or, when
// no frontier node fits, the fitting unassigned node with the smallest hash
// H(seed; 5, level, first, f, j, local id).  A growth step is one pass over a
// packed 64-bit key per node (frontier flag, gain, id) and one wave maximum.
#include <cmath>
#include <memory>
#include <mutex>

#include "kmp_dev.h"

namespace kmp {

namespace {

// ---------------------------------------------------------------- extraction
// Privatised in LDS when the block count is small (heavy contention otherwise).
constexpr int kPrivBlocks = 2048;

__global__ __launch_bounds__(kBlock) void k_block_count(const int32_t* __restrict__ part,
                                                        const int32_t* __restrict__ xadj, int32_t n, int32_t nb,
                                                        int32_t* __restrict__ bcnt, int32_t* __restrict__ bdeg,
                                                        uint32_t* __restrict__ key, uint32_t* __restrict__ val)
{
    __shared__ int32_t hc[kPrivBlocks], hd[kPrivBlocks];
    const bool priv = nb <= kPrivBlocks;
    if (priv)
        for (int i = threadIdx.x; i < nb; i += kBlock) hc[i] = hd[i] = 0;
    __syncthreads();
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int32_t b = part[v];
        int32_t d = xadj[v + 1] - xadj[v];
        if (priv) {
            atomicAdd(&hc[b], 1);
            atomicAdd(&hd[b], d);
        } else {
            atomicAdd(&bcnt[b], 1);
            atomicAdd(&bdeg[b], d);
        }
        key[v] = (uint32_t)b;
        val[v] = (uint32_t)v;
    }
    __syncthreads();
    if (priv)
        for (int i = threadIdx.x; i < nb; i += kBlock)
            if (hc[i]) {
                atomicAdd(&bcnt[i], hc[i]);
                atomicAdd(&bdeg[i], hd[i]);
            }
}

__global__ void k_local_ids(const uint32_t* __restrict__ verts, const int32_t* __restrict__ part,
                            const int32_t* __restrict__ bstart, int32_t n, int32_t* __restrict__ local)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t v = (int32_t)verts[i];
    local[v] = (int32_t)i - bstart[part[v]];
}

// Extraction over the whole device (levels whose blocks have long rows): the
// internal entries (neighbour in the same block) of the vertices of the blocks
// to split, in block order (position p of the block-sorted vertices), are
// counted, numbered by an exclusive scan over the positions, and written as
// (local neighbour, weight) in row order.  A row of at most kExtLight entries
// is walked by one thread; a longer one is cut into chunks of kExtChunk
// entries, one wavefront each, whose counts are scanned as well so that each
// chunk knows where its entries start within the row.  The greedy growing then
// reads each block's internal rows instead of walking its full rows in one
// workgroup.
constexpr int32_t kExtChunk = 1024;
constexpr int32_t kExtLight = 64;

struct ExtArgs {
    const uint32_t* verts;
    const int32_t* part;
    const int32_t* xadj;
    const int32_t* adjncy;
    const int32_t* adjwgt;
    const int32_t* local;
    const uint8_t* split;  // [blocks] the block is split at this level
    int32_t n;
    int32_t* nch;          // [n] chunks of a long row (0 for short rows and other blocks)
    const int32_t* cplan;  // [n + 1] first chunk of each position; cplan[n] = chunks
    const int32_t* crow;   // [chunks] position of each chunk
    int32_t* pc;           // [n] internal entries per position (count pass; zero before)
    int32_t* ccnt;         // [chunks] internal entries per chunk (count pass)
    const int32_t* ioff;   // [n + 1] exclusive prefix of pc (write pass)
    const int32_t* cpre;   // [chunks + 1] exclusive prefix of ccnt (write pass)
    int32_t* iw;           // [n] weighted internal degree per position (count pass; zero before)
    int32_t* bint;         // [blocks] internal entries per block (count pass; zero before)
    int2* ied;             // internal entries (write pass)
};

// chunks per position of a long row in a block to split
__global__ void k_ext_plan(ExtArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const int32_t v = (int32_t)a.verts[p];
    const int32_t d = a.xadj[v + 1] - a.xadj[v];
    a.nch[p] = a.split[a.part[v]] && d > kExtLight ? (d + kExtChunk - 1) / kExtChunk : 0;
}

// the position of every chunk: crow[c] = p for the chunks c of position p
__global__ void k_ext_rows(const int32_t* __restrict__ cplan, int32_t n, int32_t* __restrict__ crow)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    for (int32_t c = cplan[p]; c < cplan[p + 1]; ++c) crow[c] = (int32_t)p;
}

// Short rows, one thread each (eight entries in flight): WRITE = false counts,
// true writes at ioff[p] in row order.
template <bool WRITE>
__global__ void k_ext_light(ExtArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const int32_t v = (int32_t)a.verts[p];
    const int32_t b = a.part[v];
    const int32_t r0 = a.xadj[v], r1 = a.xadj[v + 1];
    if (!a.split[b] || r1 - r0 > kExtLight || r1 == r0) return;
    int32_t cnt = 0, ws = 0;
    int32_t pos = WRITE ? a.ioff[p] : 0;
    for (int32_t e0 = r0; e0 < r1; e0 += 8) {
        int32_t u[8], pu[8], wq[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) u[q] = a.adjncy[e0 + q < r1 ? e0 + q : r1 - 1];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            pu[q] = a.part[u[q]];
            wq[q] = a.adjwgt ? a.adjwgt[e0 + q < r1 ? e0 + q : r1 - 1] : 1;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (e0 + q >= r1 || pu[q] != b) continue;
            if (WRITE) a.ied[pos++] = make_int2(a.local[u[q]], wq[q]);
            ++cnt;
            ws += wq[q];
        }
    }
    if (!WRITE) {
        a.pc[p] = cnt;
        a.iw[p] = ws;
        if (cnt) atomicAdd(&a.bint[b], cnt);
    }
}

// Long rows, one wavefront per chunk: WRITE = false counts, true writes in row
// order from ioff[p] + (entries of the row's earlier chunks).
template <bool WRITE>
__global__ __launch_bounds__(kBlock) void k_ext_chunks(ExtArgs a)
{
    const int lane = threadIdx.x & 63;
    const int32_t total = a.cplan[a.n];
    for (int64_t ch = (int64_t)blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); ch < total;
         ch += (int64_t)gridDim.x * (kBlock / 64)) {
        const int32_t p = a.crow[ch];
        const int32_t v = (int32_t)a.verts[p];
        const int32_t b = a.part[v];
        const int32_t r0 = a.xadj[v], r1 = a.xadj[v + 1];
        const int32_t c0 = r0 + ((int32_t)ch - a.cplan[p]) * kExtChunk;
        const int32_t c1 = c0 + kExtChunk < r1 ? c0 + kExtChunk : r1;
        int32_t cnt = 0, ws = 0;
        int32_t pos = WRITE ? a.ioff[p] + a.cpre[ch] - a.cpre[a.cplan[p]] : 0;
        constexpr int U = kExtChunk / 64;  // the whole chunk in flight
        // every load unconditional (indices clamped into the chunk), so all are in flight
        int32_t u[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int32_t e = c0 + q * 64 + lane;
            u[q] = a.adjncy[e < c1 ? e : c1 - 1];
        }
        int32_t pu[U], wq[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const int32_t e = c0 + q * 64 + lane;
            pu[q] = a.part[u[q]];
            wq[q] = a.adjwgt ? a.adjwgt[e < c1 ? e : c1 - 1] : 1;
        }
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const bool in = c0 + q * 64 + lane < c1 && pu[q] == b;
            const int32_t w = in ? wq[q] : 0;
            if (WRITE) {
                const uint64_t m = __ballot(in);
                if (in) a.ied[pos + __popcll(m & ((1ull << lane) - 1))] = make_int2(a.local[u[q]], w);
                pos += __popcll(m);
            } else {
                cnt += in ? 1 : 0;
                ws += w;
            }
        }
        if (!WRITE) {
            for (int dd = 32; dd > 0; dd >>= 1) {
                cnt += __shfl_xor(cnt, dd, 64);
                ws += __shfl_xor(ws, dd, 64);
            }
            if (lane == 0) {
                a.ccnt[ch] = cnt;
                if (cnt) {
                    atomicAdd(&a.pc[p], cnt);
                    atomicAdd(&a.bint[b], cnt);
                }
                if (ws) atomicAdd(&a.iw[p], ws);
            }
        }
    }
}

// ---------------------------------------------------------------- GGG
constexpr int GGG_THREADS = 64 * kSeeds;

struct GGGJob {
    int32_t b, first, f, nverts;
    int32_t dsum;      // sum of degrees of the block's nodes (bound on internal entries)
    uint32_t hpre;     // H prefix over (seed; T_GGG, level) of the block's job
    uint32_t hpre_bfs; // the same over (seed; T_BFS, level) and (seed; T_RND, level)
    uint32_t hpre_rnd;
    int64_t scratch;   // byte offset into the global scratch (global and hybrid variants)
    int64_t sstride;   // the scratch of one workgroup (pool families in parallel: one each)
    int64_t soff;      // pool families in parallel: offset of the job's sides, one nverts run per family
    int64_t lk;        // L_k of the block's job
    int64_t cap0, cap1;  // bounds of the two sides (f_j L_k, or the adaptive imbalance's)
};

struct GGGArgs {
    const int32_t* xadj;
    const int32_t* adjncy;
    const int32_t* vwgt;
    const int32_t* adjwgt;
    const int32_t* part;
    const uint32_t* verts;
    const int32_t* bstart;
    const int32_t* local;
    const GGGJob* jobs;
    uint8_t* side;      // [n]
    char* scratch;      // global variant
    int32_t fm_passes;  // 2-way FM passes after each growth (0: none)
    int32_t pool;       // 1: BFS and random growths besides the GGG ones
    const uint8_t* given;  // non-NULL: no growth; FM refines these sides (by vertex) into `side`
    // set by launch_ggg_jobs: algs = 3 runs the pool's three families side by side, one
    // workgroup each (workgroup 3 j + family); every workgroup writes its best run's
    // sides (by local id) to side_alg and its (overload, cut) to res, and k_ggg_pick
    // keeps the first strictly best family in the order GGG, BFS, random
    int32_t algs;
    uint8_t* side_alg;
    int64_t* res;  // [job][family][2]
    // the block's internal rows from the extraction over the whole device (NULL: the
    // workgroup extracts them itself): by position of the block-sorted vertices, the
    // first internal entry ioff[p] (ioff[n] = all), the weighted internal degree iw[p],
    // and the entries ied (local neighbour, weight)
    const int32_t* ioff = nullptr;
    const int32_t* iw = nullptr;
    const int2* ied = nullptr;
};

// A growth keeps one 64-bit key per node, so that finding the next node is one
// load per node and a maximum:
//   bit 63      node is on the frontier (adjacent to the grown side)
//   bits 62-31  gain + 2^31 (gain = weight to the grown side - weight to the rest)
//   bits 30-0   2^31 - 1 - local id (ties go to the smaller id)
// Key 0 marks a grown node (and the padding up to a multiple of 64 nodes);
// key 1 a node that no longer fits under the cap (the grown weight only
// increases, so it never fits again and its gain no longer matters).
constexpr uint64_t kFront = 1ull << 63;
constexpr uint64_t kUnfit = 1;

__device__ inline uint64_t ggg_key(int32_t gain, uint32_t i)
{
    return ((uint64_t)((uint32_t)gain ^ 0x80000000u) << 31) | (uint64_t)(0x7FFFFFFFu - i);
}
__device__ inline int32_t ggg_gain(uint64_t k) { return (int32_t)((uint32_t)(k >> 31) ^ 0x80000000u); }
__device__ inline int32_t ggg_id(uint64_t k) { return (int32_t)(0x7FFFFFFFu - (uint32_t)(k & 0x7FFFFFFFu)); }

__host__ __device__ inline int64_t ggg_pad(int64_t nv) { return (nv + 63) & ~(int64_t)63; }

__host__ __device__ inline int64_t ggg_bytes(int64_t nv, int64_t d, bool fm)
{
    // keys (R x padded nv) u64, entries (d) and nodes (nv + 1) as int32 pairs;
    // with FM also one int32 (side << 31 | node weight) per run and node
    // and one int32 per node for its internal weighted degree
    const int64_t bytes = 8 * ((int64_t)kSeeds * ggg_pad(nv) + d + nv + 1) + (fm ? 4 * (int64_t)kSeeds * ggg_pad(nv) : 0) +
                          4 * ggg_pad(nv);
    return (bytes + 15) & ~(int64_t)15;
}

// LDS of the hybrid layout (the entries live in the global scratch)
__host__ __device__ inline int64_t ggg_hybrid_lds(int64_t nv, bool fm) { return ggg_bytes(nv, 0, fm); }

constexpr int kFmStall = 64;  // an FM pass ends after this many moves without a better prefix

// Orders a wavefront's own earlier memory operations before its later ones.
// LDS operations of a wavefront complete in issue order, so the LDS variant
// needs only the compiler ordering; the global variant waits for its stores.
template <bool LDS>
__device__ inline void fence_wave()
{
    if (LDS)
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    else
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Key layouts of a growth: 64-bit as above, or 32-bit when the block has at
// most 2048 nodes and every node's weighted degree is below 2^19 (a gain lies
// within plus or minus the node's weighted degree): bit 31 frontier, bits
// 30-11 gain + 2^19, bits 10-0 2047 - local id.  Both order candidates the
// same way; 0 and 1 keep their meaning.
struct Key64 {
    using T = uint64_t;
    static constexpr T front = kFront, unfit = kUnfit;
    __device__ static T make(int32_t gain, uint32_t i) { return ggg_key(gain, i); }
    __device__ static int32_t gain(T k) { return ggg_gain(k); }
    __device__ static int32_t id(T k) { return ggg_id(k); }
    __device__ static T wave_max(T v) { return wave_max_u64_split(v); }
};
struct Key32 {
    using T = uint32_t;
    static constexpr T front = 1u << 31, unfit = 1u;
    __device__ static T make(int32_t gain, uint32_t i) { return ((uint32_t)(gain + (1 << 19)) << 11) | (2047u - i); }
    __device__ static int32_t gain(T k) { return (int32_t)((k >> 11) & 0xFFFFFu) - (1 << 19); }
    __device__ static int32_t id(T k) { return (int32_t)(2047u - (k & 2047u)); }
    __device__ static T wave_max(T v) { return wave_max_u32_dpp(v); }
};

__device__ inline int64_t fm_over(int64_t w0, int64_t w1, int64_t cap0, int64_t cap1)
{
    return (w0 > cap0 ? w0 - cap0 : 0) + (w1 > cap1 ? w1 - cap1 : 0);
}

__device__ inline int32_t fm_room(int64_t d) { return d < 0 ? -1 : (d > INT32_MAX ? INT32_MAX : (int32_t)d); }

// 2-way FM (Fiduccia-Mattheyses) on one growth's bipartition, in its own
// wavefront.  sw[i] holds side << 31 | node weight.  In a pass, an unlocked
// node's key is front | (gain, id) with gain = weight to the other side minus
// weight to its own side; a moved node is locked with key 2 + its move index,
// so the undo after the pass needs no log.  Each step moves the unlocked node
// of largest key whose target side still has room for it; the pass ends when
// none fits or after kFmStall moves without a better prefix (less overload,
// else more total gain) and goes back to its best prefix.  Passes repeat
// until one keeps no move.  w0 (side 0's weight) is updated.
template <class KT, bool LDS>
__device__ inline void ggg_fm(typename KT::T* key, int32_t* sw, int32_t nvp, int32_t nv, const int2* nd,
                              const int2* ed, int lane, int64_t& w0, int64_t cB, int64_t cap0, int64_t cap1,
                              int passes)
{
    using T = typename KT::T;
    constexpr int32_t kSide = (int32_t)0x80000000u;
    for (int32_t i = lane; i < nvp; i += 64) sw[i] = i < nv ? ((key[i] != 0 ? kSide : 0) | nd[i].y) : 0;
    fence_wave<LDS>();
    const int32_t nchunks = nvp / 64;
    for (int p = 0; p < passes; ++p) {
        for (int32_t i = lane; i < nvp; i += 64) {
            T k = 0;
            if (i < nv) {
                const int32_t si = sw[i];
                int32_t g = 0;
                for (int32_t e = nd[i].x; e < nd[i + 1].x; ++e) {
                    const int2 uw = ed[e];
                    g += (sw[uw.x] ^ si) < 0 ? uw.y : -uw.y;
                }
                k = KT::front | KT::make(g, (uint32_t)i);
            }
            key[i] = k;
        }
        fence_wave<LDS>();
        int64_t W0 = w0, W1 = cB - w0;
        int64_t G = 0, bestG = 0, bestOver = fm_over(W0, W1, cap0, cap1), bestW0 = W0;
        int32_t t = 0, bestT = 0, since = 0;
        for (;;) {
            // a side-0 node needs room on side 1 and the other way round
            const int32_t r0 = fm_room(cap0 - W0), r1 = fm_room(cap1 - W1);
            T best = 0;
            for (int32_t c0 = 0; c0 < nchunks; c0 += 8) {
                T k[8];
                int32_t sv[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const bool in = c0 + q < nchunks;
                    k[q] = in ? key[(c0 + q) * 64 + lane] : 0;
                    sv[q] = in ? sw[(c0 + q) * 64 + lane] : 0;
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int32_t room = sv[q] < 0 ? r0 : r1;
                    const T cand = k[q] >= KT::front && (sv[q] & 0x7FFFFFFF) <= room ? k[q] : 0;
                    best = cand > best ? cand : best;
                }
            }
            best = KT::wave_max(best);
            if (best < KT::front) break;
            const int32_t pick = KT::id(best);
            const int32_t sp = sw[pick];
            const int2 pa = nd[pick], pb = nd[pick + 1];
            const int32_t spn = sp ^ kSide;  // pick's side after the move
            const int64_t c = sp & 0x7FFFFFFF;
            if (sp < 0) {
                W1 -= c;
                W0 += c;
            } else {
                W0 -= c;
                W1 += c;
            }
            G += KT::gain(best);
            fence_wave<LDS>();  // every lane has read sw[pick] before it changes
            if (lane == 0) {
                key[pick] = (T)(2 + t);
                sw[pick] = spn;
            }
            ++t;
            fence_wave<LDS>();
            for (int32_t e = pa.x + lane; e < pb.x; e += 64) {
                const int2 uw = ed[e];
                asm volatile("" ::"v"(uw.x), "v"(uw.y));  // one load for both halves
                const T k = key[uw.x];
                if (k >= KT::front) {
                    // a neighbour now on pick's side loses the edge from its gain, one across gains it
                    // in 64 bits: one edge may weigh more than 2^30; the new gain (within the
                    // node's weighted degree, at most 2^31 - 1) fits 32 bits again
                    const int64_t d = (sw[uw.x] ^ spn) >= 0 ? -2 * (int64_t)uw.y : 2 * (int64_t)uw.y;
                    key[uw.x] = KT::front | KT::make((int32_t)((int64_t)KT::gain(k) + d), (uint32_t)uw.x);
                }
            }
            fence_wave<LDS>();
            const int64_t ov = fm_over(W0, W1, cap0, cap1);
            if (ov < bestOver || (ov == bestOver && G > bestG)) {
                bestOver = ov;
                bestG = G;
                bestT = t;
                bestW0 = W0;
                since = 0;
            } else if (++since >= kFmStall) {
                break;
            }
        }
        // undo the moves after the best prefix
        for (int32_t i = lane; i < nv; i += 64) {
            const T k = key[i];
            if (k < KT::front && k >= (T)(2 + bestT)) sw[i] ^= kSide;
        }
        w0 = bestW0;
        fence_wave<LDS>();
        if (bestT == 0) break;
    }
}

// Growth algorithms of the initial-bipartitioning pool.  All three grow block
// 0 to the same target under the same cap with the same key machinery and
// differ in the key: GGG the cut gain, BFS minus the discovery index (a node
// is discovered, in adjacency order, when a neighbour joins block 0), random
// the inverted hash of the node (64-bit keys only).
enum { ALG_GGG = 0, ALG_BFS = 1, ALG_RND = 2 };

// One growth in one wavefront (seed j); lane 0 leaves the cut and the overload.
template <class KT, bool LDS, int ALG>
__device__ inline void ggg_grow(void* key_base, int32_t nvp, int32_t nv, const int2* nd, const int2* ed,
                                const int32_t* wdeg, int j, int lane, uint32_t hj, int64_t cB, int64_t t0,
                                int64_t cap0, int64_t cap1, int64_t* s_cut, int64_t* s_over, int32_t* sw_base,
                                int fm_passes)
{
    using T = typename KT::T;
    static_assert(ALG != ALG_RND || sizeof(T) == 8, "random growth keys hold a 32-bit hash");
    T* key = reinterpret_cast<T*>(key_base) + (int64_t)j * nvp;
    for (int32_t i = lane; i < nvp; i += 64) {
        T k = 0;
        if (i < nv) {
            if constexpr (ALG == ALG_GGG) {
                k = KT::make(-wdeg[i], (uint32_t)i);  // gain = weight to the grown side - weight to the rest
            } else if constexpr (ALG == ALG_BFS) {
                k = KT::make(0, (uint32_t)i);  // undiscovered
            } else {
                // the gain field holds ~hash: the largest key is the smallest hash
                const uint32_t h = hash_step(hj, (uint32_t)i, 6);
                k = KT::front | KT::make((int32_t)(~h ^ 0x80000000u), (uint32_t)i);
            }
        }
        key[i] = k;
    }
    uint32_t disc = 0;  // BFS: nodes discovered so far
    fence_wave<LDS>();
    int64_t w0 = 0;
    // GGG keeps every unassigned node's gain in its key, and adding node v to
    // the grown side changes the cut by -gain(v): the cut is summed on the way
    int64_t gcut = 0;
    const int32_t nchunks = nvp / 64;
    while (w0 < t0) {
        // the largest key: lane l reads nodes l, l + 64, ... (8 loads in flight)
        T best = 0;
        for (int32_t c0 = 0; c0 < nchunks; c0 += 8) {
            T k[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) k[q] = c0 + q < nchunks ? key[(c0 + q) * 64 + lane] : 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) best = k[q] > best ? k[q] : best;
        }
        // each lane fetches its own candidate's row and weight while the maximum is
        // reduced; the winner (node i lives in lane i mod 64) hands them over
        int2 ca = make_int2(0, 0), cb = make_int2(0, 0);
        if (best >= KT::front) {
            const int32_t ci = KT::id(best);
            ca = nd[ci];
            cb = nd[ci + 1];
        }
        best = KT::wave_max(best);
        int32_t pick;
        int32_t pw, pe0, pe1;
        int32_t pgain = 0;  // GGG: the pick's gain
        if (best >= KT::front) {
            pick = KT::id(best);
            const int src = pick & 63;
            pw = __builtin_amdgcn_readlane(ca.y, src);
            pe0 = __builtin_amdgcn_readlane(ca.x, src);
            pe1 = __builtin_amdgcn_readlane(cb.x, src);
            if constexpr (ALG == ALG_GGG) pgain = KT::gain(best);
        } else {
            // no frontier node fits: the fitting unassigned node of smallest hash
            uint64_t hb = ~0ull;  // (hash << 32) | id ; max = none
            for (int32_t i = lane; i < nv; i += 64) {
                if (key[i] == 0 || w0 + nd[i].y > cap0) continue;
                const uint64_t k = ((uint64_t)hash_step(hj, (uint32_t)i, 6) << 32) | (uint32_t)i;
                if (k < hb) hb = k;
            }
            hb = ~wave_max_u64_split(~hb);
            if (hb == ~0ull) break;
            pick = (int32_t)(hb & 0xFFFFFFFFu);
            const int2 pa = nd[pick], pb = nd[pick + 1];
            pw = pa.y;
            pe0 = pa.x;
            pe1 = pb.x;
            if constexpr (ALG == ALG_GGG) pgain = KT::gain(key[pick]);
        }
        if (w0 + pw > cap0) {
            // a frontier node that does not fit: drop it for the rest of the growth
            if (lane == 0) key[pick] = KT::unfit;
            fence_wave<LDS>();
            continue;
        }
        if (lane == 0) key[pick] = 0;
        w0 += pw;
        gcut -= pgain;
        fence_wave<LDS>();
        if constexpr (ALG == ALG_GGG) {
            for (int32_t e = pe0 + lane; e < pe1; e += 64) {
                const int2 uw = ed[e];
                asm volatile("" ::"v"(uw.x), "v"(uw.y));  // one load for both halves
                const T k = key[uw.x];
                if (k > KT::unfit)
                    key[uw.x] =
                        KT::front | KT::make((int32_t)((int64_t)KT::gain(k) + 2 * (int64_t)uw.y), (uint32_t)uw.x);
            }
        } else if constexpr (ALG == ALG_BFS) {
            // undiscovered neighbours get the next discovery indices in adjacency order
            for (int32_t e0 = pe0; e0 < pe1; e0 += 64) {
                const int32_t e = e0 + lane;
                const bool in = e < pe1;
                const int32_t u = in ? ed[e].x : 0;
                const T k = in ? key[u] : 0;
                const bool nw = in && k > KT::unfit && k < KT::front;
                const uint64_t m = __ballot(nw);
                if (nw) {
                    const uint32_t idx = disc + (uint32_t)__popcll(m & ((1ull << lane) - 1));
                    key[u] = KT::front | KT::make(-(int32_t)idx, (uint32_t)u);
                }
                disc += (uint32_t)__popcll(m);
            }
        }
        fence_wave<LDS>();
    }
    int64_t cut = 0;
    if (fm_passes > 0) {
        int32_t* sw = sw_base + (int64_t)j * nvp;
        ggg_fm<KT, LDS>(key, sw, nvp, nv, nd, ed, lane, w0, cB, cap0, cap1, fm_passes);
        for (int32_t i = lane; i < nv; i += 64) {
            if (sw[i] < 0) continue;
            for (int32_t e = nd[i].x; e < nd[i + 1].x; ++e)
                if (sw[ed[e].x] < 0) cut += ed[e].y;
        }
    } else if constexpr (ALG != ALG_GGG) {
        for (int32_t i = lane; i < nv; i += 64) {
            if (key[i] != 0) continue;
            for (int32_t e = nd[i].x; e < nd[i + 1].x; ++e)
                if (key[ed[e].x] != 0) cut += ed[e].y;
        }
    }
    for (int d = 32; d > 0; d >>= 1) cut += __shfl_xor(cut, d, 64);
    if constexpr (ALG == ALG_GGG)
        if (fm_passes == 0) cut = gcut;
    if (lane == 0) {
        s_cut[j] = cut;
        s_over[j] = (w0 > cap0 ? w0 - cap0 : 0) + (cB - w0 > cap1 ? cB - w0 - cap1 : 0);
    }
}

// Where a block's working set lives: every array in LDS, or keys, node rows
// and FM sides in LDS with the local adjacency in the global scratch (blocks
// of many internal entries: the growth reads only the winner's row there), or
// everything in the global scratch (blocks too large for either).
enum { GGG_GLOBAL = 0, GGG_LDS = 1, GGG_HYBRID = 2 };
constexpr int32_t kGggLightRow = 32;  // rows walked by one thread while a block is extracted

template <int MODE>
__global__ __launch_bounds__(GGG_THREADS) void k_ggg(GGGArgs a)
{
    constexpr bool LDS = MODE != GGG_GLOBAL;  // keys and sides in LDS
    extern __shared__ __align__(16) char lds_raw[];
    __shared__ int64_t s_red[GGG_THREADS / 64];
    __shared__ int64_t s_cut[kSeeds], s_over[kSeeds];
    __shared__ int32_t s_best;
    __shared__ int64_t s_keep_over, s_keep_cut;  // the kept run so far
    __shared__ bool s_take;
    __shared__ int32_t s_wmax;
    __shared__ int32_t s_carry;
    __shared__ int32_t s_nheavy;

    const int32_t jobi = (int32_t)(blockIdx.x / (uint32_t)a.algs);
    const int alg_first = (int)(blockIdx.x % (uint32_t)a.algs);  // 0 unless the families run side by side
    const GGGJob job = a.jobs[jobi];
    const int32_t nv = job.nverts;
    const int32_t nvp = (int32_t)ggg_pad(nv);
    const int32_t b = job.b;
    const uint32_t* vlist = a.verts + a.bstart[b];
    // this workgroup's part of the global scratch (global and hybrid layouts)
    char* const wscratch = a.scratch ? a.scratch + job.scratch + alg_first * job.sstride : nullptr;
    char* base = LDS ? lds_raw : wscratch;
    // key[R][nvp]; ed[e] = (local neighbour, edge weight); nd[i] = (row start, node weight), nd[nv].x = entries
    uint64_t* key_all = reinterpret_cast<uint64_t*>(base);
    int2* ed = reinterpret_cast<int2*>(key_all + (int64_t)kSeeds * nvp);
    int2* nd = ed + job.dsum;
    if (MODE == GGG_HYBRID) {
        nd = reinterpret_cast<int2*>(key_all + (int64_t)kSeeds * nvp);
        ed = reinterpret_cast<int2*>(wscratch);
    }
    int32_t* sw_all = reinterpret_cast<int32_t*>(nd + nv + 1);  // FM sides, R x padded nv
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

    int32_t* wdeg = sw_all + (a.fm_passes > 0 ? (int64_t)kSeeds * nvp : 0);  // internal weighted degrees
    constexpr int kWaves = GGG_THREADS / 64;
    int64_t cB = 0;
    if (a.ied) {
        // ---- the block's internal rows from the extraction over the whole device
        const int32_t p0 = a.bstart[b];
        const int32_t eb = a.ioff[p0];
        int64_t cacc = 0;
        for (int32_t i = tid; i < nv; i += GGG_THREADS) {
            const int32_t v = (int32_t)vlist[i];
            const int32_t c = a.vwgt ? a.vwgt[v] : 1;
            nd[i] = make_int2(a.ioff[p0 + i] - eb, c);
            wdeg[i] = a.iw[p0 + i];
            cacc += c;
        }
        for (int d = 32; d > 0; d >>= 1) cacc += __shfl_xor(cacc, d, 64);
        if (lane == 0) s_red[wv] = cacc;
        const int32_t E = a.ioff[p0 + nv] - eb;
        if (tid == 0) nd[nv] = make_int2(E, 0);
        if (MODE == GGG_HYBRID) {
            ed = const_cast<int2*>(a.ied) + eb;  // read in place
        } else {
            for (int32_t e = tid; e < E; e += GGG_THREADS) ed[e] = a.ied[eb + e];
        }
        __syncthreads();
        for (int q = 0; q < GGG_THREADS / 64; ++q) cB += s_red[q];
    } else {
        // ---- internal degrees (in nd[i + 1].x), internal weighted degrees and node weights.  A row
        // of the level graph can hold 10^5 entries, most of them outside the block: rows of up to
        // kGggLightRow entries are walked by one thread each (loads in groups of 8), longer ones are
        // listed (in the key array, which the growths initialise later) and walked by a whole
        // wavefront each, four 64-entry chunks in flight
        int32_t* heavy = reinterpret_cast<int32_t*>(key_all);
        if (tid == 0) s_nheavy = 0;
        __syncthreads();
        int64_t cacc = 0;
        for (int32_t i = tid; i < nv; i += GGG_THREADS) {
            const int32_t v = (int32_t)vlist[i];
            const int32_t e1 = a.xadj[v + 1];
            const int32_t c = a.vwgt ? a.vwgt[v] : 1;
            nd[i].y = c;
            cacc += c;
            if (e1 - a.xadj[v] > kGggLightRow) {
                heavy[atomicAdd(&s_nheavy, 1)] = i;
                continue;
            }
            int32_t cnt = 0, ws = 0;
            for (int32_t e0 = a.xadj[v]; e0 < e1; e0 += 8) {
                int32_t u[8];
    #pragma unroll
                for (int q = 0; q < 8; ++q) u[q] = e0 + q < e1 ? a.adjncy[e0 + q] : -1;
    #pragma unroll
                for (int q = 0; q < 8; ++q)
                    if (u[q] >= 0 && a.part[u[q]] == b) {
                        ++cnt;
                        ws += a.adjwgt ? a.adjwgt[e0 + q] : 1;
                    }
            }
            nd[i + 1].x = cnt;
            wdeg[i] = ws;
        }
        __syncthreads();
        const int32_t nheavy = s_nheavy;
        for (int32_t h = wv; h < nheavy; h += kWaves) {
            const int32_t i = heavy[h];
            const int32_t v = (int32_t)vlist[i];
            const int32_t e0 = a.xadj[v], e1 = a.xadj[v + 1];
            uint32_t cnt = 0, ws = 0;
            for (int32_t base = e0; base < e1; base += 256) {
                int32_t u[4];
    #pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int32_t e = base + q * 64 + lane;
                    u[q] = e < e1 ? a.adjncy[e] : -1;
                }
    #pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int32_t e = base + q * 64 + lane;
                    if (u[q] >= 0 && a.part[u[q]] == b) {
                        ++cnt;
                        ws += a.adjwgt ? (uint32_t)a.adjwgt[e] : 1u;
                    }
                }
            }
            cnt = group_sum_u32<64>(cnt);
            ws = group_sum_u32<64>(ws);
            if (lane == 0) {
                nd[i + 1].x = (int32_t)cnt;
                wdeg[i] = (int32_t)ws;
            }
        }
        for (int d = 32; d > 0; d >>= 1) cacc += __shfl_xor(cacc, d, 64);
        if (lane == 0) s_red[wv] = cacc;
        if (tid == 0) {
            nd[0].x = 0;
            nd[nv].y = 0;
            s_carry = 0;
        }
        __syncthreads();
        for (int q = 0; q < GGG_THREADS / 64; ++q) cB += s_red[q];
        // ---- prefix sum of internal degrees (chunks of GGG_THREADS, carry in LDS)
        for (int32_t c0 = 0; c0 < nv; c0 += GGG_THREADS) {
            const int32_t i = c0 + tid;
            int32_t x = i < nv ? nd[i + 1].x : 0;
            // inclusive scan in the wave
            for (int d = 1; d < 64; d <<= 1) {
                int32_t y = __shfl_up(x, d, 64);
                if (lane >= d) x += y;
            }
            __syncthreads();
            if (lane == 63) s_red[wv] = x;
            __syncthreads();
            int32_t pre = s_carry;
            for (int q = 0; q < wv; ++q) pre += (int32_t)s_red[q];
            if (i < nv) nd[i + 1].x = pre + x;
            __syncthreads();
            if (tid == GGG_THREADS - 1) s_carry = pre + x;
            __syncthreads();
        }
        // ---- local adjacency (ascending node id => ascending local id): short rows by one thread
        // each, the listed long rows by a wavefront each (the internal entries of a chunk keep their
        // order: ballot, then the count of lower lanes)
        for (int32_t i = tid; i < nv; i += GGG_THREADS) {
            const int32_t v = (int32_t)vlist[i];
            const int32_t e1 = a.xadj[v + 1];
            if (e1 - a.xadj[v] > kGggLightRow) continue;
            int32_t pos = nd[i].x;
            for (int32_t e0 = a.xadj[v]; e0 < e1; e0 += 8) {
                int32_t u[8], p[8], lu[8], w[8];
    #pragma unroll
                for (int q = 0; q < 8; ++q) u[q] = e0 + q < e1 ? a.adjncy[e0 + q] : -1;
    #pragma unroll
                for (int q = 0; q < 8; ++q) {
                    p[q] = u[q] >= 0 ? a.part[u[q]] : -1;
                    lu[q] = u[q] >= 0 ? a.local[u[q]] : 0;
                    w[q] = u[q] >= 0 ? (a.adjwgt ? a.adjwgt[e0 + q] : 1) : 0;
                }
    #pragma unroll
                for (int q = 0; q < 8; ++q) {
                    if (p[q] != b) continue;
                    ed[pos] = make_int2(lu[q], w[q]);
                    ++pos;
                }
            }
        }
        for (int32_t h = wv; h < nheavy; h += kWaves) {
            const int32_t i = heavy[h];
            const int32_t v = (int32_t)vlist[i];
            const int32_t e0 = a.xadj[v], e1 = a.xadj[v + 1];
            int32_t pos = nd[i].x;
            for (int32_t base = e0; base < e1; base += 64) {
                const int32_t e = base + lane;
                const int32_t u = e < e1 ? a.adjncy[e] : -1;
                const bool in = u >= 0 && a.part[u] == b;
                int2 val = make_int2(0, 0);
                if (in) val = make_int2(a.local[u], a.adjwgt ? a.adjwgt[e] : 1);
                const uint64_t m = __ballot(in);
                if (in) ed[pos + __popcll(m & ((1ull << lane) - 1))] = val;
                pos += __popcll(m);
            }
        }
        __syncthreads();

    }
    // ---- the key width: 32 bits when every gain fits (largest weighted degree)
    if (tid == 0) s_wmax = 0;
    __syncthreads();
    {
        int32_t m = 0;
        for (int32_t i = tid; i < nv; i += GGG_THREADS) m = wdeg[i] > m ? wdeg[i] : m;
        if (m) atomicMax(&s_wmax, m);
    }
    __syncthreads();
    const bool k32 = nv <= 2048 && s_wmax < (1 << 19);

    if (a.given) {
        // refinement of a given bipartition (the finer levels of the multilevel
        // bipartitioning): wavefront 0 runs the FM passes on it
        if (wv != 0) return;
        int64_t w0 = 0;
        if (k32) {
            uint32_t* key = reinterpret_cast<uint32_t*>(key_all);
            for (int32_t i = lane; i < nvp; i += 64) {
                const uint32_t sd = i < nv ? a.given[vlist[i]] : 0u;
                key[i] = sd;
                if (i < nv && sd == 0) w0 += nd[i].y;
            }
        } else {
            for (int32_t i = lane; i < nvp; i += 64) {
                const uint64_t sd = i < nv ? a.given[vlist[i]] : 0u;
                key_all[i] = sd;
                if (i < nv && sd == 0) w0 += nd[i].y;
            }
        }
        for (int d = 32; d > 0; d >>= 1) w0 += __shfl_xor(w0, d, 64);
        fence_wave<LDS>();
        if (k32)
            ggg_fm<Key32, LDS>(reinterpret_cast<uint32_t*>(key_all), sw_all, nvp, nv, nd, ed, lane, w0, cB, job.cap0,
                               job.cap1, a.fm_passes);
        else
            ggg_fm<Key64, LDS>(key_all, sw_all, nvp, nv, nd, ed, lane, w0, cB, job.cap0, job.cap1, a.fm_passes);
        for (int32_t i = lane; i < nv; i += 64) a.side[vlist[i]] = sw_all[i] < 0 ? 1 : 0;
        return;
    }

    // ---- one growth per wavefront
    const int32_t f = job.f, f0 = f / 2;
    const int64_t t0 = cB * f0 / f;
    const int64_t cap0 = job.cap0, cap1 = job.cap1;
    const int j = wv;
    // phases: the R GGG growths, then (pool) R BFS and R random growths; a phase's best run
    // replaces the kept one only if it is strictly better, so the first of equal runs is kept.
    // With the families side by side, this workgroup runs its own family only.
    const int alg_end = a.algs > 1 ? alg_first + 1 : (a.pool ? 3 : 1);
    uint8_t* const out_sides = a.algs > 1 ? a.side_alg + job.soff + (int64_t)alg_first * nv : nullptr;
    auto put_side = [&](int32_t i, uint8_t sd) {
        if (out_sides) out_sides[i] = sd;
        else a.side[vlist[i]] = sd;
    };
    for (int alg = alg_first; alg < alg_end; ++alg) {
        const uint32_t hpre = alg == ALG_GGG ? job.hpre : (alg == ALG_BFS ? job.hpre_bfs : job.hpre_rnd);
        const uint32_t hj =
            hash_step(hash_step(hash_step(hpre, (uint32_t)job.first, 3), (uint32_t)f, 4), (uint32_t)j, 5);
        const bool use32 = k32 && alg != ALG_RND;
        if (alg == ALG_GGG) {
            if (use32)
                ggg_grow<Key32, LDS, ALG_GGG>(key_all, nvp, nv, nd, ed, wdeg, j, lane, hj, cB, t0, cap0, cap1, s_cut,
                                              s_over, sw_all, a.fm_passes);
            else
                ggg_grow<Key64, LDS, ALG_GGG>(key_all, nvp, nv, nd, ed, wdeg, j, lane, hj, cB, t0, cap0, cap1, s_cut,
                                              s_over, sw_all, a.fm_passes);
        } else if (alg == ALG_BFS) {
            if (use32)
                ggg_grow<Key32, LDS, ALG_BFS>(key_all, nvp, nv, nd, ed, wdeg, j, lane, hj, cB, t0, cap0, cap1, s_cut,
                                              s_over, sw_all, a.fm_passes);
            else
                ggg_grow<Key64, LDS, ALG_BFS>(key_all, nvp, nv, nd, ed, wdeg, j, lane, hj, cB, t0, cap0, cap1, s_cut,
                                              s_over, sw_all, a.fm_passes);
        } else {
            ggg_grow<Key64, LDS, ALG_RND>(key_all, nvp, nv, nd, ed, wdeg, j, lane, hj, cB, t0, cap0, cap1, s_cut, s_over,
                                          sw_all, a.fm_passes);
        }
        __syncthreads();
        if (tid == 0) {
            int bj = 0;
            for (int q = 1; q < kSeeds; ++q) {
                const bool fq = s_over[q] > 0, fb = s_over[bj] > 0;
                bool better;
                if (fq != fb) better = !fq;
                else if (s_over[q] != s_over[bj]) better = s_over[q] < s_over[bj];
                else better = s_cut[q] < s_cut[bj];
                if (better) bj = q;
            }
            bool take = alg == alg_first;
            if (!take) {
                const bool fq = s_over[bj] > 0, fb = s_keep_over > 0;
                if (fq != fb) take = !fq;
                else if (s_over[bj] != s_keep_over) take = s_over[bj] < s_keep_over;
                else take = s_cut[bj] < s_keep_cut;
            }
            if (take) {
                s_keep_over = s_over[bj];
                s_keep_cut = s_cut[bj];
            }
            s_take = take;
            s_best = bj;
        }
        __syncthreads();
        if (s_take) {
            if (a.fm_passes > 0) {
                const int32_t* sb = sw_all + (int64_t)s_best * nvp;
                for (int32_t i = tid; i < nv; i += GGG_THREADS) put_side(i, sb[i] < 0 ? 1 : 0);
            } else if (use32) {
                const uint32_t* kb = reinterpret_cast<const uint32_t*>(key_all) + (int64_t)s_best * nvp;
                for (int32_t i = tid; i < nv; i += GGG_THREADS) put_side(i, kb[i] == 0 ? 0 : 1);
            } else {
                const uint64_t* kb = key_all + (int64_t)s_best * nvp;
                for (int32_t i = tid; i < nv; i += GGG_THREADS) put_side(i, kb[i] == 0 ? 0 : 1);
            }
        }
        __syncthreads();  // the next phase rewrites the keys
    }
    if (a.algs > 1 && tid == 0) {
        a.res[((int64_t)jobi * a.algs + alg_first) * 2] = s_keep_over;
        a.res[((int64_t)jobi * a.algs + alg_first) * 2 + 1] = s_keep_cut;
    }
}

// The pool's families run side by side: per job, the family kept is GGG unless
// BFS is strictly better (feasible first, then less overload, then a smaller
// cut), and random replaces the kept one only if strictly better, the order in
// which one workgroup would have run them; its sides go to the vertices.
__global__ __launch_bounds__(kBlock) void k_ggg_pick(const GGGJob* __restrict__ jobs, const int64_t* __restrict__ res,
                                                     const uint32_t* __restrict__ verts,
                                                     const int32_t* __restrict__ bstart,
                                                     const uint8_t* __restrict__ side_alg, uint8_t* __restrict__ side)
{
    const GGGJob job = jobs[blockIdx.x];
    const int64_t* r = res + (int64_t)blockIdx.x * 6;
    int w = 0;
    int64_t ko = r[0], kc = r[1];
    for (int q = 1; q < 3; ++q) {
        const int64_t o = r[2 * q], cu = r[2 * q + 1];
        const bool fq = o > 0, fb = ko > 0;
        const bool better = fq != fb ? !fq : (o != ko ? o < ko : cu < kc);
        if (better) {
            w = q;
            ko = o;
            kc = cu;
        }
    }
    const uint32_t* vlist = verts + bstart[job.b];
    const uint8_t* sd = side_alg + job.soff + (int64_t)w * job.nverts;
    for (int32_t i = threadIdx.x; i < job.nverts; i += blockDim.x) side[vlist[i]] = sd[i];
}

__global__ void k_relabel(int32_t* __restrict__ part, const uint8_t* __restrict__ side,
                          const int32_t* __restrict__ newidx, const uint8_t* __restrict__ split, int32_t n)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t b = part[v];
    part[v] = newidx[b] + (split[b] ? side[v] : 0);
}

__global__ void k_project(const int32_t* __restrict__ cpart, const int32_t* __restrict__ map,
                          int32_t* __restrict__ fpart, int32_t n)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) fpart[v] = cpart[map[v]];
}

// batches: projected nodes take the renumbered coarse block; nodes of jobs
// whose coarsest level is this one (map < 0) start in their job's block
__global__ void k_project_jobs(const int32_t* __restrict__ cpart, const int32_t* __restrict__ map,
                               const int32_t* __restrict__ remap, const int32_t* __restrict__ gid,
                               const int32_t* __restrict__ start_block, int32_t* __restrict__ fpart, int32_t n)
{
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t c = map ? map[v] : -1;
    fpart[v] = c >= 0 ? remap[cpart[c]] : start_block[gid[v]];
}

__global__ __launch_bounds__(kBlock) void k_block_weights(const int32_t* __restrict__ part,
                                                          const int32_t* __restrict__ vwgt, int32_t n, int32_t nb,
                                                          int64_t* __restrict__ wt)
{
    __shared__ unsigned long long h[kPrivBlocks];
    const bool priv = nb <= kPrivBlocks;
    if (priv)
        for (int i = threadIdx.x; i < nb; i += kBlock) h[i] = 0;
    __syncthreads();
    // grid-stride: a few thousand blocks cover any n, each flushes nb counters once
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long c = (unsigned long long)(vwgt ? vwgt[v] : 1);
        if (priv) atomicAdd(&h[part[v]], c);
        else atomicAdd((unsigned long long*)&wt[part[v]], c);
    }
    __syncthreads();
    if (priv)
        for (int i = threadIdx.x; i < nb; i += kBlock)
            if (h[i]) atomicAdd((unsigned long long*)&wt[i], h[i]);
}

// Cut entries: a node's own lane walks rows of up to kCutLight entries; longer
// rows are split into runs of kCutRun entries, appended to a list and walked by
// whole workgroups in a second launch, so a hub of 10^5 neighbours does not
// hold one lane for the whole kernel.  gid == NULL: one graph, the sum goes to
// spread counters; else per job (each cut edge counted from both ends).
constexpr int32_t kCutLight = 256;
constexpr int32_t kCutRun = 4096;

__device__ inline void cut_out(int64_t* out, const int32_t* gid, int32_t j, int64_t acc)
{
    if (gid) {
        job_add(out, j, acc);
    } else {
        for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
        if ((threadIdx.x & 63) == 0 && acc) spread_add(out, acc);
    }
}

__global__ __launch_bounds__(kBlock) void k_cut(const int32_t* __restrict__ xadj, const int32_t* __restrict__ adjncy,
                                                const int32_t* __restrict__ adjwgt, const int32_t* __restrict__ part,
                                                const int32_t* __restrict__ gid, int32_t n, int64_t* out,
                                                int2* __restrict__ runs, int32_t* __restrict__ nruns)
{
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = base + threadIdx.x;
        int64_t acc = 0;
        int32_t j = -1;
        if (v < n) {
            j = gid ? gid[v] : 0;
            const int32_t e0 = xadj[v], e1 = xadj[v + 1];
            if (e1 - e0 <= kCutLight) {
                const int32_t p = part[v];
                for (int32_t e = e0; e < e1; ++e)
                    if (part[adjncy[e]] != p) acc += adjwgt ? adjwgt[e] : 1;
            } else {
                const int32_t k = (e1 - e0 + kCutRun - 1) / kCutRun;
                const int32_t at = atomicAdd(nruns, k);
                for (int32_t q = 0; q < k; ++q) runs[at + q] = make_int2((int32_t)v, q);
            }
        }
        cut_out(out, gid, j, acc);
    }
}

__global__ __launch_bounds__(kBlock) void k_cut_runs(const int32_t* __restrict__ xadj,
                                                     const int32_t* __restrict__ adjncy,
                                                     const int32_t* __restrict__ adjwgt,
                                                     const int32_t* __restrict__ part, const int32_t* __restrict__ gid,
                                                     int64_t* out, const int2* __restrict__ runs,
                                                     const int32_t* __restrict__ nruns)
{
    const int32_t total = *nruns;
    for (int32_t r = blockIdx.x; r < total; r += gridDim.x) {
        const int2 run = runs[r];
        const int32_t v = run.x;
        const int32_t e1 = xadj[v + 1];
        const int32_t r0 = xadj[v] + run.y * kCutRun, r1 = r0 + kCutRun < e1 ? r0 + kCutRun : e1;
        const int32_t p = part[v];
        int64_t acc = 0;
        for (int32_t e = r0 + threadIdx.x; e < r1; e += kBlock)
            if (part[adjncy[e]] != p) acc += adjwgt ? adjwgt[e] : 1;
        cut_out(out, gid, gid ? gid[v] : 0, acc);
    }
}

// LDS of a GGG workgroup (gfx950: 160 KiB per workgroup; the static tables
// take a few hundred bytes); larger blocks run on global scratch
constexpr int64_t kLdsBudget = 144 * 1024;

}  // namespace

// ---------------------------------------------------------------- adaptive imbalance
// Paper Sec. 2 / Alg. 2: a block that is to end as f blocks is bisected with
// eps' = ((1 + eps) c(V) f / (k c(B)))^(1/r) - 1, r = ceil(log2 f); side j is
// bounded by (1 + eps') ceil(c(B) f_j / f) (Sec. 5.2's L_2 for even f).  In
// 2^32 fixed point: x = floor(2^32 (1 + eps')^r) exactly, and 2^32 (1 + eps')
// is the largest q whose power, taken in r steps p <- floor(p q / 2^32) from
// p = 2^32, stays within x.  The search starts at a floating-point estimate
// and settles on that q with exact integer comparisons only (the estimate
// never decides the result).
namespace {
using u128 = unsigned __int128;
constexpr int64_t kCapInf = int64_t(1) << 62;

bool fixed_pow_within(uint64_t q, int r, uint64_t x)
{
    const bool grows = q >= (uint64_t(1) << 32);  // then p never decreases and p q stays below 2^128
    u128 p = u128(1) << 32;
    for (int i = 0; i < r; ++i) {
        p = (p * q) >> 32;
        if (grows && p > x) return false;
    }
    return p <= x;
}

uint64_t fixed_root(uint64_t x, int r)
{
    const long double est = std::pow((long double)x / 4294967296.0L, 1.0L / (long double)r) * 4294967296.0L;
    uint64_t q = !(est > 0) ? 0 : est >= 1.8e19L ? ~uint64_t(0) : (uint64_t)est;
    if (fixed_pow_within(q, r, x)) {
        // gallop up while q + step still fits, then halve the step
        uint64_t step = 1;
        while (step && q <= ~uint64_t(0) - step && fixed_pow_within(q + step, r, x)) {
            q += step;
            step <<= 1;
        }
        for (; step; step >>= 1)
            if (q <= ~uint64_t(0) - step && fixed_pow_within(q + step, r, x)) q += step;
    } else {
        // gallop down until q - step fits, then climb back by halving steps
        uint64_t step = 1;
        while (q >= step && !fixed_pow_within(q - step, r, x)) step <<= 1;
        uint64_t lo = q >= step ? q - step : 0;  // fits (P(0) = 0)
        for (uint64_t s2 = step >> 1; s2; s2 >>= 1)
            if (fixed_pow_within(lo + s2, r, x)) lo += s2;
        q = lo;
    }
    return q;
}
}  // namespace

void adaptive_side_caps(const AdaptiveJob& j, int64_t cB, int32_t f, int64_t& cap0, int64_t& cap1)
{
    if (cB <= 0) {
        cap0 = cap1 = 0;
        return;
    }
    int r = 1;
    while ((int64_t(1) << r) < f) ++r;
    const u128 x = (u128(1) << 32) * u128(kPPM + j.e) * u128(j.cV) * u128(f) / (u128(kPPM) * u128(j.k) * u128(cB));
    if (x >> 64) {
        cap0 = cap1 = kCapInf;
        return;
    }
    const uint64_t rho = fixed_root((uint64_t)x, r);
    const int32_t f0 = f / 2;
    const int64_t share[2] = {(cB * f0 + f - 1) / f, (cB * (f - f0) + f - 1) / f};
    int64_t caps[2];
    for (int s2 = 0; s2 < 2; ++s2) {
        const u128 cap = (u128(rho) * u128(share[s2])) >> 32;
        caps[s2] = cap > u128(kCapInf) ? kCapInf : (int64_t)cap;
    }
    cap0 = caps[0];
    cap1 = caps[1];
}

namespace {

template <typename T>
DBuf<T> to_dev(Ctx& c, const std::vector<T>& v)
{
    DBuf<T> d(c, std::max<size_t>(v.size(), 1));
    if (!v.empty()) c.write(d.p, v.data(), sizeof(T) * v.size());
    return d;
}

// Launches k_ggg for `jobs` over the graph and block arrays of `a`: blocks
// whose working set fits LDS go by LDS size class when there are more blocks
// than one launch at the largest size keeps resident (a launch's LDS size is
// its largest block's, and four 512-thread workgroups fit one CU when each
// takes at most 40 KiB), else in one LDS launch (launches run one after the
// other, so splitting few blocks only serialises them); then the hybrid and
// the global layouts.
void launch_ggg_jobs(Ctx& c, GGGArgs a, const std::vector<GGGJob>& jobs_in)
{
    if (jobs_in.empty()) return;
    constexpr int kLdsClasses = 4;
    const int64_t lds_class_max[kLdsClasses] = {40 << 10, 53 << 10, 80 << 10, kLdsBudget};
    std::vector<GGGJob> lds_jobs[kLdsClasses], hyb_jobs, glob_jobs;
    int64_t lds_max[kLdsClasses] = {0, 0, 0, 0}, hyb_max = 0, scratch_total = 0, sides_total = 0;
    const bool fm = a.fm_passes > 0;
    // the pool's three families side by side: one workgroup each, with scratch and sides of its own
    a.algs = a.pool && !a.given ? 3 : 1;
    for (GGGJob jb : jobs_in) {
        const int64_t bytes = ggg_bytes(jb.nverts, jb.dsum, fm);
        const int64_t hbytes = ggg_hybrid_lds(jb.nverts, fm);
        jb.scratch = 0;
        jb.sstride = 0;
        jb.soff = sides_total;
        if (a.algs > 1) sides_total += ((int64_t)a.algs * jb.nverts + 15) & ~(int64_t)15;
        if (bytes <= kLdsBudget) {
            int q = 0;
            while (bytes > lds_class_max[q]) ++q;
            lds_jobs[q].push_back(jb);
            lds_max[q] = std::max(lds_max[q], bytes);
        } else if (hbytes <= kLdsBudget) {
            // the internal entries in global memory: the device-wide extraction's, read in
            // place, or a copy in the scratch
            jb.scratch = scratch_total;
            jb.sstride = a.ied ? 0 : ((int64_t)jb.dsum * 8 + 255) & ~(int64_t)255;
            scratch_total += a.algs * jb.sstride;
            hyb_jobs.push_back(jb);
            hyb_max = std::max(hyb_max, hbytes);
        } else {
            jb.scratch = scratch_total;
            jb.sstride = (bytes + 255) & ~(int64_t)255;
            scratch_total += a.algs * jb.sstride;
            glob_jobs.push_back(jb);
        }
    }
    {
        size_t nl = 0;
        int64_t mx = 0;
        for (int q = 0; q < kLdsClasses; ++q) {
            nl += lds_jobs[q].size();
            mx = std::max(mx, lds_max[q]);
        }
        const int64_t resident = 256 * std::max<int64_t>(1, std::min<int64_t>(4, (160 << 10) / std::max<int64_t>(mx, 1)));
        if ((int64_t)nl * a.algs <= resident)
            for (int q = 0; q + 1 < kLdsClasses; ++q) {
                lds_jobs[kLdsClasses - 1].insert(lds_jobs[kLdsClasses - 1].end(), lds_jobs[q].begin(),
                                                 lds_jobs[q].end());
                lds_jobs[q].clear();
                lds_max[kLdsClasses - 1] = mx;
            }
    }
    DBuf<char> scratch;
    if (scratch_total > 0) scratch = DBuf<char>(c, (size_t)scratch_total);
    a.scratch = scratch.p;
    DBuf<uint8_t> side_alg;
    DBuf<int64_t> res;
    if (a.algs > 1) {
        side_alg = DBuf<uint8_t>(c, (size_t)std::max<int64_t>(sides_total, 16));
        res = DBuf<int64_t>(c, jobs_in.size() * 6);
    }
    a.side_alg = side_alg.p;
    // every job list in one upload
    std::vector<GGGJob> all;
    all.reserve(jobs_in.size());
    for (int q = 0; q < kLdsClasses; ++q) all.insert(all.end(), lds_jobs[q].begin(), lds_jobs[q].end());
    all.insert(all.end(), hyb_jobs.begin(), hyb_jobs.end());
    all.insert(all.end(), glob_jobs.begin(), glob_jobs.end());
    DBuf<GGGJob> jobs(c, all.size());
    c.write(jobs.p, all.data(), sizeof(GGGJob) * all.size());
    size_t at = 0;
    for (int q = 0; q < kLdsClasses; ++q) {
        if (lds_jobs[q].empty()) continue;
        a.jobs = jobs.p + at;
        a.res = res.p ? res.p + at * 6 : nullptr;
        allow_lds((const void*)k_ggg<GGG_LDS>, (int)kLdsBudget);  // beyond the 64 KiB default
        ProfScope ps(c, KMP_PROF_GGG);
        hipLaunchKernelGGL(k_ggg<GGG_LDS>, dim3((unsigned)(lds_jobs[q].size() * a.algs)), dim3(GGG_THREADS),
                           (size_t)lds_max[q], c.stream, a);
        KMP_LAUNCH_CHECK();
        at += lds_jobs[q].size();
    }
    if (!hyb_jobs.empty()) {
        a.jobs = jobs.p + at;
        a.res = res.p ? res.p + at * 6 : nullptr;
        allow_lds((const void*)k_ggg<GGG_HYBRID>, (int)kLdsBudget);
        ProfScope ps(c, KMP_PROF_GGG);
        hipLaunchKernelGGL(k_ggg<GGG_HYBRID>, dim3((unsigned)(hyb_jobs.size() * a.algs)), dim3(GGG_THREADS),
                           (size_t)hyb_max, c.stream, a);
        KMP_LAUNCH_CHECK();
        at += hyb_jobs.size();
    }
    if (!glob_jobs.empty()) {
        a.jobs = jobs.p + at;
        a.res = res.p ? res.p + at * 6 : nullptr;
        ProfScope ps(c, KMP_PROF_GGG);
        hipLaunchKernelGGL(k_ggg<GGG_GLOBAL>, dim3((unsigned)(glob_jobs.size() * a.algs)), dim3(GGG_THREADS), 0,
                           c.stream, a);
        KMP_LAUNCH_CHECK();
    }
    if (a.algs > 1) {
        ProfScope ps(c, KMP_PROF_GGG);
        hipLaunchKernelGGL(k_ggg_pick, dim3((unsigned)all.size()), dim3(kBlock), 0, c.stream, jobs.p, res.p, a.verts,
                           a.bstart, side_alg.p, a.side);
        KMP_LAUNCH_CHECK();
    }
}

// ---------------------------------------------------------------- multilevel IP
// Multilevel initial bipartitioning (paper Sec. 5.2 "Initial Bipartitioning";
// kmp_options.ip_multilevel): the subgraphs of the blocks to split become the
// jobs of one union graph (jobs in block order, a node's union id = its job's
// offset + its local id, entries in the level graph's row order), which the
// batch LP (own seed per block, level key 64 + 64 l + i, cluster bound
// max(heaviest node, larger side bound / kIpCcf)) and the batch contraction
// coarsen level by level until a job's clustering leaves every node alone;
// k_ggg bipartitions each job's coarsest graph (the single-level growths and
// FM), and on the way back every finer level takes the projected sides and
// k_ggg's refine mode runs the FM passes on them.
constexpr int64_t kIpCcf = 18;
constexpr int32_t kIpMaxLev = 32;

// Level-0 union nodes: id, job, node weight, source vertex; rows of up to
// kGggLightRow entries are counted here, longer ones listed for k_ml_heavy.
__global__ void k_ml_nodes(const uint32_t* __restrict__ verts, const int32_t* __restrict__ part,
                           const int32_t* __restrict__ bstart, const int32_t* __restrict__ qidx,
                           const int32_t* __restrict__ uoff, const int32_t* __restrict__ xadj,
                           const int32_t* __restrict__ adjncy, const int32_t* __restrict__ vwgt, int32_t n,
                           int32_t* __restrict__ rows, int32_t* __restrict__ uvw, int32_t* __restrict__ ugid,
                           int32_t* __restrict__ usrc, int32_t* __restrict__ heavy, int32_t* __restrict__ nheavy)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = (int32_t)verts[i];
    const int32_t b = part[v];
    const int32_t q = qidx[b];
    if (q < 0) return;
    const int32_t uid = uoff[q] + (int32_t)(i - bstart[b]);
    usrc[uid] = v;
    ugid[uid] = q;
    uvw[uid] = vwgt ? vwgt[v] : 1;
    const int32_t e0 = xadj[v], e1 = xadj[v + 1];
    if (e1 - e0 > kGggLightRow) {
        heavy[atomicAdd(nheavy, 1)] = uid;
        return;
    }
    int32_t cnt = 0;
    for (int32_t e = e0; e < e1; ++e) cnt += part[adjncy[e]] == b;
    rows[uid] = cnt;
}

// Internal entries of the listed long rows, one wavefront per row (the grid
// strides over the list, whose length is read on the device).
__global__ __launch_bounds__(kBlock) void k_ml_heavy_count(const int32_t* __restrict__ heavy,
                                                           const int32_t* __restrict__ nheavy,
                                                           const int32_t* __restrict__ usrc,
                                                           const int32_t* __restrict__ part,
                                                           const int32_t* __restrict__ xadj,
                                                           const int32_t* __restrict__ adjncy,
                                                           int32_t* __restrict__ rows)
{
    const int lane = threadIdx.x & 63;
    const int32_t nh = *nheavy;
    for (int64_t h = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; h < nh;
         h += ((int64_t)gridDim.x * blockDim.x) >> 6) {
        const int32_t uid = heavy[h];
        const int32_t v = usrc[uid];
        const int32_t b = part[v];
        uint32_t cnt = 0;
        for (int32_t e = xadj[v] + lane; e < xadj[v + 1]; e += 64) cnt += part[adjncy[e]] == b;
        cnt = group_sum_u32<64>(cnt);
        if (lane == 0) rows[uid] = (int32_t)cnt;
    }
}

// Entries of the union rows: light rows by their own thread, listed rows by a
// wavefront (ballot keeps the row order).  Neighbour u becomes its job's
// offset + local[u].
__global__ __launch_bounds__(kBlock) void k_ml_fill(const int32_t* __restrict__ usrc, const int32_t* __restrict__ ugid,
                                                    const int32_t* __restrict__ uoff, int32_t N,
                                                    const int32_t* __restrict__ heavy,
                                                    const int32_t* __restrict__ nheavy,
                                                    const int32_t* __restrict__ part,
                                                    const int32_t* __restrict__ local,
                                                    const int32_t* __restrict__ xadj,
                                                    const int32_t* __restrict__ adjncy,
                                                    const int32_t* __restrict__ adjwgt,
                                                    const int32_t* __restrict__ uxadj, int32_t* __restrict__ uadj,
                                                    int32_t* __restrict__ uw)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t uid = t; uid < N; uid += stride) {
        const int32_t v = usrc[uid];
        const int32_t e0 = xadj[v], e1 = xadj[v + 1];
        if (e1 - e0 > kGggLightRow) continue;
        const int32_t b = part[v], base = uoff[ugid[uid]];
        int32_t pos = uxadj[uid];
        for (int32_t e = e0; e < e1; ++e) {
            const int32_t u = adjncy[e];
            if (part[u] != b) continue;
            uadj[pos] = base + local[u];
            uw[pos] = adjwgt ? adjwgt[e] : 1;
            ++pos;
        }
    }
    const int lane = threadIdx.x & 63;
    const int32_t nh = *nheavy;
    for (int64_t h = t >> 6; h < nh; h += stride >> 6) {
        const int32_t uid = heavy[h];
        const int32_t v = usrc[uid];
        const int32_t b = part[v], base = uoff[ugid[uid]];
        const int32_t e0 = xadj[v], e1 = xadj[v + 1];
        int32_t pos = uxadj[uid];
        for (int32_t c0 = e0; c0 < e1; c0 += 64) {
            const int32_t e = c0 + lane;
            const int32_t u = e < e1 ? adjncy[e] : -1;
            const bool in = u >= 0 && part[u] == b;
            const uint64_t m = __ballot(in);
            if (in) {
                const int32_t at = pos + __popcll(m & ((1ull << lane) - 1));
                uadj[at] = base + local[u];
                uw[at] = adjwgt ? adjwgt[e] : 1;
            }
            pos += __popcll(m);
        }
    }
}

// Job of every node of a level (members' node ranges in job order).
__global__ void k_ml_gid(const int32_t* __restrict__ moff, const int32_t* __restrict__ mjob, int32_t cnt, int32_t N,
                         int32_t* __restrict__ gid, int32_t* __restrict__ local, uint32_t* __restrict__ iota)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    int32_t lo = 0, hi = cnt - 1;  // the last member whose range starts at or before v
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (moff[mid] <= v) lo = mid;
        else hi = mid - 1;
    }
    gid[v] = mjob[lo];
    local[v] = (int32_t)v - moff[lo];
    iota[v] = (uint32_t)v;
}

__global__ void k_ml_init(const int32_t* __restrict__ vw, int32_t n, int32_t* __restrict__ label,
                          int64_t* __restrict__ cw, int32_t* __restrict__ maxc, const int32_t* __restrict__ gid)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    label[v] = (int32_t)v;
    cw[v] = vw[v];
    atomicMax(&maxc[gid[v]], vw[v]);
}

__global__ void k_ml_bounds(const int32_t* __restrict__ xadj, const int32_t* __restrict__ moff, int32_t cnt,
                            int32_t* __restrict__ out)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= cnt) out[i] = xadj[moff[i]];
}

__global__ void k_ml_project(const int32_t* __restrict__ map, const uint8_t* __restrict__ cside, int32_t n,
                             uint8_t* __restrict__ side)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n && map[v] >= 0) side[v] = cside[map[v]];
}

__global__ void k_ml_out(const int32_t* __restrict__ usrc, const uint8_t* __restrict__ uside, int32_t N,
                         uint8_t* __restrict__ side)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < N) side[usrc[u]] = uside[u];
}

struct MLLevel {
    OwnedGraph own;
    DGraph g;
    std::vector<int32_t> mem;   // member jobs, ascending
    std::vector<int32_t> moff;  // by member: first node; moff[mem.size()] = n
    std::vector<int32_t> nq;    // by job: nodes at this level
    DBuf<int32_t> gid, local, noff, map;
    DBuf<uint32_t> iota;
    DBuf<uint8_t> side;
};

// gid, local ids, identity list and per-job node offsets of a level.
void ml_tables(Ctx& c, MLLevel& L, int32_t J)
{
    const int32_t cnt = (int32_t)L.mem.size();
    const int32_t N = L.g.n;
    std::vector<int32_t> noff(J, 0);
    for (int32_t i = 0; i < cnt; ++i) noff[L.mem[i]] = L.moff[i];
    L.noff = to_dev(c, noff);
    DBuf<int32_t> dmoff = to_dev(c, L.moff), dmem = to_dev(c, L.mem);
    L.gid = DBuf<int32_t>(c, (size_t)std::max(N, 1));
    L.local = DBuf<int32_t>(c, (size_t)std::max(N, 1));
    L.iota = DBuf<uint32_t>(c, (size_t)std::max(N, 1));
    L.side = DBuf<uint8_t>(c, (size_t)std::max(N, 1));
    if (N > 0) {
        hipLaunchKernelGGL(k_ml_gid, dim3(grid_for(N)), dim3(kBlock), 0, c.stream, dmoff.p, dmem.p, cnt, N, L.gid.p,
                           L.local.p, L.iota.p);
        KMP_LAUNCH_CHECK();
    }
}

void ml_bipartition_blocks(Ctx& c, const DGraph& g, int32_t level, const GGGArgs& ga, const std::vector<GGGJob>& gj,
                           const std::vector<uint64_t>& jseed, const int32_t* hb, int32_t nb)
{
    const int32_t J = (int32_t)gj.size();
    const int32_t n = g.n;
    std::vector<int32_t> qidx(nb, -1), uoff(J + 1, 0);
    for (int32_t q = 0; q < J; ++q) {
        qidx[gj[q].b] = q;
        uoff[q + 1] = uoff[q] + gj[q].nverts;
    }
    const int32_t N0 = uoff[J];
    if (N0 == 0) return;
    // ---- level 0: the union of the blocks' subgraphs
    std::vector<std::unique_ptr<MLLevel>> L;
    L.emplace_back(new MLLevel());
    MLLevel& L0 = *L[0];
    DBuf<int32_t> usrc(c, (size_t)N0);
    {
        DBuf<int32_t> dq = to_dev(c, qidx), duoff = to_dev(c, uoff);
        DBuf<int32_t> rows(c, (size_t)N0 + 1), heavy(c, (size_t)N0), nheavy(c, 1);
        L0.own.vwgt = DBuf<int32_t>(c, (size_t)N0);
        DBuf<int32_t> ugid(c, (size_t)N0);
        c.zero(nheavy.p, sizeof(int32_t));
        hipLaunchKernelGGL(k_ml_nodes, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, ga.verts, ga.part, ga.bstart, dq.p,
                           duoff.p, g.xadj, g.adjncy, g.vwgt, n, rows.p, L0.own.vwgt.p, ugid.p, usrc.p, heavy.p,
                           nheavy.p);
        KMP_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_ml_heavy_count, dim3(grid_for(N0, kBlock / 64, 4096)), dim3(kBlock), 0, c.stream,
                           heavy.p, nheavy.p, usrc.p, ga.part, g.xadj, g.adjncy, rows.p);
        KMP_LAUNCH_CHECK();
        L0.own.xadj = DBuf<int32_t>(c, (size_t)N0 + 1);
        scan_excl_i32(c, rows.p, L0.own.xadj.p, N0, L0.own.xadj.p + N0);
        const int32_t M0 = c.read1(L0.own.xadj.p + N0);
        L0.own.adjncy = DBuf<int32_t>(c, (size_t)std::max(M0, 1));
        L0.own.adjwgt = DBuf<int32_t>(c, (size_t)std::max(M0, 1));
        hipLaunchKernelGGL(k_ml_fill, dim3(grid_for(N0, kBlock, 4096)), dim3(kBlock), 0, c.stream, usrc.p, ugid.p,
                           duoff.p, N0, heavy.p, nheavy.p, ga.part, ga.local, g.xadj, g.adjncy, g.adjwgt,
                           L0.own.xadj.p, L0.own.adjncy.p, L0.own.adjwgt.p);
        KMP_LAUNCH_CHECK();
        L0.g = L0.own.view(N0, M0);
        L0.nq.assign(J, 0);
        L0.moff.assign(1, 0);
        for (int32_t q = 0; q < J; ++q) {
            L0.mem.push_back(q);
            L0.nq[q] = gj[q].nverts;
            L0.moff.push_back(uoff[q + 1]);
        }
        ml_tables(c, L0, J);
    }
    // ---- coarsening (the deterministic sub-round LP, whatever the LP mode of the partition)
    std::vector<uint32_t> gh(J);
    for (int32_t q = 0; q < J; ++q) gh[q] = seed_hash(jseed[q]);
    DBuf<uint32_t> dgh = to_dev(c, gh);
    std::vector<int32_t> coarsest(J, 0);
    const int32_t saved_async = c.async_lp;
    c.async_lp = 0;
    for (int32_t i = 0;; ++i) {
        MLLevel& Li = *L[i];
        const int32_t N = Li.g.n;
        const uint32_t lvkey = 64u + 64u * (uint32_t)level + (uint32_t)i;
        DBuf<int32_t> label(c, (size_t)N), maxc(c, (size_t)J);
        DBuf<int64_t> cw(c, (size_t)N);
        c.zero(maxc.p, sizeof(int32_t) * J);
        hipLaunchKernelGGL(k_ml_init, dim3(grid_for(N)), dim3(kBlock), 0, c.stream, Li.g.vwgt, N, label.p, cw.p,
                           maxc.p, Li.gid.p);
        KMP_LAUNCH_CHECK();
        std::vector<int32_t> hmax(J);
        c.read(hmax.data(), maxc.p, sizeof(int32_t) * J);
        std::vector<int64_t> U(J, 0);
        for (int32_t q : Li.mem) U[q] = std::max<int64_t>(hmax[q], std::max(gj[q].cap0, gj[q].cap1) / kIpCcf);
        DBuf<int64_t> dU = to_dev(c, U);
        const JobTabs jt{Li.gid.p, dgh.p, Li.noff.p};
        LPSchedule sched;
        lp_build_schedule(c, Li.g, (int32_t)lvkey, 0, sched, jt, nullptr, J);
        LPState ls{label.p, cw.p, N, nullptr, 0, nullptr, TAG_CL, jt, Li.noff.p, dU.p};
        ls.njobs = J;
        for (size_t mi = 0; mi < Li.mem.size(); ++mi) {
            const int32_t q = Li.mem[mi];
            if (Li.nq[q] > 0 && small_job_fits(c, Li.nq[q], Li.nq[q]) && sched.job_maxdeg[q] <= c.tune.cut[1]) {
                ls.small_jobs.push_back(q);
                ls.small_start.push_back(Li.moff[mi]);
                ls.small_count.push_back(Li.nq[q]);
                ls.small_loff.push_back(Li.moff[mi]);
                ls.small_nlab.push_back(Li.nq[q]);
            }
        }
        DBuf<int64_t> mv(c, kRounds + 1);
        c.zero(mv.p, sizeof(int64_t) * (kRounds + 1));
        ls.moves_out = mv.p;
        lp_run(c, Li.g, (int32_t)lvkey, 0, &sched, ls);
        std::vector<int64_t> nc;
        count_nonempty_jobs(c, cw.p, N, jt, J, nc);
        std::vector<uint8_t> keep(J, 0);
        int32_t nkeep = 0;
        for (int32_t q : Li.mem) {
            if (nc[q] < Li.nq[q] && i + 1 < kIpMaxLev) {
                keep[q] = 1;
                ++nkeep;
            } else {
                coarsest[q] = i;
            }
        }
        if (nkeep == 0) break;
        std::unique_ptr<MLLevel> next(new MLLevel());
        Li.map = DBuf<int32_t>(c, (size_t)N);
        int32_t cn = 0;
        int64_t cm = 0;
        DBuf<uint8_t> dkeep = to_dev(c, keep);
        contract(c, Li.g, label.p, cw.p, Li.map.p, next->own, cn, cm, jt, dkeep.p);
        next->g = next->own.view(cn, cm);
        next->nq.assign(J, 0);
        next->moff.assign(1, 0);
        for (int32_t q : Li.mem)
            if (keep[q]) {
                next->mem.push_back(q);
                next->nq[q] = (int32_t)nc[q];
                next->moff.push_back(next->moff.back() + (int32_t)nc[q]);
            }
        ml_tables(c, *next, J);
        L.push_back(std::move(next));
    }
    c.async_lp = saved_async;
    // ---- the growths on every job's coarsest graph
    const int32_t depth = (int32_t)L.size() - 1;
    for (int32_t i = 0; i <= depth; ++i) {
        MLLevel& Li = *L[i];
        std::vector<int32_t> qs;
        for (int32_t q : Li.mem)
            if (coarsest[q] == i) qs.push_back(q);
        if (qs.empty()) continue;
        const int32_t cnt = (int32_t)Li.mem.size();
        DBuf<int32_t> dmoff = to_dev(c, Li.moff), bnd(c, (size_t)cnt + 1);
        hipLaunchKernelGGL(k_ml_bounds, dim3(grid_for(cnt + 1)), dim3(kBlock), 0, c.stream, Li.g.xadj, dmoff.p, cnt,
                           bnd.p);
        KMP_LAUNCH_CHECK();
        std::vector<int32_t> hbnd(cnt + 1);
        c.read(hbnd.data(), bnd.p, sizeof(int32_t) * (cnt + 1));
        std::vector<int32_t> ent(J, 0);
        for (int32_t mi = 0; mi < cnt; ++mi) ent[Li.mem[mi]] = hbnd[mi + 1] - hbnd[mi];
        std::vector<GGGJob> jobs;
        for (int32_t q : qs) {
            GGGJob jb = gj[q];
            jb.b = q;
            jb.nverts = Li.nq[q];
            jb.dsum = ent[q];
            jobs.push_back(jb);
        }
        GGGArgs a = ga;
        a.ioff = nullptr;  // subgraph rows of their own
        a.iw = nullptr;
        a.ied = nullptr;
        a.xadj = Li.g.xadj;
        a.adjncy = Li.g.adjncy;
        a.vwgt = Li.g.vwgt;
        a.adjwgt = Li.g.adjwgt;
        a.part = Li.gid.p;
        a.verts = Li.iota.p;
        a.bstart = Li.noff.p;
        a.local = Li.local.p;
        a.side = Li.side.p;
        a.given = nullptr;
        launch_ggg_jobs(c, a, jobs);
    }
    // ---- back up: projection and FM on every finer level
    for (int32_t i = depth - 1; i >= 0; --i) {
        MLLevel& Li = *L[i];
        hipLaunchKernelGGL(k_ml_project, dim3(grid_for(Li.g.n)), dim3(kBlock), 0, c.stream, Li.map.p, L[i + 1]->side.p,
                           Li.g.n, Li.side.p);
        KMP_LAUNCH_CHECK();
        if (ga.fm_passes <= 0) continue;
        const int32_t cnt = (int32_t)Li.mem.size();
        DBuf<int32_t> dmoff = to_dev(c, Li.moff), bnd(c, (size_t)cnt + 1);
        hipLaunchKernelGGL(k_ml_bounds, dim3(grid_for(cnt + 1)), dim3(kBlock), 0, c.stream, Li.g.xadj, dmoff.p, cnt,
                           bnd.p);
        KMP_LAUNCH_CHECK();
        std::vector<int32_t> hbnd(cnt + 1);
        c.read(hbnd.data(), bnd.p, sizeof(int32_t) * (cnt + 1));
        std::vector<GGGJob> jobs;
        for (int32_t mi = 0; mi < cnt; ++mi) {
            const int32_t q = Li.mem[mi];
            if (coarsest[q] <= i) continue;
            GGGJob jb = gj[q];
            jb.b = q;
            jb.nverts = Li.nq[q];
            jb.dsum = hbnd[mi + 1] - hbnd[mi];
            jobs.push_back(jb);
        }
        GGGArgs a = ga;
        a.ioff = nullptr;  // subgraph rows of their own
        a.iw = nullptr;
        a.ied = nullptr;
        a.xadj = Li.g.xadj;
        a.adjncy = Li.g.adjncy;
        a.vwgt = Li.g.vwgt;
        a.adjwgt = Li.g.adjwgt;
        a.part = Li.gid.p;
        a.verts = Li.iota.p;
        a.bstart = Li.noff.p;
        a.local = Li.local.p;
        a.side = Li.side.p;
        a.given = Li.side.p;
        a.pool = 0;
        launch_ggg_jobs(c, a, jobs);
    }
    hipLaunchKernelGGL(k_ml_out, dim3(grid_for(N0)), dim3(kBlock), 0, c.stream, usrc.p, L0.side.p, N0, ga.side);
    KMP_LAUNCH_CHECK();
}

}  // namespace

int32_t bipartition_round(Ctx& c, const DGraph& g, int32_t level, int32_t* part, BlockTab& bt,
                          const std::vector<uint8_t>& split, const std::vector<int64_t>& lk,
                          const std::vector<uint32_t>& hseed, const std::vector<AdaptiveJob>* adapt,
                          const std::vector<uint64_t>* seeds64)
{
    const int32_t n = g.n;
    const int32_t nb = bt.size();
    bool any = false;
    for (int32_t bb = 0; bb < nb; ++bb) any |= split[bb] != 0;
    if (!any) return 0;
    DBuf<uint8_t> side(c, (size_t)n);
    int32_t calls = 0;
    if (n > 0) {
        // block starts (nb + 1) and degree sums (nb) in one buffer: one read-back
        DBuf<int32_t> bsd(c, 2 * (size_t)nb + 1);
        int32_t* bstart_p = bsd.p;
        int32_t* bdeg_p = bsd.p + nb + 1;
        fill_bytes_many(c, {{bsd.p, 4 * (2 * (int64_t)nb + 1), 0}});
        DBuf<uint32_t> key(c, n), verts(c, n), k2(c, n), v2(c, n);
        hipLaunchKernelGGL(k_block_count, dim3(grid_for(n, kBlock, 256)), dim3(kBlock), 0, c.stream, part, g.xadj, n, nb,
                           bstart_p, bdeg_p, key.p, verts.p);
        KMP_LAUNCH_CHECK();
        uint32_t* vsorted = nullptr;  // the block-sorted vertices (verts or v2)
        radix_sort_pairs(c, key.p, verts.p, k2.p, v2.p, n, bits_for((uint64_t)(nb - 1)), nullptr, &vsorted);
        scan_excl_i32(c, bstart_p, bstart_p, nb, bstart_p + nb);
        DBuf<int32_t> local(c, (size_t)n);
        hipLaunchKernelGGL(k_local_ids, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, vsorted, part, bstart_p, n,
                           local.p);
        KMP_LAUNCH_CHECK();
        std::vector<int32_t> hbd(2 * (size_t)nb + 1);
        c.read(hbd.data(), bsd.p, sizeof(int32_t) * hbd.size());
        std::vector<int64_t> hbw;  // block weights, for the adaptive caps
        if (adapt) {
            DBuf<int64_t> bw(c, (size_t)nb);
            block_weights(c, g, part, nb, bw.p);
            hbw.resize(nb);
            c.read(hbw.data(), bw.p, sizeof(int64_t) * nb);
        }
        const int32_t* hb = hbd.data();
        const int32_t* hd = hbd.data() + nb + 1;
        // Levels where a block to split has rows too long to hold in LDS (its degree sum bounds
        // its internal entries) take the extraction over the whole device: the greedy growing
        // then reads the exact internal rows, and blocks whose internal entries fit LDS run
        // there.  Other levels extract inside the growth launch.
        bool ext = false;
        int64_t sdeg = 0;
        for (int32_t bb = 0; bb < nb && !c.ip_multilevel; ++bb) {
            if (!split[bb]) continue;
            sdeg += hd[bb];
            if (ggg_bytes(hb[bb + 1] - hb[bb], hd[bb], c.fm_passes > 0) > kLdsBudget) ext = true;
        }
        std::vector<int32_t> hint;  // internal entries per block (extraction over the device)
        DBuf<int32_t> ioff, iw;
        DBuf<int2> ied;
        if (ext) {
            // timed with the growth launches (class ggg): the extraction is a step of the
            // initial bipartitioning
            auto scope = std::make_unique<ProfScope>(c, KMP_PROF_GGG);
            DBuf<uint8_t> dsplit(c, (size_t)nb);
            c.write(dsplit.p, split.data(), (size_t)nb);
            // a long row of d > kExtLight entries has at most d / kExtChunk + 1 chunks
            const int64_t ubt = sdeg / kExtChunk + sdeg / (kExtLight + 1) + 1;
            DBuf<int32_t> nch(c, (size_t)n), cplan(c, (size_t)n + 1), crow(c, (size_t)ubt), pc(c, (size_t)n);
            DBuf<int32_t> ccnt(c, (size_t)ubt), cpre(c, (size_t)ubt + 1), bint(c, (size_t)nb);
            iw = DBuf<int32_t>(c, (size_t)n);
            ioff = DBuf<int32_t>(c, (size_t)n + 1);
            fill_bytes_many(c, {{ccnt.p, 4 * ubt, 0},
                                {pc.p, 4 * (int64_t)n, 0},
                                {iw.p, 4 * (int64_t)n, 0},
                                {bint.p, 4 * (int64_t)nb, 0}});
            ExtArgs ea;
            ea.verts = vsorted;
            ea.part = part;
            ea.xadj = g.xadj;
            ea.adjncy = g.adjncy;
            ea.adjwgt = g.adjwgt;
            ea.local = local.p;
            ea.split = dsplit.p;
            ea.n = n;
            ea.nch = nch.p;
            ea.cplan = cplan.p;
            ea.crow = crow.p;
            ea.pc = pc.p;
            ea.ccnt = ccnt.p;
            ea.ioff = ioff.p;
            ea.cpre = cpre.p;
            ea.iw = iw.p;
            ea.bint = bint.p;
            ea.ied = nullptr;
            hipLaunchKernelGGL(k_ext_plan, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, ea);
            KMP_LAUNCH_CHECK();
            scan_excl_i32(c, nch.p, cplan.p, n, cplan.p + n);
            hipLaunchKernelGGL(k_ext_rows, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, cplan.p, n, crow.p);
            KMP_LAUNCH_CHECK();
            const dim3 cgrid(grid_for(ubt, kBlock / 64, 65536));
            hipLaunchKernelGGL(k_ext_light<false>, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, ea);
            KMP_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_ext_chunks<false>, cgrid, dim3(kBlock), 0, c.stream, ea);
            KMP_LAUNCH_CHECK();
            scan_excl_i32(c, pc.p, ioff.p, n, ioff.p + n);
            scan_excl_i32(c, ccnt.p, cpre.p, ubt, cpre.p + ubt);
            scope.reset();
            hint.resize(nb);
            c.read(hint.data(), bint.p, sizeof(int32_t) * nb);
            int64_t tot = 0;
            for (int32_t bb = 0; bb < nb; ++bb) tot += hint[bb];
            ied = DBuf<int2>(c, (size_t)std::max<int64_t>(tot, 1));
            ea.ied = ied.p;
            ProfScope ps(c, KMP_PROF_GGG);
            hipLaunchKernelGGL(k_ext_light<true>, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, ea);
            KMP_LAUNCH_CHECK();
            hipLaunchKernelGGL(k_ext_chunks<true>, cgrid, dim3(kBlock), 0, c.stream, ea);
            KMP_LAUNCH_CHECK();
        }
        std::vector<GGGJob> gjobs;
        for (int32_t bb = 0; bb < nb; ++bb) {
            if (!split[bb]) continue;
            const int32_t jb_job = bt.job.empty() ? 0 : bt.job[bb];
            GGGJob jb;
            jb.b = bb;
            jb.first = bt.first[bb];
            jb.f = bt.f[bb];
            jb.nverts = hb[bb + 1] - hb[bb];
            jb.dsum = ext ? hint[bb] : hd[bb];
            jb.hpre = hash_step(hash_step(hseed[jb_job], TAG_GGG, 1), (uint32_t)level, 2);
            jb.hpre_bfs = hash_step(hash_step(hseed[jb_job], TAG_BFS, 1), (uint32_t)level, 2);
            jb.hpre_rnd = hash_step(hash_step(hseed[jb_job], TAG_RND, 1), (uint32_t)level, 2);
            jb.scratch = 0;
            jb.lk = lk[jb_job];
            jb.cap0 = (int64_t)(jb.f / 2) * jb.lk;
            jb.cap1 = (int64_t)(jb.f - jb.f / 2) * jb.lk;
            if (adapt) adaptive_side_caps((*adapt)[jb_job], hbw[bb], jb.f, jb.cap0, jb.cap1);
            gjobs.push_back(jb);
            ++calls;
        }
        GGGArgs a;
        a.xadj = g.xadj;
        a.adjncy = g.adjncy;
        a.vwgt = g.vwgt;
        a.adjwgt = g.adjwgt;
        a.part = part;
        a.verts = vsorted;
        a.bstart = bstart_p;
        a.local = local.p;
        a.side = side.p;
        a.scratch = nullptr;
        a.fm_passes = c.fm_passes;
        a.pool = c.ip_pool ? 1 : 0;
        a.given = nullptr;
        a.ioff = ext ? ioff.p : nullptr;
        a.iw = ext ? iw.p : nullptr;
        a.ied = ext ? ied.p : nullptr;
        if (c.ip_multilevel) {
            std::vector<uint64_t> jseed(gjobs.size());
            for (size_t q = 0; q < gjobs.size(); ++q) {
                const int32_t jb_job = bt.job.empty() ? 0 : bt.job[gjobs[q].b];
                jseed[q] = (*seeds64)[jb_job] ^ ((uint64_t)(uint32_t)gjobs[q].first << 32);
            }
            ml_bipartition_blocks(c, g, level, a, gjobs, jseed, hb, nb);
        } else {
            launch_ggg_jobs(c, a, gjobs);
        }
    }
    // renumber blocks: split blocks become (first, f0) and (first + f0, f - f0)
    std::vector<int32_t> newidx(nb);
    BlockTab nt;
    nt.first.reserve(2 * nb);
    nt.f.reserve(2 * nb);
    nt.job.reserve(2 * nb);
    for (int32_t bb = 0; bb < nb; ++bb) {
        const int32_t jb_job = bt.job.empty() ? 0 : bt.job[bb];
        newidx[bb] = nt.size();
        if (split[bb]) {
            const int32_t f0 = bt.f[bb] / 2;
            nt.first.push_back(bt.first[bb]);
            nt.f.push_back(f0);
            nt.job.push_back(jb_job);
            nt.first.push_back(bt.first[bb] + f0);
            nt.f.push_back(bt.f[bb] - f0);
            nt.job.push_back(jb_job);
        } else {
            nt.first.push_back(bt.first[bb]);
            nt.f.push_back(bt.f[bb]);
            nt.job.push_back(jb_job);
        }
    }
    if (n > 0) {
        DBuf<int32_t> dnew(c, (size_t)nb);
        DBuf<uint8_t> dsplit(c, (size_t)nb);
        c.write(dnew.p, newidx.data(), sizeof(int32_t) * nb);
        c.write(dsplit.p, split.data(), (size_t)nb);
        hipLaunchKernelGGL(k_relabel, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, part, side.p, dnew.p, dsplit.p,
                           n);
        KMP_LAUNCH_CHECK();
    }
    bt = std::move(nt);
    return calls;
}

void project(Ctx& c, const int32_t* coarse_part, const int32_t* map, int32_t* fine_part, int32_t n)
{
    if (n <= 0) return;
    ProfScope ps(c, KMP_PROF_PROJECT);
    hipLaunchKernelGGL(k_project, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, coarse_part, map, fine_part, n);
    KMP_LAUNCH_CHECK();
}

void project_jobs(Ctx& c, const int32_t* coarse_part, const int32_t* map, const int32_t* remap, const int32_t* gid,
                  const int32_t* start_block, int32_t* fine_part, int32_t n)
{
    if (n <= 0) return;
    ProfScope ps(c, KMP_PROF_PROJECT);
    hipLaunchKernelGGL(k_project_jobs, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, coarse_part, map, remap, gid,
                       start_block, fine_part, n);
    KMP_LAUNCH_CHECK();
}

void block_weights(Ctx& c, const DGraph& g, const int32_t* part, int32_t nb, int64_t* wt)
{
    c.zero(wt, sizeof(int64_t) * (size_t)nb);
    if (g.n <= 0) return;
    hipLaunchKernelGGL(k_block_weights, dim3(grid_for(g.n, kBlock, 256)), dim3(kBlock), 0, c.stream, part, g.vwgt,
                       g.n, nb, wt);
    KMP_LAUNCH_CHECK();
}

namespace {
// k_cut then k_cut_runs for the long rows (their runs listed by k_cut)
void launch_cut(Ctx& c, const DGraph& g, const int32_t* part, const int32_t* gid, int64_t* out)
{
    const int64_t cap = g.m / (kCutLight / 2) + 1;  // runs: rows above kCutLight entries hold < m / 128 of them
    DBuf<int2> runs(c, (size_t)cap);
    DBuf<int32_t> nruns(c, 1);
    c.zero(nruns.p, sizeof(int32_t));
    hipLaunchKernelGGL(k_cut, dim3(grid_for(g.n, kBlock, 1024)), dim3(kBlock), 0, c.stream, g.xadj, g.adjncy,
                       g.adjwgt, part, gid, g.n, out, runs.p, nruns.p);
    KMP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cut_runs, dim3(grid_for(cap, 1, 4096)), dim3(kBlock), 0, c.stream, g.xadj, g.adjncy,
                       g.adjwgt, part, gid, out, runs.p, nruns.p);
    KMP_LAUNCH_CHECK();
}
}  // namespace

void edge_cut_launch(Ctx& c, const DGraph& g, const int32_t* part)
{
    c.zero_spread(SP_CUT);
    if (g.n <= 0) return;
    launch_cut(c, g, part, nullptr, c.spread(SP_CUT));
}

int64_t edge_cut(Ctx& c, const DGraph& g, const int32_t* part)
{
    if (g.n <= 0) return 0;
    edge_cut_launch(c, g, part);
    return c.read_spread(SP_CUT) / 2;
}

void edge_cut_jobs(Ctx& c, const DGraph& g, const int32_t* part, const int32_t* gid, int32_t njobs,
                   std::vector<int64_t>& out)
{
    out.assign(njobs, 0);
    if (g.n <= 0) return;
    DBuf<int64_t> d(c, (size_t)njobs);
    c.zero(d.p, sizeof(int64_t) * njobs);
    launch_cut(c, g, part, gid, d.p);
    c.read(out.data(), d.p, sizeof(int64_t) * njobs);
    for (auto& x : out) x /= 2;
}

}  // namespace kmp
