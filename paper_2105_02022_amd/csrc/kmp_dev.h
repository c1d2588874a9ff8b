// Internal header of libkmp (gfx950).  Device helpers, the per-call context
// and declarations of the building blocks shared by the .hip translation
// units.  Nothing here is part of the public ABI (include/kmp.h).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdio>
#include <cstring>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/kmp.h"

namespace kmp {

// ---------------------------------------------------------------- constants
// Result-affecting constants of the deterministic reading (changing any of
// them changes partitions).
constexpr int kC = 160;              // contraction limit C (Alg. 1)
constexpr int kRounds = 5;           // LP rounds (Sec. 5.1, Sec. 5.3)
constexpr int kSub = 4;              // sub-rounds per LP round
constexpr int kSeeds = 8;            // GGG runs per block (Alg. 2 "R bipartitions")
constexpr int kFmMaxPasses = 16;     // largest accepted number of 2-way FM passes
constexpr int64_t kPPM = 1000000;    // epsilon fixed point
constexpr int kMaxLevels = 64;
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kPhi = 0x9E3779B9u;
enum : uint32_t { TAG_SUB = 1, TAG_CL = 2, TAG_REF = 3, TAG_BAL = 4, TAG_GGG = 5, TAG_BFS = 6, TAG_RND = 7 };

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& what) : std::runtime_error(what), code(c) {}
};

#define KMP_HIP(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            if (e_ == hipErrorOutOfMemory) throw ::kmp::Error(KMP_ENOMEM, hipGetErrorString(e_)); \
            throw ::kmp::Error(KMP_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));      \
        }                                                                                          \
    } while (0)

#define KMP_LAUNCH_CHECK() KMP_HIP(hipGetLastError())

// ---------------------------------------------------------------- hashing
// Tie-break hash of the deterministic reading: fmix32 is MurmurHash3's 32-bit
// finaliser; H(seed; a_1..a_t) folds fmix32 over the arguments, argument i
// offset by i * 0x9E3779B9.  The host computes the fold over the leading,
// call-invariant arguments ("prefix"); kernels finish it with hash_step.
__host__ __device__ inline uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

__host__ __device__ inline uint32_t hash_step(uint32_t h, uint32_t a, uint32_t i)
{
    return fmix32(h ^ (a + i * kPhi));
}

inline uint32_t hash_prefix(uint64_t seed, std::initializer_list<uint32_t> args)
{
    uint32_t h = fmix32((uint32_t)seed) ^ fmix32((uint32_t)(seed >> 32) + kPhi);
    uint32_t i = 1;
    for (uint32_t a : args) h = hash_step(h, a, i++);
    return h;
}

// H over (seed; a1, a2, a3) from the seed part of the prefix (kernels of a
// batch finish per-job prefixes themselves).
__host__ __device__ inline uint32_t hash3(uint32_t hseed, uint32_t a1, uint32_t a2, uint32_t a3)
{
    return hash_step(hash_step(hash_step(hseed, a1, 1), a2, 2), a3, 3);
}

inline uint32_t seed_hash(uint64_t seed) { return hash_prefix(seed, {}); }

// ---------------------------------------------------------------- device misc
__device__ inline uint64_t ballot64(bool p) { return __ballot(p); }

__device__ inline int lane_id() { return __lane_id(); }

template <typename T>
__device__ inline T shfl_xor(T v, int mask, int width = 64)
{
    return __shfl_xor(v, mask, width);
}

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int mask, int width = 64)
{
    uint32_t lo = __shfl_xor((uint32_t)v, mask, width);
    uint32_t hi = __shfl_xor((uint32_t)(v >> 32), mask, width);
    return ((uint64_t)hi << 32) | lo;
}

// Wavefront max / min of a 64-bit key without LDS traffic: DPP moves within
// each row of 16 lanes (quad swaps, half-row and row mirrors), then the four
// row results through readlane.  Every lane of the wavefront must be active;
// the result is uniform.
template <int CTRL>
__device__ inline uint64_t dpp_u64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t readlane_u64(uint64_t v, int lane)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t wave_max_u64(uint64_t v)
{
    uint64_t o;
    o = dpp_u64<0xB1>(v);   // quad_perm [1,0,3,2]
    v = o > v ? o : v;
    o = dpp_u64<0x4E>(v);   // quad_perm [2,3,0,1]
    v = o > v ? o : v;
    o = dpp_u64<0x141>(v);  // row_half_mirror
    v = o > v ? o : v;
    o = dpp_u64<0x140>(v);  // row_mirror
    v = o > v ? o : v;
    const uint64_t a = readlane_u64(v, 0), b = readlane_u64(v, 16), c = readlane_u64(v, 32), d = readlane_u64(v, 48);
    const uint64_t ab = a > b ? a : b, cd = c > d ? c : d;
    return ab > cd ? ab : cd;
}

__device__ inline uint64_t wave_min_u64(uint64_t v)
{
    return ~wave_max_u64(~v);
}

// Wavefront max of 32 bits in DPP steps only: within rows of 16 lanes (quad
// swaps, half-row and row mirrors), then row_bcast:15 into rows 1 and 3 and
// row_bcast:31 into rows 2 and 3, so lane 63 holds the maximum.  Every lane
// must be active.
template <int CTRL, int ROWS>
__device__ inline uint32_t dpp_max_step(uint32_t v)
{
    // lanes the step does not write read 0, the identity of the maximum
    const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false);
    return o > v ? o : v;
}

__device__ inline uint32_t wave_max_u32_dpp(uint32_t v)
{
    v = dpp_max_step<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v = dpp_max_step<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v = dpp_max_step<0x141, 0xF>(v);  // row_half_mirror
    v = dpp_max_step<0x140, 0xF>(v);  // row_mirror
    v = dpp_max_step<0x142, 0xA>(v);  // row_bcast:15
    v = dpp_max_step<0x143, 0xC>(v);  // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Sum over groups of WIDTH = 16 (one row) or 64 lanes in DPP steps: row
// butterflies (quad swaps, half-row and row mirrors), then for 64 lanes
// row_bcast:15 and row_bcast:31 and lane 63's total to every lane.  Every
// lane of the group ends with the group's sum; every lane must be active.
template <int CTRL, int ROWS>
__device__ inline uint32_t dpp_add_step(uint32_t v)
{
    // lanes the step does not write read 0, the identity of the sum
    return v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false);
}

template <int WIDTH>
__device__ inline uint32_t group_sum_u32(uint32_t v)
{
    static_assert(WIDTH == 16 || WIDTH == 64, "DPP groups are rows or the wavefront");
    v = dpp_add_step<0xB1, 0xF>(v);
    v = dpp_add_step<0x4E, 0xF>(v);
    v = dpp_add_step<0x141, 0xF>(v);
    v = dpp_add_step<0x140, 0xF>(v);
    if (WIDTH == 64) {
        v = dpp_add_step<0x142, 0xA>(v);
        v = dpp_add_step<0x143, 0xC>(v);
        v = (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
    }
    return v;
}

// Wavefront max of a 64-bit key in two 32-bit passes: the largest high word,
// then the largest low word among the lanes holding it (the same order as a
// 64-bit comparison).  Every lane must be active; the result is uniform.
__device__ inline uint64_t wave_max_u64_split(uint64_t v)
{
    const uint32_t hi = wave_max_u32_dpp((uint32_t)(v >> 32));
    const uint32_t lo = wave_max_u32_dpp((uint32_t)(v >> 32) == hi ? (uint32_t)v : 0u);
    return ((uint64_t)hi << 32) | lo;
}

// LDS slot for a key in a table of 2^bits slots (multiplicative hashing).
__device__ inline uint32_t slot_of(uint32_t key, int bits)
{
    return (key * 0x9E3779B1u) >> (32 - bits);
}

constexpr int kBlock = 256;

// XCD-aware work mapping.  Workgroups are dispatched round-robin over the 8
// XCDs of the chip (physical block b runs on XCD b % 8) and every XCD has its
// own L2.  Renumbering so that XCD x owns one contiguous range of logical
// blocks keeps neighbouring nodes (which share label / weight cache lines) on
// one L2.  Bijective on [0, gridDim.x).
constexpr uint32_t kXcds = 8;
__device__ inline uint32_t xcd_block()
{
    const uint32_t b = blockIdx.x, G = gridDim.x;
    const uint32_t q = G / kXcds, r = G % kXcds;
    const uint32_t x = b % kXcds, k = b / kXcds;
    return x * q + (x < r ? x : r) + k;
}

// Blocks for `items` work items at `per_block` items per block.  The default
// cap only keeps the grid inside HIP's limits: kernels written as one item per
// thread (no grid-stride loop) rely on covering every item, and batches reach
// 2^31 entries.  Pass a small cap only to kernels with grid-stride loops.
inline unsigned grid_for(int64_t items, int per_block = kBlock, unsigned cap = 0x7FFFFFFFu)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > (int64_t)cap) g = cap;
    return (unsigned)g;
}

// Workgroup size for a launch of `items` one-per-lane gathers.  A gather-heavy
// wave is limited by the L1 request rate of its compute unit, so launches of
// fewer than 64 Ki items use narrower workgroups: their waves then spread over
// all 256 compute units instead of stacking four to a unit on a few of them.
inline int spread_block(int64_t items)
{
    return items >= 256 * 256 ? 256 : items >= 256 * 128 ? 128 : 64;
}

// ---------------------------------------------------------------- profiling
// HIP events around launches of selected kernel classes (when enabled).
struct Prof {
    struct Rec {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    uint32_t mask = 0;  // classes to time (0: all)
    ~Prof();
};

// Spread counters: every logical counter owns kSpreadSlots slots, each on a
// 128-byte line of its own (kSpreadStride words apart); a block (or wavefront)
// adds to one slot and the host sums the counter's kSpreadWords words (the
// words between the slots stay 0).  Atomics on one line serialise in the L2,
// so a hot counter's adds spread over kSpreadSlots lines; kernels with many
// waves add once per block.
constexpr int kSpreadSlots = 8;
constexpr int kSpreadStride = 16;
constexpr int kSpreadWords = kSpreadSlots * kSpreadStride;
enum SpreadCounter {
    SP_RATED = 0,           // LP rated directed entries
    SP_BYTES = 1,           // + class: algorithmic bytes per profiling class (16)
    SP_NONEMPTY = 17,
    SP_CUT = 18,
    SP_VSUM = 19,
    SP_ESUM = 20,
    SP_BALMOVES = 21,
    SP_COUNT = 24
};
__device__ inline void spread_add(int64_t* base, int64_t v)
{
    const uint32_t slot = (blockIdx.x + (threadIdx.x >> 6)) & (kSpreadSlots - 1);
    atomicAdd((unsigned long long*)&base[slot * kSpreadStride], (unsigned long long)v);
}

// out[j] += x for every lane with job j >= 0.  Node ids are grouped by job, so
// a wavefront mostly holds one job: then one lane adds the wave's sum.  Every
// lane of the wavefront must call this.
__device__ inline void job_add(int64_t* out, int32_t j, int64_t x)
{
    const uint64_t valid = __ballot(j >= 0);
    if (!valid) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((unsigned long long)valid) - 1;
    const int32_t jl = __shfl(j, leader, 64);
    if (__ballot(j >= 0 && j != jl) == 0) {
        int64_t sum = j >= 0 ? x : 0;
        for (int d = 32; d > 0; d >>= 1) sum += __shfl_xor(sum, d, 64);
        if (lane == leader && sum) atomicAdd((unsigned long long*)&out[jl], (unsigned long long)sum);
    } else if (j >= 0 && x) {
        atomicAdd((unsigned long long*)&out[j], (unsigned long long)x);
    }
}

// ---------------------------------------------------------------- tuning
// Output-invariant launch choices (kmp_tuning), process-wide.
struct Tuning {
    int32_t small_level_n = 8192;  // one-workgroup LP up to this many nodes (-1 never)
    int32_t cut[4] = {16, 64, 512, 4096};  // rating tiers: largest degree of tiers 0..3
    int32_t hub_ts = 4096;                 // LDS table slots of a hub's label partition
};
bool tuning_valid(const Tuning& t);
Tuning tuning_get();
void tuning_set(const Tuning& t);

// ---------------------------------------------------------------- context
// One per library call: the stream, a pinned host buffer for scalar
// read-backs and stream-ordered device allocations released on exit.
class Ctx {
  public:
    explicit Ctx(hipStream_t s);
    // Arena mode: every device buffer of the call is carved from
    // [arena, arena + arena_bytes), a region the caller owns; nothing is
    // allocated on the device or pinned on the host, reads and writes are
    // stream-ordered copies to and from the caller's host memory followed by
    // a stream synchronisation, and buffers are cleared by fill kernels.  A
    // call that needs more than the region fails with KMP_ENOMEM.
    Ctx(hipStream_t s, void* arena, size_t arena_bytes);
    ~Ctx();
    Ctx(const Ctx&) = delete;
    Ctx& operator=(const Ctx&) = delete;

    hipStream_t stream;

    void* alloc_bytes(size_t bytes);
    template <typename T>
    T* alloc(size_t count)
    {
        return static_cast<T*>(alloc_bytes(sizeof(T) * (count > 0 ? count : 1)));
    }
    void free(void* p);
    void zero(void* p, size_t bytes);
    void sync();

    // Copy `bytes` device bytes into pinned host memory and wait.
    void read(void* host, const void* dev, size_t bytes);
    void write(void* dev, const void* host, size_t bytes);
    template <typename T>
    T read1(const T* dev)
    {
        T v;
        read(&v, dev, sizeof(T));
        return v;
    }
    // A small device scratch of 64 x int64 counters (zeroed on request).
    int64_t* counters();
    void zero_counters();
    // Spread counters (zeroed when first used in a call).
    int64_t* spread(int idx);
    void zero_spread(int idx);
    int64_t read_spread(int idx);

    Prof* prof = nullptr;  // profiling enabled when non-null
    bool force_exact = false;    // LP: contended sub-rounds take the exact path
    bool plain_loads = false;    // lane rating: plain loads instead of buffer loads
    int32_t fm_passes = 0;       // 2-way FM passes after every GGG growth
    bool ip_pool = false;        // initial bipartitioning also runs BFS and random growths
    bool adaptive_eps = false;   // bipartition sides bounded by the adaptive imbalance
    bool pq_balance = false;     // balancing by the queue balancer
    bool ip_multilevel = false;  // initial bipartitioning coarsens each block's subgraph first
    int32_t async_lp = 0;        // LP: 0 deterministic sub-rounds, 1 asynchronous, 2 asynchronous one node
                                 // per launch in visit order (the one-processing-element execution)
    int32_t small_level_n = 0;   // LP: one-workgroup levels up to this size (0: tune's, < 0 never)
    Tuning tune;                 // the process-wide tuning when the call started
    int prof_begin(int cls);
    void prof_end(int idx);
    // Events for one launch of class cls (false: not timed).  The caller
    // passes them to hipExtLaunchKernelGGL, which stamps the kernel's own start
    // and end (the duration a profiler reports for the dispatch).
    bool prof_pair(int cls, hipEvent_t& a, hipEvent_t& b);
    // Resolve the recorded events into per-class launches / ms and read the
    // per-class algorithmic byte counters.
    void prof_collect(int64_t* launches, double* ms, int64_t* bytes);
    // Device workspace taken so far (capacities of the blocks obtained).
    size_t workspace_taken() const { return ws_taken_; }

  private:
    // Device memory comes from a process-wide caching pool (per device):
    // blocks freed during the call are reused by later allocations of the
    // same call (stream order makes that safe) and return to the shared pool
    // when the call ends, after the stream has drained.
    int device_ = 0;
    size_t ws_limit_ = 0;  // KMP_WORKSPACE_LIMIT: largest workspace this call may take (0: none)
    size_t ws_taken_ = 0;  // capacity of the blocks taken by this call so far
    char* arena_ = nullptr;    // arena mode: the caller's region (nullptr: the caching pool)
    size_t arena_bytes_ = 0;
    void* arena_take(size_t cap);
    std::vector<std::pair<void*, size_t>> live_;   // (block, capacity) in use
    std::vector<std::pair<void*, size_t>> freed_;  // freed during this call
    // Pinned host staging: writes are enqueued without waiting; the chunks
    // are recycled when the call ends.
    std::vector<std::pair<void*, size_t>> pinned_chunks_;
    size_t pinned_used_ = 0;
    void* read_buf_ = nullptr;  // pinned: a flag word, then the data of the last read-back
    size_t read_bytes_ = 0;
    uint32_t read_seq_ = 0;
    int64_t* counters_ = nullptr;
    int64_t* spread_ = nullptr;
    void* stage(size_t bytes);
};

struct ProfScope {
    Ctx& c;
    int idx;
    ProfScope(Ctx& ctx, int cls) : c(ctx), idx(ctx.prof_begin(cls)) {}
    ~ProfScope() { c.prof_end(idx); }
};

// Launch on c.stream; when class cls is being timed, the kernel's own start
// and end are stamped into the class's events (hipExtLaunchKernelGGL).
#define KMP_LAUNCH_TIMED(c, cls, kernel, grid, block, shmem, ...)                                          \
    do {                                                                                                   \
        hipEvent_t ea_, eb_;                                                                               \
        if ((c).prof_pair((cls), ea_, eb_))                                                                \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, (c).stream, ea_, eb_, 0, __VA_ARGS__);        \
        else                                                                                               \
            hipLaunchKernelGGL(kernel, grid, block, shmem, (c).stream, __VA_ARGS__);                        \
        KMP_LAUNCH_CHECK();                                                                                \
    } while (0)

// RAII device buffer bound to a context.
template <typename T>
struct DBuf {
    Ctx* ctx = nullptr;
    T* p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(Ctx& c, size_t count) : ctx(&c), p(c.alloc<T>(count)), n(count) {}
    DBuf(DBuf&& o) noexcept : ctx(o.ctx), p(o.p), n(o.n) { o.p = nullptr; }
    DBuf& operator=(DBuf&& o) noexcept
    {
        reset();
        ctx = o.ctx;
        p = o.p;
        n = o.n;
        o.p = nullptr;
        return *this;
    }
    ~DBuf() { reset(); }
    void reset()
    {
        if (p && ctx) ctx->free(p);
        p = nullptr;
        n = 0;
    }
    T* get() const { return p; }
    operator T*() const { return p; }
};

// ---------------------------------------------------------------- graph view
struct DGraph {
    int32_t n = 0;
    int64_t m = 0;
    const int32_t* xadj = nullptr;
    const int32_t* adjncy = nullptr;
    const int32_t* vwgt = nullptr;    // NULL = unit
    const int32_t* adjwgt = nullptr;  // NULL = unit
};

// Owned coarse graph.
struct OwnedGraph {
    DBuf<int32_t> xadj, adjncy, vwgt, adjwgt;
    DGraph view(int32_t n, int64_t m) const
    {
        DGraph g;
        g.n = n;
        g.m = m;
        g.xadj = xadj.p;
        g.adjncy = adjncy.p;
        g.vwgt = vwgt.p;
        g.adjwgt = adjwgt.p;
        return g;
    }
};

// ---------------------------------------------------------------- primitives
// prims.hip
// Exclusive prefix sum of n int32 values into out (may alias in); returns the
// total through *total_dev (device, may be NULL).
void scan_excl_i32(Ctx& c, const int32_t* in, int32_t* out, int64_t n, int32_t* total_dev);
// Inclusive prefix sum of n int64 values.
void scan_incl_i64(Ctx& c, const int64_t* in, int64_t* out, int64_t n);
// Inclusive max-scan of n int32 values.
void scan_incl_max_i32(Ctx& c, const int32_t* in, int32_t* out, int64_t n);
// Stable LSD radix sort of (key, value) pairs by key, keys < 2^key_bits (the
// alt buffers are scratch of the same size).  With out_keys / out_vals NULL
// the result ends in keys / vals; otherwise they receive the buffers that hold
// it (the alt ones after an odd number of passes) and nothing is copied.
void radix_sort_pairs(Ctx& c, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, int64_t n,
                      int key_bits, uint32_t** out_keys = nullptr, uint32_t** out_vals = nullptr);
// m = xadj[n] and the largest degree of a CSR, in one read-back (zeroed2: two
// zeroed int32 of scratch, or NULL to allocate and clear them here).
void entries_and_max_degree(Ctx& c, const int32_t* xadj, int32_t n, int64_t& m, int32_t& maxdeg,
                            int32_t* zeroed2 = nullptr);
// Several byte fills in one launch (at most kMaxFills buffers).
constexpr int kMaxFills = 8;
struct ByteFill {
    void* p;
    int64_t bytes;
    uint8_t byte;
};
void fill_bytes_many(Ctx& c, std::initializer_list<ByteFill> fills);
void fill_i32(Ctx& c, int32_t* p, int32_t v, int64_t n);
void fill_u8(Ctx& c, uint8_t* p, uint8_t v, int64_t n);
void fill_i64(Ctx& c, int64_t* p, int64_t v, int64_t n);
inline void set_i64(Ctx& c, int64_t* p, int64_t v) { fill_i64(c, p, v, 1); }
void iota_i32(Ctx& c, int32_t* p, int64_t n);
// Sum of node / edge weights (int64; NULL weights count 1 each).
// Allow `bytes` of dynamic LDS for kernel `fn` on the current device (once per
// kernel and device; throws on failure).
void allow_lds(const void* fn, int bytes);

// Read several device int64 ranges (pointer, count) with one read-back, in order.
constexpr int kMaxReadSegs = 4;
void read_segments(Ctx& c, const std::vector<std::pair<const int64_t*, int32_t>>& segs, int64_t* host);
int64_t node_weight_sum(Ctx& c, const int32_t* vwgt, int32_t n);
int64_t edge_weight_sum(Ctx& c, const int32_t* adjwgt, int64_t m);
int bits_for(uint64_t max_value);

// ---------------------------------------------------------------- batches
// The jobs of a batch run level by level as one disjoint union of their level
// graphs, concatenated in job order.  gid[v] is the job of node v; per-job
// tables are indexed by job.  Hashes take job-local arguments (a node or label
// minus its job's offset, each job's own seed), so every job's result is the
// one it gets alone.  One graph: gid = NULL (every node is job 0, offset 0).
struct JobTabs {
    const int32_t* gid = nullptr;     // [n] job of every node
    const uint32_t* ghash = nullptr;  // [jobs] seed_hash of every job's seed
    const int32_t* noff = nullptr;    // [jobs] first node of every job at this level
};

// ---------------------------------------------------------------- LP (lp.hip)
struct LPState {
    int32_t* label;     // [n]
    int64_t* wt;        // [nlab]
    int32_t nlab;
    const int64_t* cap_vec;  // [nlab] or NULL
    int64_t cap_scalar;
    uint32_t* fav;      // [n] or NULL (clustering only)
    uint32_t tag;
    // batches: label offset of every job (node offset for clustering, block
    // offset for refinement) and per-job scalar caps (clustering) or NULL
    JobTabs jt = {};
    const int32_t* loff = nullptr;
    const int64_t* gcap = nullptr;
    // batches: jobs whose LP runs in the one-workgroup kernel (one workgroup
    // each), with their first node and node count at this level
    int32_t njobs = 0;
    std::vector<int32_t> small_jobs, small_start, small_count, small_loff, small_nlab;
    // when set, the one-workgroup LP adds its moves per round (and the largest
    // round count) here instead of returning them: no read-back per call
    int64_t* moves_out = nullptr;  // [kRounds + 1], zeroed by the caller
};

// Largest level (nodes) of the one-workgroup LP for this call; -1: never.
int32_t small_limit(const Ctx& c);
// A job of `nodes` nodes and `labels` labels may run the one-workgroup LP
// (within the cut-off, and its state fits in LDS).
bool small_job_fits(const Ctx& c, int32_t nodes, int32_t labels);

struct LPStats {
    int64_t moves[kRounds] = {0, 0, 0, 0, 0};
    int32_t exact_subrounds = 0;  // sub-rounds finished on the exact admission path
    int32_t rounds = 0;
};

// Per-level schedule: nodes grouped by (degree tier, sub-round class); the
// segment of (tier t, class s) has index t * kSub + s.
constexpr int kTiers = 5;
constexpr int kSegs = kTiers * kSub;

struct LPSchedule {
    DBuf<int32_t> order;              // node ids grouped by (tier, class); ascending id inside a segment,
                                      // except that tier-0 segments list degrees <= 8 first
    int32_t off[kSegs + 1] = {};      // segment start in `order`; off[kSegs] = scheduled nodes
    int32_t cnt[kSegs] = {};          // segment size
    DBuf<int32_t> segtab;             // device copy: [kSegs offsets][kSegs counts]
    int32_t hub_start = 0;            // hubs (last tier) of all classes are contiguous from here
    DBuf<int64_t> hub_slot_off;       // per hub: start of its global hash table
    int64_t hub_slots_total = 0;
    std::vector<int32_t> job_maxdeg;  // batches: largest degree of every job's scheduled nodes (0: none)
    int32_t class_size(int s) const
    {
        int32_t t = 0;
        for (int q = 0; q < kTiers; ++q) t += cnt[q * kSub + s];
        return t;
    }
};

// Schedule of the nodes of one level.  Batches: per-job seeds through jt, and
// only the nodes of jobs with gpart[job] != 0 are scheduled (gpart NULL: all).
void lp_build_schedule(Ctx& c, const DGraph& g, int32_t level, uint64_t seed, LPSchedule& sched,
                       const JobTabs& jt = {}, const uint8_t* gpart = nullptr, int32_t njobs = 0);
// Visit-order schedule of the asynchronous LP: segments (tier, class) as in
// lp_build_schedule, each in (degree bucket, id) order, tiers aligned to
// buckets.  Only the nodes of jobs with gpart[job] != 0 are scheduled (gpart
// NULL: all).
void lp_build_async_schedule(Ctx& c, const DGraph& g, int32_t level, uint64_t seed, LPSchedule& sched,
                             const JobTabs& jt = {}, const uint8_t* gpart = nullptr);
// Rated entries accumulate in the context's SP_RATED spread counter.
// With c.async_lp set, sched must be an asynchronous schedule.
// sched NULL: a single graph whose level the caller found small (at most the
// one-workgroup cut-off, no degree above the tier-1 cut-off, state fits LDS).
LPStats lp_run(Ctx& c, const DGraph& g, int32_t level, uint64_t seed, const LPSchedule* sched, LPState& st);
int64_t lp_subround(Ctx& c, const DGraph& g, int32_t level, int32_t round, int32_t s, uint64_t seed,
                    const LPSchedule& sched, LPState& st, const uint8_t* active, uint8_t* moved);

// Balance-mode rating (same kernels): for every node of an overloaded block,
// the adjacent non-overloaded block with the largest connection that fits
// (bal_t, -1 if none) and d = conn(target) - conn(own block) (bal_d; -conn(own)
// when there is no target).
// Batches: jt and the per-job block offsets boff make the hash job-local.
void rate_for_balance(Ctx& c, const DGraph& g, int32_t level, uint64_t seed, int32_t round,
                      const LPSchedule& sched, const int32_t* part, const int64_t* wt, const int64_t* cap,
                      const uint8_t* over, int32_t* bal_t, int64_t* bal_d, const JobTabs& jt = {},
                      const int32_t* boff = nullptr);

// ---------------------------------------------------------------- coarsening (coarsen.hip)
// Two-hop of one graph; returns the number of merges when `count` is set
// (one more read-back), else 0.  nonempty_out (may be NULL) receives the
// number of non-empty labels when no merge ran (they are then unchanged),
// else -1.
int64_t two_hop(Ctx& c, const DGraph& g, int64_t U, int32_t* label, int64_t* cw, const uint32_t* fav,
                bool count = true, int32_t* nonempty_out = nullptr);
// Two-hop of a batch: per-job bounds gU, merge limits glimit and node range
// ends gend (device, by job; jobs with limit 0 do not take part).
void two_hop_jobs(Ctx& c, const DGraph& g, const JobTabs& jt, const int64_t* gU, const int64_t* glimit,
                  const int32_t* gend, int32_t njobs, int32_t* label, int64_t* cw, const uint32_t* fav);
int32_t count_nonempty(Ctx& c, const int64_t* cw, int32_t n);
// Non-empty labels of every job (labels of job j are its node ids).
void count_nonempty_jobs(Ctx& c, const int64_t* cw, int32_t n, const JobTabs& jt, int32_t njobs,
                         std::vector<int64_t>& out);
// Contract; returns coarse sizes; allocates the coarse graph in `out`.
// Batches: only nodes of jobs with gkeep[job] != 0 are contracted (the others
// get map = -1); coarse ids stay grouped by job.
// cid_in / nc_in: coarse ids and count from contract_ids, when the caller
// already computed them (its convergence test needs the count first).
// maxdeg (may be NULL) receives the coarse graph's largest degree.
void contract(Ctx& c, const DGraph& g, const int32_t* label, const int64_t* cw, int32_t* map, OwnedGraph& out,
              int32_t& cn, int64_t& cm, const JobTabs& jt = {}, const uint8_t* gkeep = nullptr,
              DBuf<int32_t>* cid_in = nullptr, int32_t nc_in = 0, int32_t* maxdeg = nullptr);
// Coarse id of every non-empty label (exclusive prefix of the non-empty
// flags, jobs with gkeep[job] == 0 excluded); returns their number (read
// back unless the caller already knows it: known >= 0).
int32_t contract_ids(Ctx& c, const DGraph& g, const int64_t* cw, DBuf<int32_t>& cid, const JobTabs& jt = {},
                     const uint8_t* gkeep = nullptr, int32_t known = -1);

// ---------------------------------------------------------------- IP (ip.hip)
// Block table of a level: blocks in job order, ascending `first` inside a job.
struct BlockTab {
    std::vector<int32_t> first, f, job;
    int32_t size() const { return (int32_t)first.size(); }
};
// One bipartitionBlocks round over the blocks with split[b] != 0 (f >= 2);
// the table is updated.  Per job: L_k (lk) and the seed part of the hash.
// Per job: what the adaptive imbalance of a bipartition needs (c(V), k, eps in ppm).
struct AdaptiveJob {
    int64_t cV;
    int32_t k;
    int64_t e;
};
// Side caps of a block of weight cB that is to end as f blocks, bounded by the
// adaptive imbalance (both 0 for an empty block, 2^62 when unbounded).
void adaptive_side_caps(const AdaptiveJob& j, int64_t cB, int32_t f, int64_t& cap0, int64_t& cap1);
// Validates and copies the initial-bipartitioning options (fm_passes, ip_pool, adaptive_eps).
int set_ip_options(Ctx& c, const kmp_options* opt);
// seeds64 (per job, the 64-bit seeds) is needed with c.ip_multilevel.
int32_t bipartition_round(Ctx& c, const DGraph& g, int32_t level, int32_t* part, BlockTab& bt,
                          const std::vector<uint8_t>& split, const std::vector<int64_t>& lk,
                          const std::vector<uint32_t>& hseed, const std::vector<AdaptiveJob>* adapt = nullptr,
                          const std::vector<uint64_t>* seeds64 = nullptr);
void project(Ctx& c, const int32_t* coarse_part, const int32_t* map, int32_t* fine_part, int32_t n);
// Batches: nodes with map >= 0 take remap[coarse block]; the others start in
// their job's single block start_block[job].
void project_jobs(Ctx& c, const int32_t* coarse_part, const int32_t* map, const int32_t* remap,
                  const int32_t* gid, const int32_t* start_block, int32_t* fine_part, int32_t n);
void block_weights(Ctx& c, const DGraph& g, const int32_t* part, int32_t nb, int64_t* wt);
int64_t edge_cut(Ctx& c, const DGraph& g, const int32_t* part);
// Enqueue the cut count into spread counter SP_CUT (twice the cut) without reading it.
void edge_cut_launch(Ctx& c, const DGraph& g, const int32_t* part);
// Cut of every job (gid by node).
void edge_cut_jobs(Ctx& c, const DGraph& g, const int32_t* part, const int32_t* gid, int32_t njobs,
                   std::vector<int64_t>& out);

// ---------------------------------------------------------------- balance (balance.hip)
// Balancer rounds.  Batches: bt.job gives every block's job, jt/boff make the
// hashes job-local and each job stops on its own (no overload, or a round
// without moves).
// hcap: the caps on the host when the caller has them (else they are read).
// sched builds (or returns) the level's schedule; it is called only when some
// block is overloaded.
int32_t balance(Ctx& c, const DGraph& g, int32_t level, const std::vector<uint64_t>& seeds,
                const std::function<const LPSchedule&()>& sched, int32_t* part, int64_t* wt, const BlockTab& bt,
                const int64_t* cap, const JobTabs& jt = {}, const int32_t* boff = nullptr,
                const std::vector<int64_t>* hcap = nullptr);
// The queue balancer (paper Sec. 5.3 queues; kmp_options.pq_balance), same arguments.
int32_t balance_pq(Ctx& c, const DGraph& g, int32_t level, const std::vector<uint64_t>& seeds,
                const std::function<const LPSchedule&()>& sched, int32_t* part, int64_t* wt, const BlockTab& bt,
                const int64_t* cap, const JobTabs& jt = {}, const int32_t* boff = nullptr,
                const std::vector<int64_t>* hcap = nullptr);

// ---------------------------------------------------------------- validation, batches (kmp.hip)
int validate_graph(Ctx& c, const DGraph& g);
// kmp_partition_batch on `stream` with errors mapped to status codes.
int run_batch(const kmp_graph_desc* graphs, int32_t count, kmp_job_result* results, hipStream_t stream,
              const kmp_options* opt, kmp_stats* stats);

}  // namespace kmp
