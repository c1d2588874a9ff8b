// Data-parallel building blocks: per-call context, prefix scans, stable LSD
// radix sort (wave-ballot ranking, 64-wide wavefronts), fills, reductions.
#include <chrono>
#include <cstdlib>
#include <map>
#include <mutex>

#include "kmp_dev.h"

namespace kmp {

// ================================================================ context
namespace {

// Process-wide cache of device blocks per device, keyed by capacity.
struct DevicePool {
    std::mutex mu;
    std::multimap<size_t, void*> free_blocks[64];
};
DevicePool& device_pool()
{
    static DevicePool* p = new DevicePool();  // lives until process exit
    return *p;
}

// Capacity class: multiples of 1/4 of the power of two below the request.
size_t capacity_for(size_t bytes)
{
    if (bytes <= 256) return 256;
    size_t p = 256;
    while (p < bytes) p <<= 1;
    const size_t half = p >> 1, step = half >> 2;
    size_t c = half;
    while (c < bytes) c += step;
    return c;
}

// Take a cached block of capacity in [cap, 2 cap) from `m`, if any.
void* take_block(std::multimap<size_t, void*>& m, size_t cap, size_t& got)
{
    auto it = m.lower_bound(cap);
    if (it == m.end() || it->first >= 2 * cap) return nullptr;
    void* p = it->second;
    got = it->first;
    m.erase(it);
    return p;
}

std::mutex g_pinned_mu;
std::vector<std::pair<void*, size_t>> g_pinned_free;

}  // namespace

namespace {
std::mutex g_tune_mu;
Tuning g_tune;
}  // namespace

bool tuning_valid(const Tuning& t)
{
    if (t.small_level_n < -1 || t.small_level_n > (1 << 30)) return false;
    const int32_t hi[4] = {16, 64, 512, 4096};
    int32_t lo = 1;
    for (int i = 0; i < 4; ++i) {
        if (t.cut[i] < lo || t.cut[i] > hi[i]) return false;
        lo = t.cut[i];
    }
    return t.hub_ts >= 64 && t.hub_ts <= 8192 && (t.hub_ts & (t.hub_ts - 1)) == 0;
}

Tuning tuning_get()
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tune;
}

void tuning_set(const Tuning& t)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune = t;
}

Ctx::Ctx(hipStream_t s) : stream(s), tune(tuning_get())
{
    if (hipGetDevice(&device_) != hipSuccess || device_ < 0 || device_ >= 64) device_ = 0;
    // a host-side cap on the workspace of one call, so tests can drive the
    // out-of-memory path without exhausting the device
    if (const char* lim = getenv("KMP_WORKSPACE_LIMIT")) {
        char* end = nullptr;
        const unsigned long long v = strtoull(lim, &end, 10);
        if (end != lim) ws_limit_ = (size_t)v;
    }
}

Ctx::Ctx(hipStream_t s, void* arena, size_t arena_bytes)
    : stream(s), tune(tuning_get()), arena_(static_cast<char*>(arena)), arena_bytes_(arena_bytes)
{
    if (hipGetDevice(&device_) != hipSuccess || device_ < 0 || device_ >= 64) device_ = 0;
}

// Bump allocation in the caller's region (256-byte aligned blocks); blocks
// freed during the call are reused through freed_ as in pool mode.
void* Ctx::arena_take(size_t cap)
{
    if (ws_taken_ + cap > arena_bytes_)
        throw Error(KMP_ENOMEM, "scratch region exhausted (" + std::to_string(ws_taken_ + cap) + " of " +
                                    std::to_string(arena_bytes_) + " bytes)");
    void* p = arena_ + ws_taken_;
    ws_taken_ += cap;
    return p;
}

Ctx::~Ctx()
{
    (void)hipStreamSynchronize(stream);
    if (arena_) return;  // the region stays the caller's; nothing was taken from the pools
    DevicePool& dp = device_pool();
    {
        std::lock_guard<std::mutex> lk(dp.mu);
        for (auto& b : live_) dp.free_blocks[device_].emplace(b.second, b.first);
        for (auto& b : freed_) dp.free_blocks[device_].emplace(b.second, b.first);
        if (counters_) dp.free_blocks[device_].emplace((size_t)512, (void*)counters_);
        if (spread_) dp.free_blocks[device_].emplace((size_t)SP_COUNT * kSpreadWords * 8, (void*)spread_);
    }
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    for (auto& c : pinned_chunks_) g_pinned_free.push_back(c);
    if (read_buf_) g_pinned_free.emplace_back(read_buf_, read_bytes_);
}

void* Ctx::alloc_bytes(size_t bytes)
{
    const size_t cap = capacity_for(bytes);
    size_t got = 0;
    // blocks freed earlier in this call first (same stream), then the shared pool
    for (size_t i = freed_.size(); i-- > 0;) {
        if (freed_[i].second >= cap && freed_[i].second < 2 * cap) {
            auto b = freed_[i];
            freed_[i] = freed_.back();
            freed_.pop_back();
            live_.push_back(b);
            return b.first;
        }
    }
    if (arena_) {
        const size_t cap256 = (cap + 255) & ~(size_t)255;  // keeps every block 256-byte aligned
        void* p = arena_take(cap256);
        live_.emplace_back(p, cap256);
        return p;
    }
    if (ws_limit_ && ws_taken_ + cap > ws_limit_)
        throw Error(KMP_ENOMEM, "device workspace above KMP_WORKSPACE_LIMIT (" + std::to_string(ws_taken_ + cap) +
                                    " bytes)");
    void* p = nullptr;
    {
        DevicePool& dp = device_pool();
        std::lock_guard<std::mutex> lk(dp.mu);
        p = take_block(dp.free_blocks[device_], cap, got);
    }
    if (!p) {
        got = cap;
        hipError_t e = hipMalloc(&p, cap);
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            // release cached blocks and retry once
            DevicePool& dp = device_pool();
            std::lock_guard<std::mutex> lk(dp.mu);
            for (auto& kv : dp.free_blocks[device_]) (void)hipFree(kv.second);
            dp.free_blocks[device_].clear();
            e = hipMalloc(&p, cap);
            if (e != hipSuccess || !p) {
                (void)hipGetLastError();
                throw Error(KMP_ENOMEM, "device workspace allocation failed (" + std::to_string(bytes) + " bytes)");
            }
        }
    }
    ws_taken_ += got;
    live_.emplace_back(p, got);
    return p;
}

void Ctx::free(void* p)
{
    if (!p) return;
    for (size_t i = live_.size(); i-- > 0;)
        if (live_[i].first == p) {
            freed_.push_back(live_[i]);
            live_[i] = live_.back();
            live_.pop_back();
            return;
        }
}

void Ctx::zero(void* p, size_t bytes)
{
    if (!bytes) return;
    if (arena_) fill_bytes_many(*this, {{p, (int64_t)bytes, 0}});
    else KMP_HIP(hipMemsetAsync(p, 0, bytes, stream));
}

void Ctx::sync() { KMP_HIP(hipStreamSynchronize(stream)); }

// Pinned staging for host-to-device copies: a bump arena over chunks that stay
// untouched until the call ends (the copies may still be in flight).
void* Ctx::stage(size_t bytes)
{
    bytes = (bytes + 255) & ~(size_t)255;
    if (!pinned_chunks_.empty() && pinned_used_ + bytes <= pinned_chunks_.back().second) {
        void* p = static_cast<char*>(pinned_chunks_.back().first) + pinned_used_;
        pinned_used_ += bytes;
        return p;
    }
    const size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
    void* chunk = nullptr;
    size_t got = 0;
    {
        std::lock_guard<std::mutex> lk(g_pinned_mu);
        for (size_t i = 0; i < g_pinned_free.size(); ++i)
            if (g_pinned_free[i].second >= want) {
                chunk = g_pinned_free[i].first;
                got = g_pinned_free[i].second;
                g_pinned_free[i] = g_pinned_free.back();
                g_pinned_free.pop_back();
                break;
            }
    }
    if (!chunk) {
        KMP_HIP(hipHostMalloc(&chunk, want, hipHostMallocDefault));
        got = want;
    }
    pinned_chunks_.emplace_back(chunk, got);
    pinned_used_ = bytes;
    return chunk;
}

namespace {
// Small read-backs: one wavefront copies the bytes into the pinned read buffer,
// makes them visible to the host (system-scope fence) and then sets the buffer's
// flag word to `seq`; the host spins on the flag instead of synchronising the
// stream (a kernel launch and a fence instead of a runtime copy and a wake-up).
// Seeing the flag also means every earlier command of the stream has finished.
__global__ __launch_bounds__(64) void k_readback(const char* __restrict__ src, char* __restrict__ dst,
                                                 uint32_t bytes, uint32_t* flag, uint32_t seq)
{
    if ((((uintptr_t)src | (uintptr_t)dst | (uintptr_t)bytes) & 3u) == 0) {
        const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
        uint32_t* d = reinterpret_cast<uint32_t*>(dst);
        for (uint32_t i = threadIdx.x; i < bytes / 4; i += 64) d[i] = s[i];
    } else {
        for (uint32_t i = threadIdx.x; i < bytes; i += 64) dst[i] = src[i];
    }
    __threadfence_system();
    if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

constexpr size_t kFlagBytes = 64;                 // the flag word's line at the start of the buffer
constexpr size_t kFlagReadMax = 4096 - kFlagBytes;  // larger reads take the runtime copy
}  // namespace

void Ctx::read(void* host, const void* dev, size_t bytes)
{
    if (!bytes) return;
    if (arena_) {
        KMP_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, stream));
        KMP_HIP(hipStreamSynchronize(stream));
        return;
    }
    if (read_bytes_ < bytes + kFlagBytes) {
        if (read_buf_) {
            std::lock_guard<std::mutex> lk(g_pinned_mu);
            g_pinned_free.emplace_back(read_buf_, read_bytes_);
        }
        read_buf_ = nullptr;
        const size_t want = bytes + kFlagBytes < 4096 ? 4096 : bytes + kFlagBytes;
        {
            std::lock_guard<std::mutex> lk(g_pinned_mu);
            for (size_t i = 0; i < g_pinned_free.size(); ++i)
                if (g_pinned_free[i].second >= want) {
                    read_buf_ = g_pinned_free[i].first;
                    read_bytes_ = g_pinned_free[i].second;
                    g_pinned_free[i] = g_pinned_free.back();
                    g_pinned_free.pop_back();
                    break;
                }
        }
        if (!read_buf_) {
            KMP_HIP(hipHostMalloc(&read_buf_, want, hipHostMallocDefault));
            read_bytes_ = want;
        }
        __atomic_store_n(static_cast<uint32_t*>(read_buf_), 0u, __ATOMIC_RELEASE);  // no stale flag value
    }
    char* data = static_cast<char*>(read_buf_) + kFlagBytes;
    if (bytes > kFlagReadMax) {
        KMP_HIP(hipMemcpyAsync(data, dev, bytes, hipMemcpyDeviceToHost, stream));
        KMP_HIP(hipStreamSynchronize(stream));
        memcpy(host, data, bytes);
        return;
    }
    uint32_t* flag = static_cast<uint32_t*>(read_buf_);
    const uint32_t want = ++read_seq_ ? read_seq_ : ++read_seq_;  // never 0 (the cleared value)
    hipLaunchKernelGGL(k_readback, dim3(1), dim3(64), 0, stream, static_cast<const char*>(dev), data,
                       (uint32_t)bytes, flag, want);
    KMP_LAUNCH_CHECK();
    // spin for a short wait; a long one (or an error) falls back to the stream
    // synchronisation, which also reports asynchronous errors
    const auto t0 = std::chrono::steady_clock::now();
    bool seen = false;
    for (uint32_t i = 1;; ++i) {
        if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) == want) {
            seen = true;
            break;
        }
        if ((i & 1023u) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(2)) break;
    }
    if (!seen) {
        KMP_HIP(hipStreamSynchronize(stream));
        if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) != want) throw Error(KMP_EHIP, "read-back flag not set");
    }
    memcpy(host, data, bytes);
}

void Ctx::write(void* dev, const void* host, size_t bytes)
{
    if (!bytes) return;
    if (arena_) {
        KMP_HIP(hipMemcpyAsync(dev, host, bytes, hipMemcpyHostToDevice, stream));
        KMP_HIP(hipStreamSynchronize(stream));  // the host buffer may be temporary
        return;
    }
    void* st = stage(bytes);
    memcpy(st, host, bytes);
    KMP_HIP(hipMemcpyAsync(dev, st, bytes, hipMemcpyHostToDevice, stream));
}

int64_t* Ctx::counters()
{
    if (!counters_ && arena_) {
        counters_ = static_cast<int64_t*>(arena_take(512));
        zero_counters();
    }
    if (!counters_) {
        size_t got = 0;
        void* p = nullptr;
        {
            DevicePool& dp = device_pool();
            std::lock_guard<std::mutex> lk(dp.mu);
            p = take_block(dp.free_blocks[device_], 512, got);
            if (p && got != 512) {  // keep only exact 512-byte blocks for counters
                dp.free_blocks[device_].emplace(got, p);
                p = nullptr;
            }
        }
        if (!p) KMP_HIP(hipMalloc(&p, 512));
        counters_ = static_cast<int64_t*>(p);
        zero_counters();
    }
    return counters_;
}

void Ctx::zero_counters() { zero(counters(), 64 * sizeof(int64_t)); }

int64_t* Ctx::spread(int idx)
{
    if (!spread_ && arena_) {
        const size_t bytes = (size_t)SP_COUNT * kSpreadWords * sizeof(int64_t);
        spread_ = static_cast<int64_t*>(arena_take((bytes + 255) & ~(size_t)255));
        zero(spread_, bytes);
    }
    if (!spread_) {
        const size_t bytes = (size_t)SP_COUNT * kSpreadWords * sizeof(int64_t);
        size_t got = 0;
        void* p = nullptr;
        {
            DevicePool& dp = device_pool();
            std::lock_guard<std::mutex> lk(dp.mu);
            p = take_block(dp.free_blocks[device_], bytes, got);
            if (p && got != bytes) {
                dp.free_blocks[device_].emplace(got, p);
                p = nullptr;
            }
        }
        if (!p) KMP_HIP(hipMalloc(&p, bytes));
        spread_ = static_cast<int64_t*>(p);
        zero(spread_, bytes);
    }
    return spread_ + (size_t)idx * kSpreadWords;
}

void Ctx::zero_spread(int idx) { zero(spread(idx), kSpreadWords * sizeof(int64_t)); }

int64_t Ctx::read_spread(int idx)
{
    int64_t v[kSpreadWords];
    read(v, spread(idx), sizeof(v));
    int64_t s = 0;
    for (int i = 0; i < kSpreadWords; ++i) s += v[i];
    return s;
}

// Events are recycled through a process-wide pool: creating an event costs far
// more host time than recording one.
namespace {
std::mutex g_event_mu;
std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event()
{
    {
        std::lock_guard<std::mutex> lk(g_event_mu);
        if (!g_event_pool.empty()) {
            hipEvent_t e = g_event_pool.back();
            g_event_pool.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    KMP_HIP(hipEventCreate(&e));
    return e;
}
}  // namespace

Prof::~Prof()
{
    std::lock_guard<std::mutex> lk(g_event_mu);
    for (auto& r : recs) {
        if (r.a) g_event_pool.push_back(r.a);
        if (r.b) g_event_pool.push_back(r.b);
    }
}

int Ctx::prof_begin(int cls)
{
    if (!prof || (prof->mask && !((prof->mask >> cls) & 1u))) return -1;
    Prof::Rec r{cls, take_event(), nullptr};
    KMP_HIP(hipEventRecord(r.a, stream));
    prof->recs.push_back(r);
    return (int)prof->recs.size() - 1;
}

bool Ctx::prof_pair(int cls, hipEvent_t& a, hipEvent_t& b)
{
    if (!prof || (prof->mask && !((prof->mask >> cls) & 1u))) return false;
    a = take_event();
    b = take_event();
    prof->recs.push_back(Prof::Rec{cls, a, b});
    return true;
}

void Ctx::prof_end(int idx)
{
    if (!prof || idx < 0) return;
    hipEvent_t b = take_event();
    KMP_HIP(hipEventRecord(b, stream));
    prof->recs[idx].b = b;
}

void Ctx::prof_collect(int64_t* launches, double* ms, int64_t* bytes)
{
    for (int i = 0; i < KMP_PROF_CLASSES; ++i) {
        launches[i] = 0;
        ms[i] = 0;
        bytes[i] = 0;
    }
    if (!prof) return;
    sync();
    for (auto& r : prof->recs) {
        if (!r.b) continue;
        float t = 0;
        KMP_HIP(hipEventElapsedTime(&t, r.a, r.b));
        launches[r.cls] += 1;
        ms[r.cls] += t;
    }
    // the classes' counters are adjacent: one read-back for all of them
    std::vector<int64_t> v((size_t)KMP_PROF_CLASSES * kSpreadWords);
    read(v.data(), spread(SP_BYTES), v.size() * sizeof(int64_t));
    for (int i = 0; i < KMP_PROF_CLASSES; ++i)
        for (int j = 0; j < kSpreadWords; ++j) bytes[i] += v[(size_t)i * kSpreadWords + j];
}

int bits_for(uint64_t max_value)
{
    int b = 0;
    while (b < 64 && (max_value >> b) != 0) ++b;
    return b;
}

// ================================================================ scans
namespace {

constexpr int SCAN_IT = 8;
constexpr int SCAN_TILE = kBlock * SCAN_IT;

struct OpAdd {
    template <typename T>
    __device__ T operator()(T a, T b) const { return a + b; }
};
struct OpMax {
    template <typename T>
    __device__ T operator()(T a, T b) const { return a > b ? a : b; }
};

template <typename T>
__device__ inline T shfl_up_t(T v, unsigned d) { return __shfl_up(v, d, 64); }

// One DPP step of a 32-bit wavefront scan: lanes without a source (or outside
// ROWS) combine with the identity.
template <int CTRL, int ROWS, typename T, typename Op>
__device__ inline T dpp_scan_step(T v, Op op, T identity)
{
    const T o = (T)__builtin_amdgcn_update_dpp((int)identity, (int)v, CTRL, ROWS, 0xF, false);
    return op(o, v);
}

// Inclusive wavefront scan: row_shr 1, 2, 4, 8 inside rows of 16 lanes, then
// row_bcast:15 into rows 1 and 3 and row_bcast:31 into rows 2 and 3 (32-bit
// values in DPP steps; wider ones through lane shuffles).  All lanes active.
template <typename T, typename Op>
__device__ inline T wave_scan_incl(T v, Op op, T identity)
{
    if constexpr (sizeof(T) == 4) {
        v = dpp_scan_step<0x111, 0xF>(v, op, identity);  // row_shr:1
        v = dpp_scan_step<0x112, 0xF>(v, op, identity);  // row_shr:2
        v = dpp_scan_step<0x114, 0xF>(v, op, identity);  // row_shr:4
        v = dpp_scan_step<0x118, 0xF>(v, op, identity);  // row_shr:8
        v = dpp_scan_step<0x142, 0xA>(v, op, identity);  // row_bcast:15
        v = dpp_scan_step<0x143, 0xC>(v, op, identity);  // row_bcast:31
    } else {
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            T y = shfl_up_t(v, d);
            if (lane >= d) v = op(y, v);
        }
    }
    return v;
}

// The value of the previous lane (lane 0: identity).
template <typename T>
__device__ inline T wave_prev(T v, T identity)
{
    if constexpr (sizeof(T) == 4) {
        return (T)__builtin_amdgcn_update_dpp((int)identity, (int)v, 0x138, 0xF, 0xF, false);  // wave_shr:1
    } else {
        const T p = __shfl_up(v, 1, 64);
        return (threadIdx.x & 63) ? p : identity;
    }
}

// Inclusive scan of one value per thread across a 256-thread block.
template <typename T, typename Op>
__device__ T block_scan_incl(T v, Op op, T* lds_waves, T identity)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_scan_incl<T, Op>(v, op, identity);
    if (lane == 63) lds_waves[w] = v;
    __syncthreads();
    if (w > 0) {
        T pre = lds_waves[0];
        for (int i = 1; i < w; ++i) pre = op(pre, lds_waves[i]);
        v = op(pre, v);
    }
    __syncthreads();
    return v;
}

// Per-tile reduction.
template <typename T, typename Op>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const T* __restrict__ in, int64_t n, T* __restrict__ partial,
                                                        T identity)
{
    __shared__ T lds[4];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IT;
    Op op;
    T acc = identity;
#pragma unroll
    for (int j = 0; j < SCAN_IT; ++j)
        if (base + j < n) acc = op(acc, in[base + j]);
    T tot = block_scan_incl<T, Op>(acc, op, lds, identity);
    if (threadIdx.x == kBlock - 1) partial[blockIdx.x] = tot;
}

// Scan tiles; tile t starts from carry partial_excl[t] (or identity when NULL).
// A single block may also process all tiles sequentially (`tiles_per_block`).
template <typename T, typename Op>
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const T* in, T* out, int64_t n, const T* __restrict__ partial_excl,
                                                       int tiles_per_block, bool inclusive, T identity,
                                                       T* total_out)
{
    __shared__ T lds[4];
    __shared__ T carry_s;
    Op op;
    T carry = identity;
    if (partial_excl) carry = partial_excl[blockIdx.x];
    for (int t = 0; t < tiles_per_block; ++t) {
        const int64_t tile = (int64_t)blockIdx.x * tiles_per_block + t;
        const int64_t base = tile * SCAN_TILE + (int64_t)threadIdx.x * SCAN_IT;
        if (tile * SCAN_TILE >= n) break;
        T v[SCAN_IT];
        T acc = identity;
#pragma unroll
        for (int j = 0; j < SCAN_IT; ++j) {
            v[j] = base + j < n ? in[base + j] : identity;
            acc = op(acc, v[j]);
        }
        T incl = block_scan_incl<T, Op>(acc, op, lds, identity);
        // exclusive prefix of this thread = incl - own (recompute via op: prefix before thread)
        T run = op(carry, incl);
        // derive this thread's exclusive start: shift inclusive totals by one thread
        T prev = wave_prev<T>(incl, identity);
        __shared__ T wave_last[4];
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        if (lane == 63) wave_last[w] = incl;
        __syncthreads();
        T start;
        if (lane > 0) start = op(carry, prev);
        else if (w > 0) start = op(carry, wave_last[w - 1]);
        else start = carry;
#pragma unroll
        for (int j = 0; j < SCAN_IT; ++j) {
            if (base + j < n) {
                T nx = op(start, v[j]);
                out[base + j] = inclusive ? nx : start;
                start = nx;
            } else {
                start = op(start, v[j]);
            }
        }
        if (threadIdx.x == kBlock - 1) carry_s = run;
        __syncthreads();
        carry = carry_s;
        __syncthreads();
    }
    if (total_out && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total_out = carry;
}

template <typename T>
__global__ void k_set_one(T* p, T v)
{
    if (threadIdx.x == 0) *p = v;
}

template <typename T, typename Op>
void scan_impl(Ctx& c, const T* in, T* out, int64_t n, bool inclusive, T identity, T* total_dev)
{
    if (n <= 0) {
        if (total_dev) {
            hipLaunchKernelGGL(k_set_one<T>, dim3(1), dim3(64), 0, c.stream, total_dev, identity);
            KMP_LAUNCH_CHECK();
        }
        return;
    }
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (tiles <= 8) {
        hipLaunchKernelGGL((k_scan_tiles<T, Op>), dim3(1), dim3(kBlock), 0, c.stream, in, out, n, (const T*)nullptr,
                           (int)tiles, inclusive, identity, total_dev);
        KMP_LAUNCH_CHECK();
        return;
    }
    DBuf<T> part(c, (size_t)tiles);
    hipLaunchKernelGGL((k_scan_reduce<T, Op>), dim3((unsigned)tiles), dim3(kBlock), 0, c.stream, in, n, part.p,
                       identity);
    KMP_LAUNCH_CHECK();
    // exclusive scan of the tile partials (recursive)
    scan_impl<T, Op>(c, part.p, part.p, tiles, false, identity, nullptr);
    hipLaunchKernelGGL((k_scan_tiles<T, Op>), dim3((unsigned)tiles), dim3(kBlock), 0, c.stream, in, out, n, part.p, 1,
                       inclusive, identity, total_dev);
    KMP_LAUNCH_CHECK();
}

}  // namespace

void scan_excl_i32(Ctx& c, const int32_t* in, int32_t* out, int64_t n, int32_t* total_dev)
{
    scan_impl<int32_t, OpAdd>(c, in, out, n, false, 0, total_dev);
}

void scan_incl_i64(Ctx& c, const int64_t* in, int64_t* out, int64_t n)
{
    scan_impl<int64_t, OpAdd>(c, in, out, n, true, (int64_t)0, nullptr);
}

void scan_incl_max_i32(Ctx& c, const int32_t* in, int32_t* out, int64_t n)
{
    scan_impl<int32_t, OpMax>(c, in, out, n, true, INT32_MIN, nullptr);
}

// ================================================================ radix sort
namespace {

constexpr int RS_IT = 8;
constexpr int RS_TILE = kBlock * RS_IT;

__global__ __launch_bounds__(kBlock) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                    int32_t* __restrict__ hist, int nblk)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    // every load issued together (indices clamped to the last key), then counted
    uint32_t kt[RS_IT];
#pragma unroll
    for (int j = 0; j < RS_IT; ++j) {
        const int64_t idx = base + (int64_t)j * kBlock + threadIdx.x;
        kt[j] = keys[idx < n ? idx : n - 1];
    }
#pragma unroll
    for (int j = 0; j < RS_IT; ++j)
        if (base + (int64_t)j * kBlock + threadIdx.x < n) atomicAdd(&cnt[(kt[j] >> shift) & 255u], 1u);
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = (int32_t)cnt[threadIdx.x];
}

// Stable scatter: element order inside a tile is (slot j, thread) = index order.
__global__ __launch_bounds__(kBlock) void k_rs_scatter(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                       uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                       int64_t n, int shift, const int32_t* __restrict__ offs,
                                                       int nblk)
{
    __shared__ uint32_t s_off[256];
    __shared__ uint32_t s_cnt[4][256];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    s_off[tid] = (uint32_t)offs[(int64_t)tid * nblk + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    const uint64_t lanes_below = (1ull << lane) - 1ull;
    // the tile's pairs loaded up front, indices clamped to the last pair so
    // that every load is issued together (invalid ones are never written)
    uint32_t kt[RS_IT], vt[RS_IT];
#pragma unroll
    for (int j = 0; j < RS_IT; ++j) {
        const int64_t idx = base + (int64_t)j * kBlock + tid;
        const int64_t ci = idx < n ? idx : n - 1;
        kt[j] = kin[ci];
        vt[j] = vin[ci];
    }
#pragma unroll
    for (int j = 0; j < RS_IT; ++j) {
#pragma unroll
        for (int i = 0; i < 4; ++i) s_cnt[i][tid] = 0;
        __syncthreads();
        const int64_t idx = base + (int64_t)j * kBlock + tid;
        const bool valid = idx < n;
        const uint32_t k = kt[j], v = vt[j];
        uint32_t d = (k >> shift) & 255u;
        uint64_t peers = ballot64(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bal = ballot64(bit);
            peers &= bit ? bal : ~bal;
        }
        const int rank = __popcll(peers & lanes_below);
        if (valid && rank == 0) s_cnt[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = s_off[d] + (uint32_t)rank;
            for (int ww = 0; ww < w; ++ww) pos += s_cnt[ww][d];
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        s_off[tid] += s_cnt[0][tid] + s_cnt[1][tid] + s_cnt[2][tid] + s_cnt[3][tid];
        __syncthreads();
    }
}

}  // namespace

// Small sorts in one workgroup: the pairs stay in LDS (two buffers) and every
// 4-bit digit pass is a stable counting sort: thread t owns a contiguous chunk,
// counts its digits into column t of a digit-major table, the table is scanned,
// and each thread places its chunk in order.  Same result as the multi-pass
// sort (a stable sort by key is unique).
constexpr int kRsSmallMax = 8192;
constexpr int kRsSmallThreads = kBlock;  // the block scan assumes kBlock threads

__global__ __launch_bounds__(kRsSmallThreads) void k_rs_small(uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                           int32_t n, int key_bits)
{
    extern __shared__ __align__(16) uint32_t s_rs[];
    uint32_t* bk[2] = {s_rs, s_rs + n};
    uint32_t* bv[2] = {s_rs + 2 * n, s_rs + 3 * n};
    uint32_t* cnt = s_rs + 4 * n;  // [16 digits][kRsSmallThreads]
    __shared__ uint32_t s_w4[kRsSmallThreads / 64];
    const int t = threadIdx.x;
    for (int32_t i = t; i < n; i += kRsSmallThreads) {
        bk[0][i] = keys[i];
        bv[0][i] = vals[i];
    }
    const int32_t chunk = (n + kRsSmallThreads - 1) / kRsSmallThreads;
    const int32_t lo = t * chunk < n ? t * chunk : n, hi = lo + chunk < n ? lo + chunk : n;
    int cur = 0;
    for (int shift = 0; shift < key_bits; shift += 4) {
        __syncthreads();
        uint32_t c16[16];
#pragma unroll
        for (int d = 0; d < 16; ++d) c16[d] = 0;
        for (int32_t i = lo; i < hi; ++i) {
            const uint32_t d = (bk[cur][i] >> shift) & 15u;
#pragma unroll
            for (int q = 0; q < 16; ++q) c16[q] += d == (uint32_t)q;
        }
#pragma unroll
        for (int d = 0; d < 16; ++d) cnt[d * kRsSmallThreads + t] = c16[d];
        __syncthreads();
        // exclusive scan of the 16 x kRsSmallThreads table in digit-major order:
        // thread t sums entries [16 t, 16 t + 16), the totals are scanned, then
        // each thread rewrites its 16 entries as starts
        uint32_t run = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) run += cnt[16 * t + q];
        uint32_t base = block_scan_incl<uint32_t, OpAdd>(run, OpAdd{}, s_w4, 0u) - run;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const uint32_t x = cnt[16 * t + q];
            cnt[16 * t + q] = base;
            base += x;
        }
        __syncthreads();
#pragma unroll
        for (int d = 0; d < 16; ++d) c16[d] = cnt[d * kRsSmallThreads + t];
        for (int32_t i = lo; i < hi; ++i) {
            const uint32_t k = bk[cur][i], d = (k >> shift) & 15u;
            uint32_t pos = 0;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                pos = d == (uint32_t)q ? c16[q] : pos;
                c16[q] += d == (uint32_t)q;
            }
            bk[cur ^ 1][pos] = k;
            bv[cur ^ 1][pos] = bv[cur][i];
        }
        cur ^= 1;
    }
    __syncthreads();
    for (int32_t i = t; i < n; i += kRsSmallThreads) {
        keys[i] = bk[cur][i];
        vals[i] = bv[cur][i];
    }
}

void radix_sort_pairs(Ctx& c, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, int64_t n,
                      int key_bits, uint32_t** out_keys, uint32_t** out_vals)
{
    if (out_keys) *out_keys = keys;
    if (out_vals) *out_vals = vals;
    if (n <= 1 || key_bits <= 0) return;
    if (n <= kRsSmallMax) {
        const size_t lds = sizeof(uint32_t) * (4 * (size_t)n + 16 * kRsSmallThreads);
        // LDS beyond the 64 KiB default
        allow_lds((const void*)k_rs_small, (int)(sizeof(uint32_t) * (4 * kRsSmallMax + 16 * kRsSmallThreads)));
        hipLaunchKernelGGL(k_rs_small, dim3(1), dim3(kRsSmallThreads), lds, c.stream, keys, vals, (int32_t)n,
                           key_bits);
        KMP_LAUNCH_CHECK();
        return;
    }
    const int nblk = (int)((n + RS_TILE - 1) / RS_TILE);
    DBuf<int32_t> hist(c, (size_t)nblk * 256);
    uint32_t *ks = keys, *vs = vals, *kd = keys_alt, *vd = vals_alt;
    for (int shift = 0; shift < key_bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(kBlock), 0, c.stream, ks, n, shift, hist.p, nblk);
        KMP_LAUNCH_CHECK();
        scan_excl_i32(c, hist.p, hist.p, (int64_t)nblk * 256, nullptr);
        hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(kBlock), 0, c.stream, ks, vs, kd, vd, n, shift, hist.p,
                           nblk);
        KMP_LAUNCH_CHECK();
        std::swap(ks, kd);
        std::swap(vs, vd);
    }
    if (out_keys || out_vals) {
        if (out_keys) *out_keys = ks;
        if (out_vals) *out_vals = vs;
        return;
    }
    if (ks != keys) {
        KMP_HIP(hipMemcpyAsync(keys, ks, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, c.stream));
        KMP_HIP(hipMemcpyAsync(vals, vs, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, c.stream));
    }
}

// ================================================================ fills, sums
namespace {

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_iota(int32_t* p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_sum_i32(const int32_t* __restrict__ p, int64_t n, int64_t* out)
{
    __shared__ int64_t ws[kBlock / 64];
    int64_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc += p[i];
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int q = 0; q < kBlock / 64; ++q) t += ws[q];
        if (t) spread_add(out, t);
    }
}

}  // namespace

namespace {
struct FillList {
    unsigned char* p[kMaxFills];
    int64_t bytes[kMaxFills];
    uint32_t word[kMaxFills];  // the byte repeated four times
};

// blockIdx.y = buffer; 4-byte stores over the aligned body, bytes at the ends
__global__ __launch_bounds__(kBlock) void k_fill_many(FillList L)
{
    const int q = blockIdx.y;
    unsigned char* p = L.p[q];
    const int64_t nb = L.bytes[q];
    const uint64_t a = (uint64_t)p;
    const int64_t head = (int64_t)((4 - (a & 3)) & 3) < nb ? (int64_t)((4 - (a & 3)) & 3) : nb;
    const int64_t words = (nb - head) >> 2;
    uint32_t* w = reinterpret_cast<uint32_t*>(p + head);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t; i < words; i += stride) w[i] = L.word[q];
    const unsigned char b = (unsigned char)L.word[q];
    if (t < head) p[t] = b;
    const int64_t tail0 = head + (words << 2);
    if (t < nb - tail0) p[tail0 + t] = b;
}
}  // namespace

void fill_bytes_many(Ctx& c, std::initializer_list<ByteFill> fills)
{
    FillList L;
    int nf = 0;
    int64_t mx = 0;
    for (const ByteFill& f : fills) {
        if (!f.p || f.bytes <= 0) continue;
        if (nf == kMaxFills) throw Error(KMP_EINVAL, "too many buffers in one fill");
        L.p[nf] = static_cast<unsigned char*>(f.p);
        L.bytes[nf] = f.bytes;
        L.word[nf] = 0x01010101u * f.byte;
        mx = std::max<int64_t>(mx, f.bytes / 4 + 4);
        ++nf;
    }
    if (nf == 0) return;
    hipLaunchKernelGGL(k_fill_many, dim3(grid_for(mx, kBlock, 4096), nf), dim3(kBlock), 0, c.stream, L);
    KMP_LAUNCH_CHECK();
}

void fill_i32(Ctx& c, int32_t* p, int32_t v, int64_t n)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, c.stream, p, v, n);
    KMP_LAUNCH_CHECK();
}
void fill_u8(Ctx& c, uint8_t* p, uint8_t v, int64_t n)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<uint8_t>, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, c.stream, p, v, n);
    KMP_LAUNCH_CHECK();
}
void fill_i64(Ctx& c, int64_t* p, int64_t v, int64_t n)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<int64_t>, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, c.stream, p, v, n);
    KMP_LAUNCH_CHECK();
}
void iota_i32(Ctx& c, int32_t* p, int64_t n)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n, kBlock, 4096)), dim3(kBlock), 0, c.stream, p, n);
    KMP_LAUNCH_CHECK();
}

namespace {

// out[0] = xadj[n]; out[1] = max over v of xadj[v + 1] - xadj[v] (out zeroed)
// One atomic per workgroup (atomics on one address serialise; the grid is
// capped at one workgroup per compute unit).
__global__ __launch_bounds__(kBlock) void k_max_deg(const int32_t* __restrict__ xadj, int32_t n, int32_t* out)
{
    __shared__ int32_t s_m[kBlock / 64];
    int32_t m = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        m = max(m, xadj[v + 1] - xadj[v]);
    for (int q = 32; q > 0; q >>= 1) m = max(m, __shfl_xor(m, q, 64));
    if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) m = max(m, s_m[w]);
        if (m) atomicMax(&out[1], m);
        if (blockIdx.x == 0) out[0] = xadj[n];
    }
}

}  // namespace

void entries_and_max_degree(Ctx& c, const int32_t* xadj, int32_t n, int64_t& m, int32_t& maxdeg, int32_t* zeroed2)
{
    DBuf<int32_t> own;
    int32_t* out = zeroed2;
    if (!out) {
        own = DBuf<int32_t>(c, 2);
        fill_bytes_many(c, {{own.p, 8, 0}});
        out = own.p;
    }
    hipLaunchKernelGGL(k_max_deg, dim3(grid_for(n, kBlock, 256)), dim3(kBlock), 0, c.stream, xadj, n, out);
    KMP_LAUNCH_CHECK();
    int32_t h[2];
    c.read(h, out, sizeof(h));
    m = h[0];
    maxdeg = h[1];
}

// ---------------------------------------------------------------- kernel attributes
void allow_lds(const void* fn, int bytes)
{
    static std::mutex mu;
    static std::vector<std::pair<const void*, int>> done;  // (kernel, device)
    int dev = 0;
    KMP_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    for (const auto& d : done)
        if (d.first == fn && d.second == dev) return;
    KMP_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    done.emplace_back(fn, dev);
}

// ---------------------------------------------------------------- packed read-back
namespace {
struct Segs {
    const int64_t* p[kMaxReadSegs];
    int32_t n[kMaxReadSegs];
    int32_t count;
};

__global__ __launch_bounds__(kBlock) void k_gather_segs(Segs s, int64_t* __restrict__ out)
{
    int64_t o = 0;
    for (int q = 0; q < s.count; ++q) {
        for (int32_t i = threadIdx.x; i < s.n[q]; i += blockDim.x) out[o + i] = s.p[q][i];
        o += s.n[q];
    }
}
}  // namespace

void read_segments(Ctx& c, const std::vector<std::pair<const int64_t*, int32_t>>& segs, int64_t* host)
{
    if (segs.empty() || segs.size() > (size_t)kMaxReadSegs) throw std::invalid_argument("read_segments");
    Segs s{};
    int64_t total = 0;
    s.count = (int32_t)segs.size();
    for (size_t q = 0; q < segs.size(); ++q) {
        s.p[q] = segs[q].first;
        s.n[q] = segs[q].second;
        total += segs[q].second;
    }
    if (total == 0) return;
    DBuf<int64_t> buf(c, (size_t)total);
    hipLaunchKernelGGL(k_gather_segs, dim3(1), dim3(kBlock), 0, c.stream, s, buf.p);
    KMP_LAUNCH_CHECK();
    c.read(host, buf.p, sizeof(int64_t) * (size_t)total);
}

int64_t node_weight_sum(Ctx& c, const int32_t* vwgt, int32_t n)
{
    if (!vwgt) return n;
    if (n <= 0) return 0;
    c.zero_spread(SP_VSUM);
    hipLaunchKernelGGL(k_sum_i32, dim3(grid_for(n, kBlock, 1024)), dim3(kBlock), 0, c.stream, vwgt, (int64_t)n,
                       c.spread(SP_VSUM));
    KMP_LAUNCH_CHECK();
    return c.read_spread(SP_VSUM);
}

int64_t edge_weight_sum(Ctx& c, const int32_t* adjwgt, int64_t m)
{
    if (!adjwgt) return m;
    if (m <= 0) return 0;
    c.zero_spread(SP_ESUM);
    hipLaunchKernelGGL(k_sum_i32, dim3(grid_for(m, kBlock, 1024)), dim3(kBlock), 0, c.stream, adjwgt, m,
                       c.spread(SP_ESUM));
    KMP_LAUNCH_CHECK();
    return c.read_spread(SP_ESUM);
}

}  // namespace kmp
