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
#include <chrono>
#include <cmath>
#include <memory>

#include "kmp_dev.h"

namespace kmp {

namespace {

using clk = std::chrono::steady_clock;
double ms_since(clk::time_point t) { return std::chrono::duration<double, std::milli>(clk::now() - t).count(); }

void init_pool_once()
{
    static bool done = false;
    if (done) return;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
    }
    done = true;
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

struct Level {
    DGraph g;
    OwnedGraph own;      // storage for coarse levels
    DBuf<int32_t> map;   // to the next coarser level
    std::unique_ptr<LPSchedule> sched;
};

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

struct Common {
    int64_t cV = 0;
    int64_t e = 0;
    int64_t lk = 0;
};

int check_args(const int32_t* xadj, int32_t n, int64_t m, int32_t k, double eps, const int32_t* out)
{
    if (n < 0 || k < 1 || !(eps >= 0.0) || eps > 1000.0 || m < 0 || m > INT32_MAX) return KMP_EINVAL;
    if (n > 0 && (!xadj || !out)) return KMP_EINVAL;
    return KMP_OK;
}

// Checks m == xadj[n] and the int32 bounds of the weight sums; returns c(V).
int64_t prepare(Ctx& c, const DGraph& g)
{
    int32_t xn = 0;
    c.read(&xn, g.xadj + g.n, sizeof(int32_t));
    if ((int64_t)xn != g.m) throw Error(KMP_EINVAL, "m != xadj[n]");
    if (g.m > 0 && !g.adjncy) throw Error(KMP_EINVAL, "adjncy is NULL");
    int64_t sums[2] = {node_weight_sum(c, g.vwgt, g.n), edge_weight_sum(c, g.adjwgt, g.m)};
    if (sums[0] > INT32_MAX || sums[1] / 2 > INT32_MAX) throw Error(KMP_EOVERFLOW, "weight sum exceeds int32");
    return sums[0];
}

int partition_impl(const DGraph& g0, int32_t k, double eps, uint64_t seed, int32_t* out_part, hipStream_t stream,
                   const kmp_options* opt, kmp_stats* st)
{
    auto t_start = clk::now();
    init_pool_once();
    Ctx c(stream);
    std::unique_ptr<Prof> prof;
    const bool phase_sync = opt && opt->profile >= 2;  // phase timers wait for the device (profile = 2)
    if (opt && opt->profile) {
        prof.reset(new Prof());
        prof->mask = opt->profile_classes;
        c.prof = prof.get();
    }
    const int64_t cV = prepare(c, g0);
    if (opt && opt->validate) {
        int rc = validate_graph(c, g0);
        if (rc != KMP_OK) return rc;
    }
    const int64_t e = eps_ppm(eps);
    const int64_t W = (cV + k - 1) / k;
    const int64_t lk = W * (kPPM + e) / kPPM;
    if (st) st->lk = lk;
    const int32_t n = g0.n;
    if (k == 1) {
        fill_i32(c, out_part, 0, n);
        c.sync();
        if (st) {
            st->max_block_weight = cV;
            st->level_n[0] = n;
            st->level_m[0] = g0.m;
            st->ms_total = ms_since(t_start);
        }
        return cV > lk ? KMP_IMBALANCED : KMP_OK;
    }

    // ---------------- coarsening
    std::vector<std::unique_ptr<Level>> lv;
    lv.emplace_back(new Level());
    lv[0]->g = g0;
    int32_t kc = std::min<int64_t>(k, n / kC);
    double ms_lp = 0, ms_con = 0, ms_ip = 0, ms_ref = 0;
    int64_t moves_cl = 0, moves_ref = 0, rated = 0, contracted = 0;
    while (lv.back()->g.n > 2 * kC && (int)lv.size() - 1 < kMaxLevels) {
        Level& L = *lv.back();
        const DGraph& g = L.g;
        const int32_t level = (int32_t)lv.size() - 1;
        auto t0 = clk::now();
        const int64_t U = level_U(g.n, kc, cV, e);
        L.sched.reset(new LPSchedule());
        lp_build_schedule(c, g, level, seed, *L.sched);
        DBuf<int32_t> label(c, (size_t)g.n);
        DBuf<int64_t> cw(c, (size_t)g.n);
        DBuf<uint32_t> fav(c, (size_t)g.n);
        hipLaunchKernelGGL(k_iota_weights, dim3(grid_for(g.n)), dim3(kBlock), 0, c.stream, g.vwgt, g.n, label.p, cw.p,
                           fav.p);
        KMP_LAUNCH_CHECK();
        LPState ls{label.p, cw.p, g.n, nullptr, U, fav.p, TAG_CL};
        LPStats lps = lp_run(c, g, level, seed, *L.sched, ls);
        for (int r = 0; r < kRounds; ++r) moves_cl += lps.moves[r];
        rated += lps.rated_edges;
        two_hop(c, g, U, label.p, cw.p, fav.p);
        const int32_t nc = count_nonempty(c, cw.p, g.n);
        ms_lp += ms_since(t0);
        if (20LL * nc > 19LL * g.n) break;  // converged: keep this level as the coarsest
        auto t1 = clk::now();
        std::unique_ptr<Level> next(new Level());
        L.map = DBuf<int32_t>(c, (size_t)g.n);
        int32_t cn = 0;
        int64_t cm = 0;
        contract(c, g, label.p, cw.p, L.map.p, next->own, cn, cm);
        next->g = next->own.view(cn, cm);
        contracted += g.m;
        if (phase_sync) c.sync();
        ms_con += ms_since(t1);
        lv.push_back(std::move(next));
    }
    const int32_t Lc = (int32_t)lv.size() - 1;
    if (st) {
        st->levels = Lc;
        for (int32_t l = 0; l <= Lc; ++l) {
            st->level_n[l] = lv[l]->g.n;
            st->level_m[l] = lv[l]->g.m;
        }
    }

    // ---------------- uncoarsening
    std::vector<int32_t> first{0}, fcount{k};
    DBuf<int32_t> part(c, (size_t)lv[Lc]->g.n);
    c.zero(part.p, sizeof(int32_t) * (size_t)lv[Lc]->g.n);
    int32_t bip = 0, brounds = 0;
    DBuf<int64_t> wt, cap;
    for (int32_t l = Lc; l >= 0; --l) {
        Level& L = *lv[l];
        const DGraph& g = L.g;
        auto t0 = clk::now();
        if (l < Lc) {
            DBuf<int32_t> fine(c, (size_t)g.n);
            project(c, part.p, L.map.p, fine.p, g.n);
            part = std::move(fine);
        }
        int32_t kp = (l == 0) ? k : std::min(k, ceil2_div_C(g.n));
        kp = std::max(kp, 2);
        auto t1 = clk::now();
        while ((int32_t)first.size() < kp) bip += bipartition_round(c, g, l, part.p, first, fcount, lk, seed);
        if (phase_sync) c.sync();
        ms_ip += ms_since(t1);
        auto t2 = clk::now();
        const int32_t nb = (int32_t)first.size();
        wt = DBuf<int64_t>(c, (size_t)nb);
        cap = DBuf<int64_t>(c, (size_t)nb);
        block_weights(c, g, part.p, nb, wt.p);
        std::vector<int64_t> hcap(nb);
        for (int32_t b = 0; b < nb; ++b) hcap[b] = (int64_t)fcount[b] * lk;
        c.write(cap.p, hcap.data(), sizeof(int64_t) * nb);
        if (!L.sched) {
            L.sched.reset(new LPSchedule());
            lp_build_schedule(c, g, l, seed, *L.sched);
        }
        brounds += balance(c, g, l, seed, *L.sched, part.p, wt.p, nb, cap.p);
        LPState ls{part.p, wt.p, nb, cap.p, 0, nullptr, TAG_REF};
        LPStats lps = lp_run(c, g, l, seed, *L.sched, ls);
        for (int r = 0; r < kRounds; ++r) moves_ref += lps.moves[r];
        rated += lps.rated_edges;
        if (phase_sync) c.sync();
        ms_ref += ms_since(t2) + (ms_since(t0) - ms_since(t1));
        // the finer level no longer needs this level's storage
        if (l < Lc) lv[l + 1].reset();
    }
    // ---------------- final block ids and status
    const int32_t nb = (int32_t)first.size();
    DBuf<int32_t> dfirst(c, (size_t)nb);
    c.write(dfirst.p, first.data(), sizeof(int32_t) * nb);
    hipLaunchKernelGGL(k_final_ids, dim3(grid_for(n)), dim3(kBlock), 0, c.stream, part.p, dfirst.p, n, out_part);
    KMP_LAUNCH_CHECK();
    std::vector<int64_t> hw(nb);
    c.read(hw.data(), wt.p, sizeof(int64_t) * nb);
    int64_t maxw = 0;
    for (int64_t x : hw) maxw = std::max(maxw, x);
    if (st) {
        st->cut = edge_cut(c, g0, part.p);
        st->max_block_weight = maxw;
        st->bipartitions = bip;
        st->balance_rounds = brounds;
        st->lp_cluster_moves = moves_cl;
        st->lp_refine_moves = moves_ref;
        st->lp_rated_edges = rated;
        st->contracted_edges = contracted;
        st->ms_coarsen_lp = ms_lp;
        st->ms_contract = ms_con;
        st->ms_initial = ms_ip;
        st->ms_refine = ms_ref;
    }
    c.sync();
    if (st) {
        st->ms_total = ms_since(t_start);
        if (prof) c.prof_collect(st->prof_launches, st->prof_ms, st->prof_bytes);
    }
    c.prof = nullptr;
    return maxw > lk ? KMP_IMBALANCED : KMP_OK;
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

}  // namespace

}  // namespace kmp

using namespace kmp;

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
                              (hipStream_t)stream, opt, stats);
    });
}

int kmp_partition(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt, int32_t n,
                  int64_t m, int32_t k, double epsilon, uint64_t seed, int32_t* out_part, void* stream)
{
    return kmp_partition_ex(xadj, adjncy, vwgt, adjwgt, n, m, k, epsilon, seed, out_part, stream, nullptr, nullptr);
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
        LPStats r = lp_run(c, g, level, seed, sched, ls);
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
    if (n < 0 || !nblocks || *nblocks < 1 || !first || !fcount || (n > 0 && (!xadj || !part))) return KMP_EINVAL;
    return (int)guarded([&]() -> int64_t {
        init_pool_once();
        Ctx c((hipStream_t)stream);
        int32_t m32 = 0;
        if (n > 0) c.read(&m32, xadj + n, sizeof(int32_t));
        DGraph g = make_graph(xadj, adjncy, vwgt, adjwgt, n, m32);
        std::vector<int32_t> f(first, first + *nblocks), fc(fcount, fcount + *nblocks);
        bipartition_round(c, g, level, part, f, fc, lk, seed);
        c.sync();
        for (size_t i = 0; i < f.size(); ++i) {
            first[i] = f[i];
            fcount[i] = fc[i];
        }
        *nblocks = (int32_t)f.size();
        return KMP_OK;
    });
}

int kmp_balance(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt, int32_t n,
                int32_t level, uint64_t seed, int32_t* part, int64_t* wt, int32_t nb, const int64_t* cap,
                void* stream)
{
    if (n < 0 || nb < 1 || (n > 0 && (!xadj || !part || !wt || !cap))) return KMP_EINVAL;
    if (n == 0) return 0;
    return (int)guarded([&]() -> int64_t {
        init_pool_once();
        Ctx c((hipStream_t)stream);
        int32_t m32 = 0;
        c.read(&m32, xadj + n, sizeof(int32_t));
        DGraph g = make_graph(xadj, adjncy, vwgt, adjwgt, n, m32);
        LPSchedule sched;
        lp_build_schedule(c, g, level, seed, sched);
        int32_t r = balance(c, g, level, seed, sched, part, wt, nb, cap);
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
        LPStats r = lp_run(c, g, level, seed, sched, ls);
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

}  // extern "C"
