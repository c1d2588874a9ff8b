/*
 * kmp.h -- C ABI of libkmp, a gfx950 (MI355X) implementation of the data-
 * parallel hot path of deep multilevel graph partitioning (Gottesbueren,
 * Heuer, Sanders, Schulz, Seemaier, "Deep Multilevel Graph Partitioning").
 *
 * Problem (paper Sec. 2, "Notation and Definitions"): given an undirected
 * graph G = (V, E, c, w) with positive integer node weights c and edge
 * weights w, split V into k blocks of weight at most
 * L_k = (1 + eps) * ceil(c(V) / k) (the bound the paper's experiments check,
 * Sec. 2 footnote and Sec. 6) while minimising the weight of cut edges.
 *
 * Method (paper Alg. 1 / Alg. 2, Sec. 4-5): coarsen by size-constrained label
 * propagation (LP) and contraction until about 2C nodes remain (C = 160);
 * bipartition the coarsest graph; while projecting back, bipartition blocks
 * until level l has min(k, ceil2(n_l / C)) blocks; balance; refine with k-way
 * LP.  The LP here is a deterministic "sub-round" reading of the paper's
 * asynchronous LP, so results depend only on (graph, k, eps, seed).
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE (HBM) pointers on the current HIP device,
 *     owned by the caller.  Inputs are read only; outputs are written fully.
 *   - Graphs are symmetric CSR: xadj[n+1] row offsets (int32, xadj[0] = 0),
 *     adjncy[m] neighbour ids (int32), m = xadj[n] = number of DIRECTED
 *     entries (twice the number of edges).  vwgt[n] node weights and
 *     adjwgt[m] edge weights may be NULL (all ones).  Neighbour order within a
 *     row is free; self-loops and duplicates are not allowed.
 *   - Sum of node weights and half the sum of edge weights must fit in int32.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     The library enqueues all work on it and synchronises it before return
 *     (the scheduler reads per-level scalars).  Workspace comes from a
 *     process-wide caching pool of device blocks on the current device: a
 *     call takes blocks from it (allocating only when no cached block fits)
 *     and hands them back when it returns, so after the first calls of a size
 *     nothing is allocated; the cached blocks stay allocated until the
 *     process ends.  The environment variable KMP_WORKSPACE_LIMIT (bytes,
 *     read at the start of every call) caps the workspace one call may take;
 *     a call that needs more fails with KMP_ENOMEM (for tests of that path).
 *   - Calls on different streams may run concurrently from different threads.
 *   - Return value: 0 = OK; 1 = KMP_IMBALANCED (output written, but some block
 *     exceeds L_k; possible only with non-unit node weights); negative codes
 *     below are errors and leave the output undefined.
 */
#ifndef KMP_H
#define KMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KMP_OK 0
#define KMP_IMBALANCED 1
#define KMP_EINVAL (-1)    /* n < 0, k < 1, eps < 0, eps > 1000 or NaN, NULL required pointer, m != xadj[n] */
#define KMP_EGRAPH (-2)    /* invalid CSR (checked only when validation is requested) */
#define KMP_EOVERFLOW (-3) /* sum(vwgt) or sum(adjwgt)/2 exceeds INT32_MAX */
#define KMP_ENOMEM (-4)    /* device workspace allocation failed */
#define KMP_EHIP (-5)      /* a HIP runtime call failed */
#define KMP_ETOOLARGE (-6) /* input beyond the limits of kmp_partition_noalloc */

#define KMP_MAX_LEVELS 64

/* Options for kmp_partition_ex (all fields zero = defaults). */
typedef struct kmp_options {
    int32_t validate;       /* 1: check the CSR on the device first (KMP_EGRAPH on failure) */
    int32_t profile;        /* 1: time kernel classes with HIP events (fills kmp_stats.prof_*);
                               2: also synchronise at phase boundaries for the ms_* phase timers */
    uint32_t profile_classes; /* bit i set: time class i only (fewer event records); 0: all classes */
    int32_t force_exact;    /* 1: every LP sub-round with a contended proposal takes the host-synchronised
                               exact admission path (by default only sub-rounds with more than 4096
                               contended proposals do); implies small_level_n = -1.  The output does not
                               depend on it. */
    int32_t small_level_n;  /* LP calls on levels of at most this many nodes (and no node of degree > 64)
                               run in one workgroup launch: 0 = default (8192), -1 = never.  The output
                               does not depend on it. */
    int32_t plain_loads;    /* 1: the lane rating kernel gathers with plain loads instead of buffer loads
                               (used on graphs of 2^29 or more entries anyway); for tests.  The output
                               does not depend on it. */
    int32_t fm_passes;      /* 0..16: passes of 2-way FM refinement (paper Sec. 5.2) applied to each of
                               the R greedy-growing bipartitions before the best one is kept; 0 = none
                               (the default).  Moves the unlocked node of largest cut gain whose target
                               side has room, locks it; a pass returns to its best prefix (least overload,
                               then most gain) and ends when no node fits or after 64 moves without a
                               better prefix.  Out of range: KMP_EINVAL.  The output depends on it. */
    int32_t ip_pool;        /* 1: the initial bipartitioning pool of paper Sec. 5.2: besides the R greedy
                               growths, R breadth-first growths (discovery order; seed and restarts by
                               hash) and R random growths (hash order), all to the same target under the
                               same caps (and each refined when fm_passes > 0); the lowest (overload, cut)
                               is kept, the first of equal runs in the order GGG, BFS, random.  0: GGG
                               only (the default); other values: KMP_EINVAL.  The output depends on it. */
    int32_t adaptive_eps;   /* 1: every bipartition bounds its sides by the adaptive imbalance of paper
                               Sec. 2 / Alg. 2 (the L_2 bound of Sec. 5.2): a block B that is to end as f
                               blocks is split with eps' = ((1 + eps) c(V) f / (k c(B)))^(1/ceil(log2 f)) - 1
                               and side j (f_j = floor(f/2) or ceil(f/2) blocks) bounded by
                               (1 + eps') ceil(c(B) f_j / f), evaluated exactly in integers (2^32 fixed
                               point: the largest q whose r-fold stepwise-floored power p <- p q / 2^32
                               stays within floor(2^32 (1 + eps')^r)).  0: sides bounded by f_j L_k (the
                               default); other values: KMP_EINVAL.  The output depends on it. */
    int32_t pq_balance;     /* 1: the queue balancer of paper Sec. 5.3 instead of sorted rounds: per pass,
                               every overloaded block in ascending index fills a queue with just enough of
                               its nodes by relative gain (d c(v) for d >= 0, d / c(v) otherwise; then id),
                               from their pass-start targets, then takes the best node while overloaded:
                               its target and gain are recomputed; if either changed it is offered again
                               when it is a border node, else it moves and its neighbours still in the
                               block are offered once per pass; passes repeat while a block is overloaded
                               and the last pass moved.  One GPU thread per job runs a pass (the blocks of
                               a job depend on each other).  0: sorted rounds (the default); other values:
                               KMP_EINVAL.  The output depends on it. */
    int32_t async_lp;       /* every LP call (coarsening and refinement) in the asynchronous mode of paper
                               Sec. 5.1 "Parallelization" / Sec. 5.3 "Local Improvement" instead of the
                               deterministic sub-rounds: nodes visited by degree bucket floor(log2 d) then
                               id (Sec. 5.1 "Iteration Order"), all at once, each rated against the current
                               labels and weights and moved at once; clustering updates the two cluster
                               weights with fetch-and-add after checking the bound against the weights it
                               read (concurrent moves may exceed U, as in the paper), refinement reserves
                               the target's weight with compare-and-swap (the bound holds strictly).
                               0: deterministic (the default); 1: asynchronous (the output may differ from
                               run to run); 2: asynchronous executed one node per launch in visit order,
                               the execution by a single processing element (deterministic; for tests,
                               slow); other values: KMP_EINVAL.  The output depends on it. */
    int32_t ip_multilevel;  /* 1: multilevel initial bipartitioning (paper Sec. 5.2): the subgraph of every
                               block to split is coarsened with the deterministic LP (cluster bound
                               max(heaviest node, larger side bound / 18), the block's own seed
                               seed XOR (first << 32), no two-hop) and contraction until a clustering
                               leaves every node alone; the coarsest graph is bipartitioned by the growths
                               above (with FM and the pool as set), and each finer level refines the
                               projected sides with fm_passes FM passes.  0: single-level growths (the
                               default); other values: KMP_EINVAL.  The output depends on it. */
} kmp_options;

/* Kernel classes reported when kmp_options.profile is set. */
#define KMP_PROF_CLASSES 16
enum {
    KMP_PROF_RATE_T0 = 0,      /* LP rating, degree <= 16 (one lane per node)         */
    KMP_PROF_RATE_T1 = 1,      /* LP rating, degree <= 64 (16 lanes per node)         */
    KMP_PROF_RATE_T2 = 2,      /* LP rating, degree <= 4096 (wavefront / workgroup)   */
    KMP_PROF_RATE_HUB = 3,     /* LP rating, degree > 4096 (global hash)              */
    KMP_PROF_ADMIT = 4,        /* admission of uncontended targets                    */
    KMP_PROF_APPLY = 5,        /* apply admitted moves                                */
    KMP_PROF_LP_SMALL = 6,     /* whole LP call of a small level in one workgroup     */
    KMP_PROF_ACTIVE = 7,       /* next-round active set                               */
    KMP_PROF_CONTRACT_ROWS = 8,/* contraction: LDS aggregation of coarse rows         */
    KMP_PROF_CONTRACT = 9,     /* contraction: relabel, bucketing, heavy rows, copy   */
    KMP_PROF_TWO_HOP = 10,
    KMP_PROF_GGG = 11,         /* batched greedy graph growing                        */
    KMP_PROF_BALANCE = 12,
    KMP_PROF_PROJECT = 13,     /* projection, relabel, block weights                  */
    KMP_PROF_SCHEDULE = 14,    /* per-level sub-round class / degree-tier schedule    */
    KMP_PROF_OTHER = 15
};

/* Statistics filled by kmp_partition_ex (host memory, may be NULL). */
typedef struct kmp_stats {
    int64_t cut;                            /* final edge cut (paper Sec. 2)            */
    int64_t lk;                             /* L_k = floor(ceil(c(V)/k) (10^6 + e) / 10^6) */
    int64_t max_block_weight;
    int32_t levels;                         /* number of contractions L                  */
    int32_t bipartitions;                   /* number of bipartitioned blocks (GGG calls) */
    int32_t balance_rounds;
    int32_t lp_exact_subrounds;             /* LP sub-rounds finished on the exact admission path */
    int32_t level_n[KMP_MAX_LEVELS + 1];    /* nodes per level                           */
    int64_t level_m[KMP_MAX_LEVELS + 1];    /* directed entries per level                */
    int64_t lp_cluster_moves;
    int64_t lp_refine_moves;
    int64_t lp_rated_edges;                 /* directed entries read by LP rating kernels */
    int64_t contracted_edges;               /* sum of m_l over contracted levels          */
    double ms_total;                        /* wall time of the call                      */
    double ms_coarsen_lp;                   /* host-timed phases (device-synchronised only with profile = 2) */
    double ms_contract;
    double ms_initial;                      /* bipartitioning (extraction + GGG)          */
    double ms_refine;                       /* balance + refinement + projection          */
    /* filled when kmp_options.profile is set: per kernel class, the number of
     * launches, the summed HIP-event duration of those launches and, for the
     * LP rating, one-workgroup LP and contraction-row classes, their
     * algorithmic bytes (bytes the algorithm must move: rating 25 B per rated
     * node + 12 B per rated directed entry, 8 B when edge weights are unit;
     * the one-workgroup LP counts its rating bytes only; contraction rows 12 B
     * per fine entry + 12 B per member node + 8 B per coarse entry + 16 B per
     * coarse row). */
    int64_t prof_launches[KMP_PROF_CLASSES];
    double prof_ms[KMP_PROF_CLASSES];
    int64_t prof_bytes[KMP_PROF_CLASSES];
    int64_t workspace_bytes;                /* device workspace the call took (block capacities) */
} kmp_stats;

/*
 * kmp_partition: partition (xadj, adjncy, vwgt, adjwgt) into k blocks with
 * imbalance eps and tie-break seed `seed`; writes out_part[v] in [0, k).
 * Paper: Alg. 1 (deep MGP driver), Alg. 2 (bipartitionBlocks), Sec. 5.
 * Special cases: n = 0 -> OK, nothing written; k = 1 -> all zeros; k > n is
 * allowed (some blocks stay empty).
 */
int kmp_partition(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt,
                  int32_t n, int64_t m, int32_t k, double epsilon, uint64_t seed, int32_t* out_part,
                  void* stream);

/* As kmp_partition, with options (may be NULL) and statistics (may be NULL). */
int kmp_partition_ex(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt,
                     int32_t n, int64_t m, int32_t k, double epsilon, uint64_t seed, int32_t* out_part,
                     void* stream, const kmp_options* opt, kmp_stats* stats);

/*
 * kmp_partition_noalloc: kmp_partition_ex that allocates nothing, for callers
 * that cannot allocate device or pinned host memory (code around graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Every
 * device buffer of the call is carved from a fixed scratch region of
 * KMP_NOALLOC_SCRATCH_BYTES that the library holds on each device it runs on,
 * from the first call there until the process ends; host reads and writes
 * are plain stream-ordered copies followed by a synchronisation of `stream`.
 * The output equals kmp_partition_ex's for the same arguments.
 * Limits: n <= KMP_NOALLOC_MAX_N and m <= KMP_NOALLOC_MAX_M, else
 * KMP_ETOOLARGE and nothing runs; opt->profile must be 0 (KMP_EINVAL), the
 * other options are honoured; a call whose workspace would still exceed the
 * region returns KMP_ENOMEM.  The region is shared by all calls on a device:
 * calls from this process on one device run one at a time (a lock is held
 * for the whole call), and each call clears what it needs, so no state
 * carries from one call to the next.  Two processes each hold their own
 * region.  stats (may be NULL) as for kmp_partition_ex; workspace_bytes
 * reports how much of the region the call used.
 */
#define KMP_NOALLOC_MAX_N 65536
#define KMP_NOALLOC_MAX_M 1048576
#define KMP_NOALLOC_SCRATCH_BYTES (256ull << 20)
int kmp_partition_noalloc(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt,
                          int32_t n, int64_t m, int32_t k, double epsilon, uint64_t seed, int32_t* out_part,
                          void* stream, const kmp_options* opt, kmp_stats* stats);

/* One job of a batch: a graph in the layout above plus its own k, eps, seed
 * and output array (all device pointers owned by the caller). */
typedef struct kmp_graph_desc {
    const int32_t* xadj;
    const int32_t* adjncy;
    const int32_t* vwgt;    /* NULL = unit */
    const int32_t* adjwgt;  /* NULL = unit */
    int32_t n;
    int32_t k;
    int64_t m;              /* = xadj[n] */
    double epsilon;
    uint64_t seed;
    int32_t* out_part;      /* [n], values in [0, k) */
} kmp_graph_desc;

/* Per-job result of kmp_partition_batch (host memory). */
typedef struct kmp_job_result {
    int32_t status;                       /* KMP_OK, KMP_IMBALANCED or a negative code for this job */
    int32_t levels;                       /* number of contractions                          */
    int64_t cut;
    int64_t max_block_weight;
    int64_t lk;
    int32_t level_n[KMP_MAX_LEVELS + 1];  /* nodes per level                                 */
} kmp_job_result;

/*
 * kmp_partition_batch: partition `count` independent graphs in one pass of
 * the hot path.  The jobs run level by level as one disjoint union of their
 * level graphs (the paper's algorithm per job, Alg. 1 / Alg. 2, Sec. 5), so
 * one kernel launch serves every job that is at that step; each job's output
 * equals what kmp_partition returns for it alone (same graph, k, eps, seed).
 * A job with invalid arguments gets its error code in results[i].status and
 * does not stop the others.  results may be NULL; opt / stats as for
 * kmp_partition_ex (stats: counters summed over the batch, cut = sum of cuts).
 * The call synchronises `stream` before returning (the scheduler reads
 * per-level scalars of every job, so the batch is not asynchronous; callers
 * that need asynchrony submit to the server below, whose worker threads run
 * the batches).  Returns KMP_OK once every
 * job has its status, or a negative code for the call itself (count < 0,
 * graphs == NULL with count > 0, HIP errors, device memory exhausted).
 */
int kmp_partition_batch(const kmp_graph_desc* graphs, int32_t count, kmp_job_result* results, void* stream,
                        const kmp_options* opt, kmp_stats* stats);

/*
 * Serving loop with continuous batching (jobs arriving over time).
 *
 * kmp_server_create starts `workers` (1..16) host threads on the current
 * device, each with its own non-blocking HIP stream (the server owns its
 * streams: it takes a worker count, not a caller stream, because batches
 * overlap on the device only from streams of their own).  Submitted jobs wait
 * in arrival order.  A free worker opens a batch with the oldest waiting job
 * once its estimated device footprint (160 B per node + 96 B per directed
 * entry + 1 MiB) fits in what is left of hbm_budget_bytes, or nothing else
 * runs (a job larger than the whole budget then runs alone); it adds later
 * waiting jobs of the same size class (n + m within a factor of four) and the
 * same options whose footprints still fit, up to 256, and runs them as one
 * batch (as kmp_partition_batch).  Jobs that arrive while batches run are
 * admitted by the next free worker, so their work overlaps on the device.
 * The footprint is an estimate used for admission; the memory itself comes
 * from the caching pool described above.  Each job's output equals
 * kmp_partition_ex's for it alone with the options current at its
 * submission.  Returns NULL on invalid arguments or when no stream / thread
 * can be created.
 *
 * kmp_server_submit copies the descriptor and returns at once with a job id;
 * the job's device arrays must stay valid and untouched until its result has
 * been taken.  kmp_server_poll (non-blocking) returns 0 while the job is
 * pending and 1 once it is done, filling `result` (the job's status, cut,
 * levels; the status is inside `result`, not a separate int) and
 * `latency_ms` (completion minus submission, host steady clock; both may be
 * NULL) and forgetting the job; kmp_server_wait blocks until then.  Unknown
 * ids, and ids whose result another thread has taken meanwhile, give
 * KMP_EINVAL.  kmp_server_destroy finishes every submitted job, then stops
 * the workers.
 */
typedef struct kmp_server kmp_server;

typedef struct kmp_server_stats {
    int64_t jobs_submitted;
    int64_t jobs_done;
    int64_t batches;          /* batches run so far          */
    int64_t max_batch_jobs;   /* largest batch               */
    int64_t queued;           /* jobs waiting now            */
    int64_t hbm_in_use;       /* footprint of running batches */
    int32_t running_batches;
    int32_t reserved;
} kmp_server_stats;

kmp_server* kmp_server_create(size_t hbm_budget_bytes, int32_t workers);
int kmp_server_submit(kmp_server* server, const kmp_graph_desc* job, uint64_t* job_id);
int kmp_server_poll(kmp_server* server, uint64_t job_id, kmp_job_result* result, double* latency_ms);
int kmp_server_wait(kmp_server* server, uint64_t job_id, kmp_job_result* result, double* latency_ms);
int kmp_server_stats_get(kmp_server* server, kmp_server_stats* stats);
void kmp_server_destroy(kmp_server* server);

/*
 * kmp_server_set_options: the initial-bipartitioning options (fm_passes,
 * ip_pool, adaptive_eps, pq_balance; meaning and ranges as in kmp_options) for every job submitted
 * after the call (a job keeps the options current at its submission; only
 * jobs with equal options share a batch); the other fields of *opt are
 * ignored.  opt == NULL restores the defaults.  Out-of-range values give
 * KMP_EINVAL and change nothing.  Each job's output then equals
 * kmp_partition_ex's with its options for it alone.
 */
int kmp_server_set_options(kmp_server* server, const kmp_options* opt);

/* ------------------------------------------------------------------------
 * Tuning.  Launch choices that change how the path runs on the device but
 * never its output (the partition depends only on graph, k, epsilon and seed).
 * They are process-wide: every call reads them once when it starts.  The
 * rating tiers follow the degree ranges of the rating kernels: degree <=
 * tier0_deg one lane per node; <= tier1_deg 16 lanes with a 128-slot LDS
 * table; <= tier2_deg a wavefront with a 1024-slot table; <= tier3_deg a
 * workgroup with an 8192-slot table; above, the
 * hub tier: the row in runs of 4096 entries, split by label partition, each
 * partition summed in an LDS table of hub_lds_slots slots (each LDS table of
 * tiers 1-3 has at least twice as many slots as the largest degree it may
 * hold, which bounds the ranges).
 * ------------------------------------------------------------------------ */
typedef struct kmp_tuning {
    int32_t small_level_n;  /* LP calls on levels of at most this many nodes with no node of degree > 64
                               run in one workgroup launch; -1 = never (range -1 .. 2^30; default 8192) */
    int32_t tier0_deg;      /* 1 .. 16, default 16     */
    int32_t tier1_deg;      /* tier0_deg .. 64, default 64      */
    int32_t tier2_deg;      /* tier1_deg .. 512, default 512    */
    int32_t tier3_deg;      /* tier2_deg .. 4096, default 4096  */
    int32_t hub_lds_slots;  /* slots of the LDS table that sums a label partition of a hub (degree above
                               tier3_deg): a power of two 64 .. 8192; 0 = the default 4096.  A partition
                               with more distinct labels takes a global table instead. */
    int32_t reserved[2];    /* 0 */
} kmp_tuning;

/* Set the process-wide tuning (NULL: the defaults).  KMP_EINVAL, and no
 * change, if a value is outside its range. */
int kmp_set_tuning(const kmp_tuning* tuning);
/* Current process-wide tuning.  KMP_EINVAL if tuning is NULL. */
int kmp_get_tuning(kmp_tuning* tuning);

typedef struct kmp_autotune_report {
    int32_t configs;        /* settings timed                                  */
    int32_t reps;           /* timed calls per setting (median taken)          */
    double ms_start;        /* median ms of kmp_partition with the start setting */
    double ms_best;         /* median ms with the chosen setting               */
} kmp_autotune_report;

/*
 * kmp_autotune: time kmp_partition on the given job (device arrays, as for
 * kmp_partition_batch; graph->out_part receives the partition) under a set
 * of candidate tunings and keep the fastest.  Coordinate search from the
 * current setting: small_level_n over {-1, 2048, 4096, 8192, 16384, 32768},
 * then each tier cut-off over {its default, half of it}; a candidate replaces
 * the current value only if its median time over `reps` calls (1..50, after
 * one untimed call) is at least 2% lower.  Every candidate's partition must equal the
 * first one's bit for bit: a difference returns KMP_EHIP (a defect, since
 * tuning never changes the output).  On success the chosen tuning is set
 * process-wide and copied to *chosen (may be NULL); report may be NULL.
 * Calls in other threads meanwhile run under whichever setting is current.
 */
int kmp_autotune(const kmp_graph_desc* graph, int32_t reps, void* stream, kmp_tuning* chosen,
                 kmp_autotune_report* report);

/* Human-readable text for a status code (static storage). */
const char* kmp_strerror(int code);

/* Library version, "major.minor.patch" (static storage). */
const char* kmp_version(void);

/* ------------------------------------------------------------------------
 * Step entry points.  Each runs one step of the pipeline on the device with
 * the same semantics as inside kmp_partition, so a caller (or a test) can
 * drive and check the steps one at a time.  Same conventions as above; all
 * arrays are device pointers; every call synchronises `stream`.
 * ------------------------------------------------------------------------ */

/*
 * kmp_lp_cluster: size-constrained LP clustering of one coarsening level
 * (paper Sec. 2 "Size-Constrained Label Propagation", Sec. 5.1): start from
 * singletons, at most 5 rounds of 4 hash-assigned sub-rounds, cluster weight
 * bound U, tie-break hashes keyed by (seed, level).  Outputs label[n]
 * (cluster ids in [0,n)), cw[n] cluster weights (int64, indexed by label),
 * fav[n] favoured cluster (0xFFFFFFFF = none).  moves[5] (host pointer, may be
 * NULL) receives moves per round.  Returns rounds run (>= 0) or an error.
 */
int kmp_lp_cluster(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt,
                   int32_t n, int32_t level, int64_t U, uint64_t seed, int32_t* label, int64_t* cw,
                   uint32_t* fav, int64_t* moves, void* stream);

/*
 * kmp_two_hop: two-hop merging of singleton clusters with the same favoured
 * cluster (paper Sec. 5.1 "Two-hop Clustering") when fewer than half of the
 * nodes were merged.  Updates label[n] and cw[n] in place.  Returns the number
 * of merges (>= 0) or an error.
 */
int64_t kmp_two_hop(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt,
                    int32_t n, int64_t U, int32_t* label, int64_t* cw, const uint32_t* fav, void* stream);

/*
 * kmp_contract: contract the clustering label[n] (paper Sec. 2 "Multilevel
 * Graph Partitioning"): coarse id = rank of the label among non-empty labels,
 * coarse node weight = member sum, parallel edges summed, intra-cluster edges
 * dropped, coarse neighbours ascending.  Writes map[n]; *cn and *cm (host
 * pointers) receive the coarse sizes.  The coarse arrays cxadj[n+1],
 * cadjncy[m], cvwgt[n], cadjwgt[m] are caller buffers sized for the fine
 * graph (upper bounds).
 */
int kmp_contract(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt,
                 int32_t n, const int32_t* label, int32_t* map, int32_t* cn, int64_t* cm, int32_t* cxadj,
                 int32_t* cadjncy, int32_t* cvwgt, int32_t* cadjwgt, void* stream);

/*
 * kmp_bipartition_round: one call of bipartitionBlocks (paper Alg. 2): every
 * block b with final count fcount[b] >= 2 is split by multi-seed greedy graph
 * growing into (first[b], floor(f/2)) and (first[b] + floor(f/2), ceil(f/2)),
 * caps f0 * lk and f1 * lk; blocks are renumbered in ascending `first`.
 * part[n] (device) is updated in place.  first/fcount are HOST arrays of
 * capacity 2 * (*nblocks) updated in place; *nblocks (host) is updated.
 */
int kmp_bipartition_round(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt,
                          const int32_t* adjwgt, int32_t n, int32_t level, int32_t* part, int32_t* nblocks,
                          int32_t* first, int32_t* fcount, int64_t lk, uint64_t seed, void* stream);

/*
 * kmp_bipartition_round_ex: kmp_bipartition_round with fm_passes (0..16,
 * else KMP_EINVAL) passes of 2-way FM refinement (paper Sec. 5.2) applied to
 * each growth before the lowest (overload, cut) is kept, and ip_pool (0 or 1,
 * else KMP_EINVAL) adding the breadth-first and random growths of the paper's
 * pool; both as described at kmp_options.  fm_passes = ip_pool = 0 is
 * kmp_bipartition_round.
 */
int kmp_bipartition_round_ex(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt,
                             const int32_t* adjwgt, int32_t n, int32_t level, int32_t* part, int32_t* nblocks,
                             int32_t* first, int32_t* fcount, int64_t lk, uint64_t seed, int32_t fm_passes,
                             int32_t ip_pool, void* stream);

/*
 * kmp_balance: k-way balancing by relative gain (paper Sec. 5.3
 * "Balancing") of part[n] over nb blocks with block weights wt[nb] (int64,
 * updated) and caps cap[nb] (int64).  Returns the number of rounds run.
 */
int kmp_balance(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt,
                int32_t n, int32_t level, uint64_t seed, int32_t* part, int64_t* wt, int32_t nb,
                const int64_t* cap, void* stream);

/*
 * kmp_balance_ex: kmp_balance with pq = 1 selecting the queue balancer
 * described at kmp_options.pq_balance (pq = 0: sorted rounds; other values
 * KMP_EINVAL).  Returns the rounds (passes) run.
 */
int kmp_balance_ex(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt,
                   int32_t n, int32_t level, uint64_t seed, int32_t* part, int64_t* wt, int32_t nb,
                   const int64_t* cap, int32_t pq, void* stream);

/*
 * kmp_lp_refine: k-way LP refinement (paper Sec. 5.3 "Local Improvement")
 * of part[n] over nb blocks, block weights wt[nb] (int64, updated; each the
 * node weight of its block, below 2^31), strict caps cap[nb] (int64).
 * moves[5] (host, may be NULL).  Returns rounds run.
 */
int kmp_lp_refine(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt,
                  int32_t n, int32_t level, uint64_t seed, int32_t* part, int64_t* wt, int32_t nb,
                  const int64_t* cap, int64_t* moves, void* stream);

/*
 * kmp_lp_subround: one sub-round (rate, admit, apply) of LP from an arbitrary
 * state: nodes of sub-round class s that are active (active[n] bytes, NULL =
 * all) are rated against the current labels; `tag` selects the tie-break
 * family (2 = clustering, 3 = refinement); cap is cap_vec[nlab] if non-NULL
 * else cap_scalar.  label[n], wt[nlab] (int64) updated; wt[L] must be the
 * weight of label L (the node weights of its members, so below 2^31);
 * fav[n] (may be NULL) written for rated nodes; moved[n] bytes set for moved
 * nodes.
 * Returns the number of moves or an error.
 */
int64_t kmp_lp_subround(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt,
                        const int32_t* adjwgt, int32_t n, int32_t level, int32_t round, int32_t s, uint32_t tag,
                        uint64_t seed, int32_t* label, int64_t* wt, int32_t nlab, const int64_t* cap_vec,
                        int64_t cap_scalar, const uint8_t* active, uint32_t* fav, uint8_t* moved,
                        void* stream);

/*
 * kmp_lp_async: a whole LP call in the asynchronous mode described at
 * kmp_options.async_lp (paper Sec. 5.1 "Parallelization" and "Iteration
 * Order", Sec. 5.3 "Local Improvement") from an arbitrary state: at most 5
 * rounds, stop after a round without moves, round r > 0 rates only nodes with
 * a neighbour that moved in round r - 1.  tag 2: clustering (fetch-and-add,
 * the bound may be exceeded by concurrent moves); tag 3: refinement
 * (compare-and-swap, the bound holds strictly); other tags: KMP_EINVAL.
 * label[n] in [0, nlab) and wt[nlab] (int64, the label sums) are updated; the
 * bound of label K is cap_vec[K] if cap_vec is non-NULL, else cap_scalar;
 * fav[n] (may be NULL) receives the favoured label of every rated node
 * (0xFFFFFFFF = none).  serial = 1 runs one node per launch in visit order
 * (deterministic, slow; 0 or 1, else KMP_EINVAL).  moves[5] (host, may be
 * NULL) receives moves per round.  Returns the rounds run or an error.
 */
int kmp_lp_async(const int32_t* xadj, const int32_t* adjncy, const int32_t* vwgt, const int32_t* adjwgt, int32_t n,
                 int32_t level, uint32_t tag, uint64_t seed, int32_t* label, int64_t* wt, int32_t nlab,
                 const int64_t* cap_vec, int64_t cap_scalar, uint32_t* fav, int64_t* moves, int32_t serial,
                 void* stream);

#ifdef __cplusplus
}
#endif

#endif /* KMP_H */
