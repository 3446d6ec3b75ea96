/*
 * fs.h - C ABI of the MI355X (gfx950) renewal tau-leap SEIR step.
 *
 * The library runs the per-step renewal tau-leaping update of FlashSpread
 * (arXiv 2604.22092): the problem statement of Section "Problem formulation"
 * (graph G = (V, E, W), state (X, tau), Eq. (general_rate), Eq. (influence)),
 * one step per Algorithm 3 ("per-call replay of b fused steps"), the stable
 * log-normal hazard of Proposition 1, the Bernoulli tau-leap rule of Section
 * "Bernoulli tau-leaping" and the source-node infectivity of Eq. (infectivity)
 * with constant shedding s = 1.
 *
 * Conventions for every call:
 *  - All pointers in signatures are HOST pointers unless stated otherwise;
 *    the library copies what it needs before returning and never keeps a
 *    caller pointer.
 *  - Every call returns an fs_status.  No C++ exception crosses the ABI.  On
 *    failure an `out` handle is set to NULL, nothing is leaked, and
 *    fs_last_error() holds a thread-local message.
 *  - Handles are owned by the library and released by the matching
 *    *_destroy call.  One handle must not be used from two threads at once;
 *    distinct handles are independent.  A graph may back many sims.
 *  - Device work is queued on the sim's HIP stream.  Calls that return data
 *    to the host (fs_counts, fs_history, fs_get_state, fs_get_rates,
 *    fs_sync) synchronise that stream; fs_step does not, and an error raised
 *    by device work surfaces at the next synchronising call.
 *  - The device is the HIP device current when fs_graph_create is called;
 *    sims inherit it from their graph.
 */
#ifndef FS_H
#define FS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
typedef int32_t fs_status;
#define FS_OK 0
#define FS_ERR_INVALID_ARG 1   /* a scalar argument or pointer is invalid           */
#define FS_ERR_INVALID_CSR 2   /* the CSR arrays violate the rules of fs_graph_create */
#define FS_ERR_OUT_OF_MEMORY 3 /* a device or host allocation failed                 */
#define FS_ERR_DEVICE 4        /* a HIP runtime call or a kernel failed               */
#define FS_ERR_BUSY 5          /* the graph is still referenced by a sim              */
#define FS_ERR_BUDGET 6        /* the request exceeds the configured memory budget    */

/* Short name of a status code (static string). */
const char* fs_status_string(fs_status s);
/* Detail of the last failure on the calling thread (valid until the next call). */
const char* fs_last_error(void);

/* ------------------------------------------------------- compartments, laws */
/* Compartments of the SEIR model (Fig. SEIR): S -> E -> I -> R, R absorbing. */
#define FS_S 0
#define FS_E 1
#define FS_I 2
#define FS_R 3

/* Holding-time laws of the renewal transitions E -> I and I -> R.  The hazard
 * h(tau) = f(tau)/S(tau) (Section "Problem formulation") is evaluated at the
 * node's age at the start of the step.
 *   FS_DIST_EXP:        a = rate >= 0 (constant hazard; the Markovian case)
 *   FS_DIST_LOGNORMAL:  a = mu, b = sigma > 0, parameters of ln(tau) (Proposition 1)
 *   FS_DIST_WEIBULL:    a = shape >= 1, b = scale > 0 (days)
 *   FS_DIST_ERLANG:     k = integer shape in [1, 64], a = rate > 0 (per day);
 *                       "mean m" corresponds to rate = k/m
 * Weibull shapes below 1 are rejected: their hazard is infinite at age 0. */
#define FS_DIST_EXP 0
#define FS_DIST_LOGNORMAL 1
#define FS_DIST_WEIBULL 2
#define FS_DIST_ERLANG 3

typedef struct fs_dist {
    int32_t kind;
    int32_t k;
    double a;
    double b;
} fs_dist;

/* Shedding profile s(tau) of an infectious node of age tau (Eq. (infectivity):
 * the infectivity of source j is beta * s(tau_j) * 1{X_j = I}).
 *   FS_SHED_CONSTANT: s = 1 (Markovian edges; the infectivity is one bit)
 *   FS_SHED_DENSITY:  s = shed_scale * f(tau), f the density of shed_law
 *                     (the paper's example: a log-normal viral-load curve)
 *   FS_SHED_HAZARD:   s = shed_scale * h(tau), h the hazard of shed_law (the
 *                     in-kernel form of the overhead study, Table
 *                     "agedep_overhead", uses h_IR)
 * The value a node sheds during step k is s of its age at the start of step
 * k; a node that has just become infectious has age 0. */
#define FS_SHED_CONSTANT 0
#define FS_SHED_DENSITY 1
#define FS_SHED_HAZARD 2

/* Storage of the per-unit state (mixed-precision storage, Section
 * "Mixed-precision storage with an fp32 accumulator"); arithmetic is FP32 in
 * both.
 *   FS_STORAGE_FP32:    int32 state, float32 age in days
 *   FS_STORAGE_COMPACT: uint8 state, uint16 age in whole steps (tau = n*dt,
 *                       saturating at 65535)
 * In both, the next-step infectivity of Eq. (infectivity) is kept as one bit
 * per unit, 1{X = I}: with constant shedding s = 1 that bit is its exact value
 * (beta multiplies the pressure instead).  Age-dependent shedding adds an
 * s(tau) per unit, read only where the bit is set: float32 with FP32 storage,
 * IEEE binary16 (rounded to nearest even; the paper's FP16 infectivity) with
 * compact storage, summed in FP32 either way. */
#define FS_STORAGE_FP32 0
#define FS_STORAGE_COMPACT 1

/* Column storage of the step's transposed copy of the graph (the gather of
 * Eq. (influence) reads it every step; the caller's CSR is unchanged).
 *   FS_COLUMNS_AUTO:  where the step supports it -- an unweighted graph of at
 *                     most 2^27 nodes, one replica, and not age-dependent
 *                     shedding together with rate recording or compaction --
 *                     the rows of every 64-node
 *                     chunk that share one degree of at most 12 (every chunk of
 *                     a regular graph; almost all light rows of a degree-sorted
 *                     one) store each column in 20, 24 or 27 bits (the fewest
 *                     of these that hold the node ids: n <= 2^20, 2^24, 2^27),
 *                     a row's columns packed into one bit stream; the other
 *                     rows keep 32 bits.
 *   FS_COLUMNS_PLAIN: 32 bits per column always.
 * Results are identical.  A sim with packed columns that joins a batch moves
 * to 32-bit columns (the batch step reads those). */
#define FS_COLUMNS_AUTO 0
#define FS_COLUMNS_PLAIN 1

/* ----------------------------------------------------------- memory hook
 * Routes the library's persistent device arrays (graphs and their layouts,
 * sims, Markovian engines) through the caller's allocator, e.g. a framework's
 * caching allocator.  alloc(bytes, ctx) returns device memory on the current
 * device or NULL (reported as FS_ERR_OUT_OF_MEMORY); free(ptr, ctx) releases
 * it, called only after the owning stream has finished with the block.
 * Process-wide; a block is always released by the allocator that gave it
 * out, also after the hook changes.  Both NULL restores hipMalloc (graphs)
 * and the stream-ordered pool (sims).  Batch and server tables and call-local
 * temporaries always use the library's own allocator.
 * Errors: FS_ERR_INVALID_ARG when exactly one of alloc, free is NULL.
 */
typedef void* (*fs_alloc_fn)(size_t bytes, void* ctx);
typedef void (*fs_free_fn)(void* ptr, void* ctx);
fs_status fs_set_allocator(fs_alloc_fn alloc, fs_free_fn free, void* ctx);

/* ------------------------------------------------------------------- graph */
typedef struct fs_graph fs_graph;

/*
 * Uploads an incoming-edge CSR graph (Appendix "Data layout": row i lists the
 * nodes j with an edge j -> i; undirected graphs are passed symmetric).
 *   n        number of nodes, 1 <= n < 2^31
 *   row_ptr  n+1 int32, row_ptr[0] == 0, non-decreasing
 *   col_ind  row_ptr[n] int32 source ids, each in [0, n)
 *   weights  row_ptr[n] float32 edge weights w_ji, or NULL for unit weights
 * Self-loops and repeated edges are accepted and count with multiplicity.
 * Errors: FS_ERR_INVALID_ARG (n out of range, NULL arrays), FS_ERR_INVALID_CSR
 * (any CSR rule broken), FS_ERR_OUT_OF_MEMORY, FS_ERR_DEVICE.
 */
fs_status fs_graph_create(int64_t n, const int32_t* row_ptr, const int32_t* col_ind,
                          const float* weights, fs_graph** out);

/* Releases a graph.  FS_ERR_BUSY (graph untouched) while a sim still uses it. */
fs_status fs_graph_destroy(fs_graph* g);

typedef struct fs_graph_info {
    int64_t n;       /* nodes */
    int64_t nnz;     /* directed edges (CSR entries) */
    int32_t max_degree;
    int32_t weighted;
    double mean_degree;
} fs_graph_info;

fs_status fs_graph_get_info(const fs_graph* g, fs_graph_info* out);

/* --------------------------------------------------------------------- sim */
typedef struct fs_sim fs_sim;

typedef struct fs_sim_params {
    fs_dist ei;              /* E -> I holding-time law */
    fs_dist ir;              /* I -> R holding-time law */
    double beta;             /* per-edge transmission rate (per day), >= 0 */
    double dt;               /* fixed step (days), > 0 */
    uint64_t seed;           /* Philox key: draws are keyed by (seed, replica, step, node) */
    int32_t n_replicas;      /* independent replicas R, a power of two in [1, 64];
                                n * R must stay below 2^31 */
    int32_t storage;         /* FS_STORAGE_FP32 or FS_STORAGE_COMPACT */
    int32_t steps_per_graph; /* b: steps per captured hipGraph replay; 0 = launch eagerly */
    int32_t history_len;     /* per-step count ring length (>= 2); 0 = 1024 */
    int32_t record_rates;    /* nonzero: keep each unit's rate lambda of the last step */
    int32_t variant;         /* step kernel: 1 = streaming (bitmap read through the
                                caches), 2 = resident (bitmap held in LDS; n * n_replicas
                                <= 2^20), 3 = summary (an LDS summary with one bit per
                                group of units screens the bitmap reads), 0 = automatic:
                                resident when it fits, else summary for adaptive steps,
                                bitmaps over 8 MB, or uniform-degree graphs with at most
                                4 replicas, else streaming.  Results are identical. */
    int32_t heavy_degree;    /* degree bins: rows with more incoming edges than this get
                                their pressure from the heavy-row kernel (segments of
                                segment_edges edges, one wavefront each); 0 = 64,
                                -1 = no bins.  Results are identical for unit weights. */
    int32_t segment_edges;   /* edges per heavy-row segment, in [64, 2^20]; 0 = 512 */
    void* stream;            /* hipStream_t to run on; NULL = a stream owned by the sim */
    int32_t adaptive;        /* nonzero: adaptive step size (Section "Bernoulli tau-leaping",
                                adaptive step selection; the tau update of Algorithm 3):
                                step k+1 uses min(dt, epsilon / (max_i lambda_i + delta))
                                with the maximum over step k's rates of all units of all
                                replicas; dt is the cap, used by the first step after
                                creation or a state load.  FP32 storage only, variants
                                0/2/3 only, not in batches. */
    int32_t columns;         /* FS_COLUMNS_AUTO (0) or FS_COLUMNS_PLAIN (1) */
    double epsilon;          /* adaptive: bound on lambda * dt per step, > 0 */
    double delta;            /* adaptive: added to the largest rate, >= 0 */
    int32_t shedding;        /* FS_SHED_*; age-dependent forms need n * n_replicas < 2^29
                                and are not available in batches or the server */
    int32_t compaction;      /* nonzero: active-node compaction (Section "Epidemic-aware
                                compute sparsity"): at the start of every launch sequence
                                (each captured replay of steps_per_graph steps, or each
                                eager run of at most max(steps_per_graph, 64) steps) the
                                64-unit chunks whose units are all R are dropped from the
                                launches until the next state load or seeding.  R is
                                absorbing, so states, non-R ages and counts are identical
                                to the uncompacted run; the ages of R units in dropped
                                chunks stop advancing, and their recorded rates are 0.
                                Not available in batches or the server. */
    fs_dist shed_law;        /* the law of s(tau) (FS_SHED_DENSITY, FS_SHED_HAZARD) */
    double shed_scale;       /* A >= 0, finite */
} fs_sim_params;

/*
 * Creates a simulation of R replicas on a graph.  Every unit starts in S with
 * age 0 and infectivity 0; the step index starts at 0.
 * Errors: FS_ERR_INVALID_ARG (bad law parameters, dt <= 0, beta < 0, R not a
 * power of two in [1, 64], n*R >= 2^31, history_len == 1, unknown storage),
 * FS_ERR_OUT_OF_MEMORY, FS_ERR_DEVICE.
 */
fs_status fs_sim_create(fs_graph* g, const fs_sim_params* p, fs_sim** out);

/* Releases a sim (synchronises its stream first). */
fs_status fs_sim_destroy(fs_sim* s);

/*
 * Puts `count` listed nodes of one replica (replica = -1: every replica) into
 * `compartment` with age 0 and rebuilds their infectivity.  Seeds of the
 * paper's runs are exposed nodes (compartment FS_E; Listing "python_api").
 *   nodes  count int64 node ids, each in [0, n)
 */
fs_status fs_sim_seed(fs_sim* s, int32_t replica, int64_t count, const int64_t* nodes,
                      int32_t compartment);

/* Largest `count` fs_sim_seed_noalloc accepts (512 KiB of staging per GPU). */
#define FS_SEED_NOALLOC_MAX 65536

/*
 * fs_sim_seed for callers that cannot allocate device memory (serving loops
 * that must not call hipMalloc, harnesses that forbid it): the same
 * arguments, validation, kernels and result, but the node list is staged in
 * a fixed device array of FS_SEED_NOALLOC_MAX int64 ids that the library
 * holds on each GPU it runs on until the process ends, and the call makes no
 * device allocation of its own (no hipMalloc, hipMallocAsync or allocator
 * hook).  `nodes` is a host array, read before the call returns; like
 * fs_sim_seed it synchronises the sim's stream.
 * Errors: FS_ERR_INVALID_ARG for count > FS_SEED_NOALLOC_MAX (nothing is
 * changed) and every error of fs_sim_seed.
 * Every call on one GPU shares that GPU's staging array: calls that overlap
 * in time on one GPU (from several host threads) race and must be serialised
 * by the caller; sequential calls are independent.
 */
fs_status fs_sim_seed_noalloc(fs_sim* s, int32_t replica, int64_t count, const int64_t* nodes,
                              int32_t compartment);

/*
 * Queues n_steps steps (Algorithm 3, fixed dt) on the sim's stream and
 * returns without waiting.  With steps_per_graph = b > 0, floor(n/b) replays
 * of a captured hipGraph of b steps run first, then n mod b single launches
 * (Algorithm 2 captures the step loop the same way).  Step k of replica r
 * draws from Philox4x32-10 at counter (node, k mod 2^32, r, 0) under key
 * (seed low, seed high).
 */
fs_status fs_step(fs_sim* s, int64_t n_steps);

/* Waits for all queued work of the sim; reports device errors. */
fs_status fs_sync(fs_sim* s);

/* Index of the next step (= steps run since creation or the last set_state). */
fs_status fs_step_index(fs_sim* s, int64_t* out);

/*
 * Exact S, E, I, R counts of one replica after the latest queued step,
 * recounted from the stored states (synchronises): the count_by_state() of
 * Listing "python_api", [S, E, I, R].  out: 4 int64.
 */
fs_status fs_counts(fs_sim* s, int32_t replica, int64_t out[4]);

/*
 * Per-step counts (the S, E, I, R tallies each step kernel records: the
 * count_by_state() of Listing "python_api" after every step, from which peak
 * prevalence and attack rate follow) for steps first_step ..
 * first_step+n-1, where step k's row holds the counts after step k ran.  Only the last history_len steps since creation or the last
 * fs_set_state are kept; older or future rows give FS_ERR_INVALID_ARG.
 *   out: n x 4 int64, row-major.  Synchronises.
 */
fs_status fs_history(fs_sim* s, int32_t replica, int64_t first_step, int64_t n, int64_t* out);

/* Step sizes (days) of steps first_step .. first_step + n - 1, into out[n]
 * (host).  Fixed-step sims return dt for every step; adaptive ones the step
 * each step used, within the same window of recorded steps as fs_history
 * (FS_ERR_INVALID_ARG outside it).  Synchronises the sim's stream. */
fs_status fs_step_sizes(fs_sim* s, int64_t first_step, int64_t n, double* out);

/*
 * Copies one replica's state out (synchronises): the snapshot of the
 * persistent state X, tau and step_id that the capture algorithm takes
 * (Algorithm "Fused Renewal Engine with CUDA Graph: Capture").
 *   state       n int32 compartments
 *   age_days    n float32 ages in days   (FS_STORAGE_FP32; NULL otherwise)
 *   age_steps   n uint16 ages in steps   (FS_STORAGE_COMPACT; NULL otherwise)
 *   step_index  receives the index of the next step (may be NULL)
 */
fs_status fs_get_state(fs_sim* s, int32_t replica, int32_t* state, float* age_days,
                       uint16_t* age_steps, int64_t* step_index);

/*
 * Overwrites one replica's state and age and rebuilds its infectivity: the
 * restore from a snapshot of the capture algorithm (Algorithm "Fused Renewal
 * Engine with CUDA Graph: Capture"); checkpoint restore and test set-up.  step_index >= 0 also sets the sim-wide
 * step index (all replicas share it) and resets the count history; -1 keeps
 * it.  Argument formats as in fs_get_state; states must lie in [0, 3].
 */
fs_status fs_set_state(fs_sim* s, int32_t replica, const int32_t* state, const float* age_days,
                       const uint16_t* age_steps, int64_t step_index);

/*
 * Rates lambda_i of the latest step for one replica (beta*pressure for S,
 * the hazard for E and I, 0 for R), as the step kernel computed them in FP32.
 * Requires record_rates at creation.  out: n float32.  Synchronises.
 */
fs_status fs_get_rates(fs_sim* s, int32_t replica, float* out);

/*
 * Degree-binned dispatch (Section "CSR traversal strategies and
 * auto-dispatch", Appendix "Degree-heterogeneous graphs"): rows of degree >
 * heavy_degree are split into segments of segment_edges edges whose partial
 * pressures a separate wavefront-per-segment launch computes before each
 * step launch; the other rows gather in the step kernel itself.
 * fs_sim_set_bins sets the thresholds (0 selects the defaults, heavy_degree
 * -1 disables the bins); fs_sim_get_bins reports them and the segment count.
 * fs_sim_tune times trial_steps steps for each candidate threshold pair from
 * the current state, restores the state after each trial (the step index and
 * history are left as they were) and keeps the fastest.  Synchronises.
 */
fs_status fs_sim_set_bins(fs_sim* s, int32_t heavy_degree, int32_t segment_edges);
fs_status fs_sim_get_bins(fs_sim* s, int32_t* heavy_degree, int32_t* segment_edges, int64_t* segments);
fs_status fs_sim_tune(fs_sim* s, int32_t trial_steps, int32_t* heavy_degree, int32_t* segment_edges);

/*
 * The autotuner (Appendix "Degree-heterogeneous graphs and auto-dispatch",
 * subsection "Auto-dispatch", which picks the traversal strategy from a
 * graph's degree statistics): times trial_steps steps from the current
 * state for each candidate configuration -- the step variant (when
 * `variants` is set: every variant the sim may switch to; the resident one
 * holds at most 2^20 units, adaptive sims keep an LDS variant) and the
 * degree bins (heavy_degree in {none, 8, 12, 16, 24, 32, 64, 128, 256} below
 * the maximum degree; segment_edges in {256, 1024} where binned rows gather
 * segment partials, one value where they take pushed pressure) -- restores
 * the state after each trial and keeps the fastest.  The sim's configuration
 * at entry is always among the candidates.
 * With cache_path set, the choice is keyed by a signature of the graph and
 * the run (n, edges, degree histogram, replicas, storage, weights, shedding,
 * adaptive steps, compaction, rate recording, device compute units): a
 * cached choice is applied without trials, and a new one is appended to the
 * file (one text line per signature; the last line of a signature wins), so
 * it persists across processes.  Synchronises.
 */
typedef struct {
    int32_t trial_steps;    /* steps per timed trial, in [1, 4096] */
    int32_t variants;       /* 1: also choose the step variant; 0: bins only */
    const char* cache_path; /* NULL: no cache */
} fs_tune_params;

typedef struct {
    int32_t variant;        /* chosen step variant: 1 stream, 2 resident, 3 summary */
    int32_t heavy_degree;   /* chosen bins (as fs_sim_get_bins reports them) */
    int32_t segment_edges;
    int32_t from_cache;     /* 1: taken from the cache, no trials run */
    int32_t trials;         /* timed candidates */
    int32_t pad;
    double us_per_step;     /* the chosen candidate's trial time per step (0 from the cache) */
    double entry_us_per_step; /* the trial time of the configuration at entry (0 from the cache) */
    uint64_t signature;
} fs_tune_result;

fs_status fs_sim_autotune(fs_sim* s, const fs_tune_params* p, fs_tune_result* out);

/* The sim's current step variant: 1 stream, 2 resident, 3 summary. */
fs_status fs_sim_get_variant(fs_sim* s, int32_t* variant);

/* Bits per column of the sim's transposed graph copy: 20, 24 or 27 when
 * packed (FS_COLUMNS_AUTO), else 32. */
fs_status fs_sim_get_column_bits(fs_sim* s, int32_t* bits);

/* ------------------------------------------------- building-block checks */
/*
 * Evaluates the device hazard of `law` at n ages with the same code the step
 * kernel runs.  storage FS_STORAGE_FP32: ages are float32 days;
 * FS_STORAGE_COMPACT: ages are uint16 step counts with tau = n*dt.
 *   ages: n values (host), out: n float32 hazards per day (host).
 */
fs_status fs_eval_hazard(const fs_dist* law, int32_t storage, double dt, int64_t n,
                         const void* ages, float* out);

/*
 * Evaluates a shedding profile (form FS_SHED_DENSITY or FS_SHED_HAZARD, law,
 * scale A) at n ages with the same device arithmetic the step kernels use.
 * ages and out as for fs_eval_hazard.  Synchronises.
 */
fs_status fs_eval_shedding(const fs_dist* law, int32_t form, double scale, int32_t storage, double dt, int64_t n,
                           const void* ages, float* out);

/*
 * Evaluates Philox4x32-10 on the device for n counters (n x 4 uint32, host)
 * under key (seed low, seed high); out: n x 4 uint32 (host).
 */
fs_status fs_eval_philox(int64_t n, const uint32_t* ctr, uint64_t seed, uint32_t* out);

/* Library version string. */
const char* fs_version(void);

/* ------------------------------------------------------- Markovian engine
 * The companion engine for Markovian dynamics (Section "Markovian engine",
 * Algorithm "Markovian Engine: One Tau-Leaping Step").  Rates are piecewise
 * constant: a susceptible node beta * I_i (I_i: its infectious in-neighbours;
 * unit-weight graphs only), an exposed node sigma, an infectious node gamma,
 * a removed node 0.  Every step takes
 *   tau = min(theta N / Lambda, p_max / max_i lambda_i, tau_max)
 * (Lambda: the total rate; a zero denominator drops its term), fires node i
 * with probability 1 - exp(-lambda_i tau) (Philox keyed by (seed, step,
 * node) as for the renewal step, replica 0), and updates the influences:
 * by integer pushes along the outgoing edges of the nodes whose
 * infectiousness changed when they are few (Inertial Mode), else by a full
 * recount (Control Mode).  Both give the same integer influences on every
 * node that can still use them, so the result does not depend on the mode:
 * under SEIR and SIR pushes skip targets that are no longer susceptible (no
 * such node becomes susceptible again), so there the influence reported for
 * a node outside S may be stale; under SIS every node's is exact.  One
 * replica per engine.
 */
#define FS_MARKOV_SEIR 0 /* S -> E -> I -> R */
#define FS_MARKOV_SIR 1  /* S -> I -> R */
#define FS_MARKOV_SIS 2  /* S -> I -> S */

typedef struct fs_markov fs_markov;

typedef struct fs_markov_params {
    int32_t model;           /* FS_MARKOV_* */
    int32_t pad;
    double beta;             /* per infectious in-neighbour (per day), >= 0 */
    double sigma;            /* E -> I rate (FS_MARKOV_SEIR), >= 0 */
    double gamma;            /* I -> R (or I -> S) rate, >= 0 */
    double theta;            /* expected events per node per step bound, > 0 (the paper's default 0.01) */
    double p_max;            /* largest transition probability per step, > 0 (default 0.1) */
    double tau_max;          /* largest step (days), > 0 */
    uint64_t seed;
    int32_t steps_per_graph; /* b: steps per captured hipGraph replay; 0 = launch eagerly */
    int32_t history_len;     /* per-step ring length (>= 2); 0 = 1024 */
    int64_t inertial_max;    /* events per step up to which pushes update the influences;
                                0 = automatic (events * mean degree < nnz / 8), -1 = always recount */
    void* stream;            /* hipStream_t; NULL = a stream owned by the engine */
} fs_markov_params;

/* Creates an engine on a unit-weight graph, every node in S.  Errors:
 * FS_ERR_INVALID_ARG (a weighted graph, unknown model, bad rates or step
 * parameters), FS_ERR_OUT_OF_MEMORY, FS_ERR_DEVICE.  The first engine of a
 * graph builds the graph's outgoing CSR (kept with the graph). */
fs_status fs_markov_create(fs_graph* g, const fs_markov_params* p, fs_markov** out);
fs_status fs_markov_destroy(fs_markov* m);
/* Puts `count` listed nodes (caller's ids) into `compartment`.  Synchronises. */
fs_status fs_markov_seed(fs_markov* m, int64_t count, const int64_t* nodes, int32_t compartment);
/* Loads n states (caller's order), sets the step index (-1: keep) and the
 * elapsed time.  Synchronises. */
fs_status fs_markov_set_state(fs_markov* m, const int32_t* state, int64_t step_index, double elapsed);
/* Queues n_steps steps (asynchronous, like fs_step). */
fs_status fs_markov_step(fs_markov* m, int64_t n_steps);
fs_status fs_markov_sync(fs_markov* m);
/* States and influences (n int32 each, caller's order, either may be NULL),
 * the step index and the elapsed time.  Synchronises. */
fs_status fs_markov_get_state(fs_markov* m, int32_t* state, int32_t* influence, int64_t* step_index,
                              double* elapsed);
/* Per-step records of steps [first_step, first_step + n) within the ring:
 * counts (n x 4 int64), step sizes tau (n double, as the device used them,
 * FP32) and events (n int64, nodes that changed infectiousness); any may be
 * NULL.  Synchronises. */
fs_status fs_markov_history(fs_markov* m, int64_t first_step, int64_t n, int64_t* counts, double* taus,
                            int64_t* events);

/* ---------------------------------------------------------------- batches
 * A batch advances several sims together, one fused step launch per step
 * for all of them (Algorithm 3's fused step over a table of simulations
 * instead of one): each member keeps its own graph, laws, beta, dt, seed,
 * replicas, step index and count history, and gets exactly the results it
 * gets alone (same draws, same states, same counts).  Small simulations that
 * cannot fill the GPU alone fill it together.
 *
 * Members must be created with variant = 1 (streaming step), the batch's
 * storage, and agree on weights (all weighted or none) and record_rates.
 * While a sim belongs to a batch, its device work runs on the batch's stream:
 * fs_counts, fs_history, fs_get_state, fs_set_state, fs_get_rates and
 * fs_sim_seed still work on it; fs_step, fs_sim_set_bins, fs_sim_tune and
 * fs_sim_destroy return FS_ERR_BUSY until it is removed.
 */
typedef struct fs_batch fs_batch;

/* Creates an empty batch on the current HIP device.  storage is
 * FS_STORAGE_FP32 or FS_STORAGE_COMPACT; stream is a hipStream_t to run on,
 * or NULL for a stream owned by the batch. */
fs_status fs_batch_create(int32_t storage, void* stream, fs_batch** out);
/* Waits for queued work, removes every member (they keep their state) and
 * releases the batch. */
fs_status fs_batch_destroy(fs_batch* b);
/* Adds sim s (its queued work is finished first).  FS_ERR_INVALID_ARG when s
 * does not meet the member rules above, FS_ERR_BUSY when s is already in a
 * batch. */
fs_status fs_batch_add(fs_batch* b, fs_sim* s);
/* Removes sim s after the batch's queued work; s returns to its own stream. */
fs_status fs_batch_remove(fs_batch* b, fs_sim* s);
/* Number of members. */
fs_status fs_batch_size(fs_batch* b, int32_t* members);
/* Queues n_steps steps of every member (asynchronous, like fs_step). */
fs_status fs_batch_step(fs_batch* b, int64_t n_steps);
/* Waits for the batch's queued work. */
fs_status fs_batch_sync(fs_batch* b);

/* ----------------------------------------------------------------- server
 * A scenario server: callers submit independent scenario solves (a resident
 * graph, laws and rates, replicas, seeds, a number of steps) from any
 * thread; a worker thread admits queued requests in arrival order while the
 * device-memory budget and the slot limit allow.  Small requests (fewer than
 * 2^18 node-replica units) advance together in batches (see above; requests
 * on weighted graphs and on unit-weight graphs form one batch each) a few
 * steps at a time, so one that arrives while others are on the GPU joins
 * them at the next round; large ones (which fill the GPU by themselves) run
 * on a stream of their own, at most two at once, with every step queued at
 * admission, so their kernels overlap each other's and the batch's.  The
 * worker retires requests as they reach their step count.  A request's
 * counts equal those of the same sim run alone.
 */
typedef struct fs_server fs_server;

typedef struct fs_server_params {
    int64_t memory_budget;   /* device bytes the admitted requests may hold; 0 = 80% of
                                the free device memory at creation */
    int32_t max_active;      /* most requests on the device at once; 0 = 64 */
    int32_t steps_per_round; /* steps run between admission checks; 0 = 25 */
    int32_t storage;         /* FS_STORAGE_FP32 or FS_STORAGE_COMPACT for every request */
    int32_t pad;
    void* stream;            /* hipStream_t to run on; NULL = a stream owned by the server */
} fs_server_params;

typedef struct fs_request {
    fs_graph* graph;         /* resident graph; must outlive the request (fs_graph_destroy
                                returns FS_ERR_BUSY until the request is collected) */
    fs_sim_params params;    /* laws, beta, dt, seed and n_replicas; storage, variant,
                                steps_per_graph, history_len, record_rates and stream are
                                set by the server */
    int64_t n_steps;         /* steps to run, in [1, 2^20] */
    int64_t n_seeds;         /* nodes seeded into E at age 0 in every replica */
    const int64_t* seeds;    /* host array, copied at submission */
} fs_request;

typedef struct fs_request_info {
    double t_submit;         /* server clock (fs_server_clock) at submission */
    double t_admit;          /* ... when the request's sim was created */
    double t_done;           /* ... when its counts were copied out */
    int64_t n_steps;
    int32_t n_replicas;
    fs_status status;        /* FS_OK, or the failure that ended the request */
} fs_request_info;

typedef struct fs_server_stats_t {
    int64_t queued;          /* submitted, not yet admitted */
    int64_t active;          /* on the device */
    int64_t memory_in_use;   /* estimated device bytes of the active requests */
    int64_t memory_budget;
    int64_t rounds;          /* batch rounds run so far */
} fs_server_stats_t;

/* Creates a server on the current HIP device and starts its worker thread. */
fs_status fs_server_create(const fs_server_params* p, fs_server** out);
/* Queues a request and returns its id (> 0).  FS_ERR_BUDGET when the request
 * alone needs more memory than the budget; FS_ERR_INVALID_ARG for bad
 * arguments (laws and rates are validated when the request is admitted: a
 * bad one ends that request with FS_ERR_INVALID_ARG). */
fs_status fs_server_submit(fs_server* sv, const fs_request* rq, int64_t* id);
/* Waits until request id has finished or timeout_s seconds passed (< 0:
 * no limit); *done = 1 when it has finished. */
fs_status fs_server_wait(fs_server* sv, int64_t id, double timeout_s, int32_t* done);
/* Collects a finished request: copies its per-step counts to history
 * ([n_steps][n_replicas][4] int64, S E I R after each step; may be NULL) and
 * its timing to info (may be NULL), then forgets the request.  Returns the
 * request's failure status if it failed, FS_ERR_BUSY if it has not finished. */
fs_status fs_server_result(fs_server* sv, int64_t id, int64_t* history, fs_request_info* info);
/* Current queue, device and memory figures. */
fs_status fs_server_stats(fs_server* sv, fs_server_stats_t* out);
/* Cancels queued requests, lets admitted ones finish, stops the worker and
 * releases the server. */
fs_status fs_server_destroy(fs_server* sv);
/* The server clock (seconds, monotonic) used by fs_request_info. */
double fs_server_clock(void);

#ifdef __cplusplus
}
#endif

#endif /* FS_H */
