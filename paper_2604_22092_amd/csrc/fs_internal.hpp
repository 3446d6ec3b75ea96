// Layouts shared by the step kernels and the host runtime of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fsi {

enum : int32_t { ST_S = 0, ST_E = 1, ST_I = 2, ST_R = 3 };
enum : int32_t { K_EXP = 0, K_LN = 1, K_WB = 2, K_ERL = 3 };

// Workgroup size of the helper kernels (four wave64 wavefronts).
constexpr int WG = 256;
// Workgroup size of the count reduce (sixteen wavefronts: a step of the
// streaming variant with many replicas leaves up to max_step_grid(R) * 4R
// partial counts, one block reads them all).
constexpr int RED_TPB = 1024;
// Step kernel variants, all walking 64-unit chunks per wavefront:
//  MODE_STREAM   bitmap read through the caches; STREAM_TPB threads per workgroup;
//  MODE_RESIDENT the whole bitmap (up to RESIDENT_BITS units) held in LDS;
//  MODE_SUMMARY  an LDS summary with one bit per group of units (set when any
//                unit of the group is infectious; at most SUMMARY_BITS bits)
//                screens the reads of the bitmap, which stays in global memory.
// The two LDS variants run one RESIDENT_TPB-thread workgroup per compute unit.
enum : int32_t { MODE_STREAM = 0, MODE_RESIDENT = 1, MODE_SUMMARY = 2 };
constexpr int STREAM_TPB = 256;
constexpr int RESIDENT_TPB = 1024;
constexpr uint32_t RESIDENT_BITS = 1u << 20;
constexpr uint32_t SUMMARY_BITS = 1u << 20;
// Light rows of a chunk whose rows all have the same degree d <= UNIFORM_MAX_DEG
// have their edge slots loaded ahead with the chunk's state (the preload depth).
#ifndef FS_UMAX
#define FS_UMAX 12
#endif
constexpr int UNIFORM_MAX_DEG = FS_UMAX;
// Entries of the hazard table of a fixed-step sim (StepArgs::htab).
constexpr uint32_t HTAB_LEN = 8192;
// Bitmaps are allocated in whole 512-unit tiles (8 words of 64 bits).
constexpr uint32_t BITMAP_TILE = 512;
// Active-chunk compaction: the refresh runs one workgroup of WG_REFRESH
// threads, each taking 16 flags per tile, so flag arrays are padded to whole
// tiles of LIVE_TILE chunks.
constexpr int WG_REFRESH = 1024;
constexpr uint32_t LIVE_TILE = 16 * WG_REFRESH;

// Hazard parameters, prepared on the host in double precision and rounded
// once.  Ages reach the device in a unit u: days (FP32 storage) or steps of
// dt (compact storage, integer ages n with tau = n*dt).
//   log-normal: h = K / (x * erfcx(z)),  z = (ln x + c) * g
//               K = sqrt(2/pi)/(sigma*u), c = ln u - mu, g = 1/(sigma sqrt 2)
//   Weibull:    h = K * exp((ln x + c) * g)
//               K = shape/scale, c = ln(u/scale), g = shape - 1
//   Erlang:     h = K / R(1/(xr*x)), xr = rate*u, K = rate,
//               R(y) = sum_{j<k} (k-1)!/j! y^(k-1-j)
//   exponential h = K
struct HazardDev {
    int32_t kind;
    int32_t k;
    float K;
    float c_hi, c_lo;
    float g_hi, g_lo;
    float x_hi, x_lo;
};

// Shedding profile s(x) of an infectious unit of age x (Eq. (infectivity)),
// in the age unit u of the storage, prepared on the host in double precision
// with the scale A folded in:
//   hazard form (density == 0): s = A h(x), the hazard of `hz` with K scaled by A;
//   density form (density != 0), s = A f(x) by hz.kind:
//     log-normal:  s = K exp(-z^2) / x,  z = (ln x + c) g,  K = A / (sigma sqrt(2 pi) u)
//     Weibull:     s = K exp(g t - exp(m t)),  t = ln x + c,  K = A shape / scale,
//                  g = shape - 1, m = shape
//     Erlang:      s = K exp((k - 1) ln y - y - lf),  y = xr x,  K = A rate, lf = ln (k - 1)!
//     exponential: s = K exp(-y),  y = xr x,  K = A rate
//   with c, g and xr = rate u as in HazardDev; x = 0 gives s0 (the right limit).
struct ShedDev {
    HazardDev hz;
    int32_t density;
    float s0;
    float m_hi, m_lo;
    float lf_hi, lf_lo;
};

// The laws of a sim in device memory (StepArgs::hz_dev, shed_dev): the step
// reads them there, where a hazard or a shedding value is evaluated, so they
// hold no registers through the walk.
struct LawsDev {
    HazardDev hz[2]; // [0] E -> I, [1] I -> R
    ShedDev shed;
};

// Device-resident control block of a simulation.  `step` is the index of the
// first step of the launch sequence being run: step launch j of a sequence
// runs step (step + j), and the reduce launch that ends the sequence adds its
// length (its last block to finish, counted in `done`).  Captured sequences
// therefore need no per-replay arguments and no step kernel touches a shared
// counter.
struct Ctl {
    unsigned long long step;
    unsigned long long adapt_from; // adaptive step: the step that uses the cap (creation, state load)
    uint32_t done;                 // blocks of the running reduce launch that have finished; 0 between launches
    uint32_t pad;
};

// Kernel arguments of one fused step launch.
struct StepArgs {
    const int32_t* row_ptr;
    const int32_t* col_ind;
    const float* weights; // nullptr: unit weights
    void* state;          // int32 (FP32 storage) or uint8 (compact), [n][R]
    void* age;            // float days or uint16 steps, [n][R]
    void* iota0;          // infectivity bitmaps, bit u = 1{X_u = I}; step k reads
    void* iota1;          // iota[k & 1] and writes iota[(k + 1) & 1]
    float* rates;         // optional per-unit lambda (debug), [n][R]; nullptr: none
    const Ctl* ctl;
    uint32_t* part;       // per-workgroup counts [chunk slot][grid][R][4]
    int32_t n;
    int32_t lgR;          // R = 1 << lgR replicas
    uint32_t step_off;    // j: this launch runs step ctl->step + j, partial slot j
    // MODE_SUMMARY: one summary bit per group of 32 * 2^sum_shift units
    // (2^sum_shift 32-bit bitmap words)
    int32_t sum_shift;
    int32_t same_kind;    // E and I laws share a kind: one hazard call per lane
    int32_t pad0;
    HazardDev hz[2];      // [0] E -> I, [1] I -> R
    // the same two laws in device memory (LawsDev::hz)
    const HazardDev* hz_dev;
    float beta;
    float dt;
    uint32_t key0, key1;  // Philox key = (seed low, seed high)
    // degree bins: rows with degree > heavy_deg take their pressure from the
    // segment partials of the heavy-row kernel (first segment heavy_first[node],
    // ceil(degree / seg_edges) segments); nullptr heavy_first: no such rows
    const int32_t* heavy_first;
    const void* seg_part; // [segment][R]: uint32 counts, or float with weights
    int32_t heavy_deg;
    int32_t seg_edges;
    // pushed pressure of the binned rows (unit weights and constant shedding,
    // where a row's pressure is the integer count of its infectious
    // in-neighbours; nullptr hub_T: the rows read their segment partials).
    // Binned rows are the internal nodes [hub_base, n) of the degree-sorted
    // order, hub unit h = (node - hub_base) * R + replica.  Step k takes h's
    // pressure as hub_T[(k - 1) & 1][h] + hub_D[k % 3][h] (modulo 2^32),
    // stores it into hub_T[k & 1][h] and clears hub_D[(k + 2) % 3][h]; a unit
    // of node j entering I (E -> I) or leaving it (I -> R) in step k adds +1
    // or -1 to hub_D[(k + 1) % 3][h] of every binned row listing j as an
    // in-neighbour (hub_out_idx[hub_out_ptr[j] .. hub_out_ptr[j + 1]), the
    // rows' hub indices, once per occurrence).
    uint32_t* hub_T;      // [2][hub_units]
    uint32_t* hub_D;      // [3][hub_units]
    const int32_t* hub_out_ptr;
    const int32_t* hub_out_idx;
    int32_t hub_base;
    uint32_t hub_units;
    // light rows in wavefront-transposed order: for the Q = 64/R nodes of chunk
    // c, edge j of every row with more than j light edges is stored at
    // chunk_meta[c].x + (edges j' < j of the chunk) + (rank of the row among
    // the chunk's rows with more than j edges); chunk_meta[c].y is the light
    // degree all the chunk's rows share (full chunks only), or 255.  ldeg[node]
    // is the row's degree, or HEAVY_ROW for a binned row.
    const uint16_t* ldeg;
    const uint2* chunk_meta;
    // the caller's id of each (internal) node: the draws are keyed by it
    const int32_t* orig_id;
    // every chunk uniform with this degree (<= UNIFORM_MAX_DEG) and no heavy
    // rows: chunk c starts at slot c * (64 / R) * udeg; else -1
    int32_t udeg;
    // bits per column of a uniform layout's packed columns (20, 24 or 27), or
    // 0 for 32-bit columns; col_t then holds the packed words (see the step)
    int32_t pbits;
    const int32_t* col_t;
    const float* w_t;
    // MODE_SUMMARY: summary of the step's input bitmap, sum_bits bits
    const uint32_t* summary;
    uint32_t sum_bits;
    // adaptive step size: dt is the cap; step k reads the per-workgroup rate
    // maxima of step k-1 from lam_part[((k-1) & 1) * grid ..] and writes its
    // own to lam_part[(k & 1) * grid ..]; block 0 records the step in
    // dt_hist[k % hist_len]
    int32_t adaptive;
    float* lam_part;
    float* dt_hist;
    float eps, delta;
    uint32_t hist_len;
    uint32_t pad1;
    // age-dependent shedding (shedding kernels only): float s(tau) of every
    // unit that is infectious, [n][R], ping-pong like the bitmaps (only units
    // whose bit is set are ever read)
    void* shed0; // float32 (FP32 storage) or IEEE binary16 (compact) per unit
    void* shed1;
    const ShedDev* shed_dev; // the profile s, in device memory (LawsDev::shed)
    // active-chunk compaction (nullptr act: off): the launch walks the chunks
    // act[2 .. 2 + act[0]) (ascending); every other chunk holds only R units
    // and is skipped, and act[1] R units per replica are added to the counts
    // of workgroup 0.  When live is set (the last step of a launch sequence,
    // whose flags the next sequence's refresh reads), every processed chunk
    // stores 1 in live[chunk] when it held a unit that is not R at the start
    // of the step, else 0.
    const uint32_t* act;
    uint8_t* live;
    // hazards at the ages fixed steps reach (fixed-step sims; nullptr: none).
    // A unit entering E or I has age 0, and each step without a transition
    // adds dt in FP32, so its age is a_m after m steps: a_0 = 0, a_{m+1} =
    // a_m + dt (compact storage: a_m = m).  htab[m] = (a_m, hazard of the
    // E -> I law at a_m, of the I -> R law, 0) for m < htab_len, evaluated by
    // the step's own hazard code; a unit whose age equals a_m, m = rint(age *
    // htab_inv), takes its hazard from the table, any other age (a state
    // load's arbitrary ages, ages past the table) is evaluated.
    const float4* htab;
    uint32_t htab_len;
    float htab_inv;
};

// Arguments of the summary launch that follows a step launch (or a bitmap
// rebuild): it summarises bitmap iota[(ctl->step + step_off + after) & 1].
struct SumArgs {
    const unsigned long long* iota0;
    const unsigned long long* iota1;
    const Ctl* ctl;
    unsigned long long* summary;
    uint32_t words;     // 64-bit words per bitmap
    uint32_t sum_words; // 64-bit words of the summary
    int32_t sum_shift;  // groups of 32 * 2^sum_shift units, as in StepArgs
    uint32_t step_off;
    uint32_t after;     // 1: the bitmap written by step ctl->step + step_off
    uint32_t pad;
};

constexpr uint16_t HEAVY_ROW = 0xFFFF;

// One segment of a heavy row: edges [e_begin, e_end) of row `row`.
struct Segment {
    int32_t row, e_begin, e_end, pad;
};

// Kernel arguments of the heavy-row pressure launch of one step.
struct HeavyArgs {
    const int32_t* col_ind;
    const float* weights;
    const Segment* segs;
    void* seg_part;
    const void* iota0;
    const void* iota1;
    const Ctl* ctl;
    uint32_t nseg;
    int32_t lgR;
    uint32_t step_off;
    uint32_t units;     // N * R: the bits the resident variant copies into LDS
    const void* shed0; // shedding kernels: the s(tau) buffers of StepArgs
    const void* shed1;
    const void* state;  // start-of-step states: segments of rows that are not S
    int32_t storage;    // in any replica are skipped (0: int32 states, 1: uint8)
    int32_t pad2;
};

// One member's count reduction in a batch: per-workgroup partials of G
// workgroups, C = 4R counters each, summed into the H-slot history ring.
struct RedArgs {
    Ctl* ctl;
    const uint32_t* part;
    uint32_t* hist;
    uint32_t G, C, H, pad;
};

// Upper bound on step workgroups (they loop over tiles beyond it), chosen so
// the per-workgroup count partials of a launch sequence stay small.
inline uint32_t max_step_grid(int R) { return R <= 4 ? 16384u : (R <= 16 ? 4096u : 2048u); }

} // namespace fsi
