// The fused step of the renewal tau-leap (FlashSpread, arXiv 2604.22092,
// Algorithm 3 with Eq. (influence), Eq. (infectivity), Proposition 1 and the
// Bernoulli tau-leap rule) as templates, instantiated by the kernel sources
// of the library (constant shedding in one, age-dependent shedding in the
// other, so the two compile in parallel).
#pragma once

#include <hip/hip_runtime.h>

#include "fs_device.hpp"
#include "fs_internal.hpp"

namespace fsk {

using namespace fsi;

template <int STORAGE>
struct Store;
template <>
struct Store<0> {
    using state_t = int32_t;
    using age_t = float;
    static constexpr uint32_t shed_bytes = 4; // s(tau) as float32
};
template <>
struct Store<1> {
    using state_t = uint8_t;
    using age_t = uint16_t;
    static constexpr uint32_t shed_bytes = 2; // s(tau) as IEEE binary16
};

__device__ __forceinline__ uint32_t age_bits(float a) { return __float_as_uint(a); }
__device__ __forceinline__ uint32_t age_bits(uint16_t a) { return a; }
template <class T>
__device__ __forceinline__ float age_from_bits(uint32_t w);
template <>
__device__ __forceinline__ float age_from_bits<float>(uint32_t w) { return __uint_as_float(w); }
template <>
__device__ __forceinline__ float age_from_bits<uint16_t>(uint32_t w) { return (float)w; }
__device__ __forceinline__ float age_units(float a) { return a; }
__device__ __forceinline__ float age_units(uint16_t a) { return (float)a; }
__device__ __forceinline__ float age_next(float a, float dt) { return a + dt; }
__device__ __forceinline__ uint16_t age_next(uint16_t a, float) { return a == 65535 ? a : (uint16_t)(a + 1); }
template <class T>
__device__ __forceinline__ T age_from_raw(uint32_t w);
template <>
__device__ __forceinline__ float age_from_raw<float>(uint32_t w) { return __uint_as_float(w); }
template <>
__device__ __forceinline__ uint16_t age_from_raw<uint16_t>(uint32_t w) { return (uint16_t)w; }
__device__ __forceinline__ uint32_t age_to_raw(float a) { return __float_as_uint(a); }
__device__ __forceinline__ uint32_t age_to_raw(uint16_t a) { return a; }

// Infectivity is held as one bit per unit (bit u = 1{X_u = I}); with constant
// shedding s = 1 this is the exact value of Eq. (infectivity) without beta.
__device__ __forceinline__ uint32_t bit_at(const uint32_t* __restrict__ w, uint32_t b)
{
    return (w[b >> 5] >> (b & 31)) & 1u;
}

__device__ __forceinline__ uint32_t lds_bit(const uint32_t* __restrict__ w, uint32_t b)
{
    return __builtin_amdgcn_ubfe(w[b >> 5], b & 31, 1);
}

// Raw buffer accesses.  Word 3 of the descriptor (0x00020000) is the gfx9
// raw-buffer format: 32-bit data, no swizzle, range checked against the byte
// count in word 2.  An access whose offset is outside that range reads 0 and
// writes nothing, with no memory request.  The step uses this instead of
// branches: lanes and slots that must not touch memory get offset OOB, and
// every path issues the same memory instructions, so the compiler can wait
// for exactly the loads it needs while later loads are still in flight.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int BUF_WORD3 = 0x00020000;
constexpr uint32_t OOB = 0x80000000u; // beyond every byte range used here (< 2^31)

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, BUF_WORD3);
}
__device__ __forceinline__ uint32_t ld32(rsrc_t r, uint32_t off) { return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0); }
__device__ __forceinline__ void st32(rsrc_t r, uint32_t off, uint32_t v) { __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)off, 0, 0); }

// Stored shedding values (age-dependent shedding): float32 with FP32 storage,
// IEEE binary16 with compact storage (its value rounded to nearest even;
// every binary16 value is exact in float).  shed_at reads unit `unit` when
// `take` is set, else nothing (0).
__device__ __forceinline__ float half_bits_to_float(uint32_t h) { return (float)__builtin_bit_cast(_Float16, (uint16_t)h); }
__device__ __forceinline__ uint32_t float_to_half_bits(float f) { return __builtin_bit_cast(uint16_t, (_Float16)f); }
template <int STORAGE>
__device__ __forceinline__ float shed_at(rsrc_t r, uint32_t unit, bool take)
{
    if (STORAGE == 0) return __uint_as_float(ld32(r, take ? unit << 2 : OOB));
    return half_bits_to_float(__builtin_amdgcn_raw_buffer_load_b16(r, take ? (int)(unit << 1) : (int)OOB, 0, 0));
}
template <int STORAGE>
__device__ __forceinline__ void shed_put(rsrc_t r, uint32_t unit, bool put, float v)
{
    if (STORAGE == 0) st32(r, put ? unit << 2 : OOB, __float_as_uint(v));
    else __builtin_amdgcn_raw_buffer_store_b16((uint16_t)float_to_half_bits(v), r, put ? (int)(unit << 1) : (int)OOB, 0, 0);
}

// Element access of the storage types through a buffer descriptor.
template <class T>
struct BufIO;
template <>
struct BufIO<int32_t> {
    __device__ static uint32_t ld(rsrc_t r, uint32_t i) { return ld32(r, i << 2); }
    __device__ static void st(rsrc_t r, uint32_t i, uint32_t v) { st32(r, i << 2, v); }
};
template <>
struct BufIO<float> {
    __device__ static uint32_t ld(rsrc_t r, uint32_t i) { return ld32(r, i << 2); }
    __device__ static void st(rsrc_t r, uint32_t i, uint32_t v) { st32(r, i << 2, v); }
};
template <>
struct BufIO<uint8_t> {
    __device__ static uint32_t ld(rsrc_t r, uint32_t i) { return __builtin_amdgcn_raw_buffer_load_b8(r, (int)i, 0, 0); }
    __device__ static void st(rsrc_t r, uint32_t i, uint32_t v)
    {
        __builtin_amdgcn_raw_buffer_store_b8((uint8_t)v, r, (int)i, 0, 0);
    }
};
template <>
struct BufIO<uint16_t> {
    __device__ static uint32_t ld(rsrc_t r, uint32_t i)
    {
        return __builtin_amdgcn_raw_buffer_load_b16(r, (int)(i << 1), 0, 0);
    }
    __device__ static void st(rsrc_t r, uint32_t i, uint32_t v)
    {
        __builtin_amdgcn_raw_buffer_store_b16((uint16_t)v, r, (int)(i << 1), 0, 0);
    }
};
// Element index that is out of range for every descriptor built here.
constexpr uint32_t OOB_ELEM = OOB >> 2;


// Infectivity bit b of the step's input for a lane that wants it (use):
// from the LDS copy (MODE_RESIDENT), from global memory (MODE_STREAM), or
// from global memory only when the LDS summary says its group holds an
// infectious unit (MODE_SUMMARY).  Lanes that do not want it read nothing
// from global memory and get 0.  b must be a valid unit index.
// The LDS words are read for every lane and the result selected afterwards:
// with the read inside a condition, the compiler makes a branch of every
// gathered slot and waits for each read on its own.
template <int MODE>
__device__ __forceinline__ uint32_t fetch_bit(const uint32_t* __restrict__ lds, rsrc_t gbits, uint32_t b,
                                              int32_t sum_shift, bool use)
{
    if (MODE == MODE_RESIDENT) {
        const uint32_t w = lds_bit(lds, b);
        return use ? w : 0u;
    }
    bool go = use;
    if (MODE == MODE_SUMMARY) {
        const uint32_t sb = lds_bit(lds, b >> (5 + sum_shift));
        go = use & (sb != 0u);
    }
    const uint32_t w = ld32(gbits, go ? (b >> 5) << 2 : OOB);
    return (w >> (b & 31)) & 1u;
}

// Light-row edge slots loaded ahead for chunks whose rows share one light
// degree (every chunk of a regular graph): slot j of row q is col_t[base +
// j*Q + q], so these loads need only the chunk's metadata and are issued with
// the state and age loads.
constexpr int UMAX = UNIFORM_MAX_DEG;
// Edge slots per batch of the general (mixed-degree) gather.
constexpr int JB = 8;
// Edge slots past the preload depth of a uniform chunk are loaded JT at a
// time, every load of a batch issued before its first use.
constexpr int JT = 16;
// chunk_meta[c].y of a chunk whose rows do not share one light degree.
constexpr uint32_t MIXED_CHUNK = 255u;
// Chunks of 64 units each wavefront takes per pass; the hazards and draws of
// a pass are evaluated on compacted lanes.
#ifndef FS_CU
#define FS_CU 1
#endif
constexpr int CU = FS_CU;
// Issue the next pass's loads before processing the current one.
#ifndef FS_PREFETCH
#define FS_PREFETCH 1
#endif
constexpr bool PREFETCH = FS_PREFETCH != 0;

// A device-memory pointer rebuilt from its bits.  It goes through a pointer
// to the global address space, so that the accesses through it are global
// ones (a pointer made from an integer is generic, and generic accesses
// count against the LDS counter too, so that an LDS wait would also wait
// for them).
template <class T>
__device__ __forceinline__ T* as_global(unsigned long long v)
{
    return (T*)(__attribute__((address_space(1))) T*)v;
}

// A wave-uniform pointer passed through an empty asm where it is used, so
// that neither it nor the addresses formed from it are hoisted out of the
// walk (held through the walk they would be spilled to vector lanes, and
// every use would pay lane reads).
template <class T>
__device__ __forceinline__ T* opaque_uniform(T* p)
{
    const unsigned long long v = (unsigned long long)p;
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v), hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    return as_global<T>(((unsigned long long)hi << 32) | lo);
}

// A wave-uniform offset held in a vector register: every use of it is
// per-lane address arithmetic, and in a scalar register it would be one more
// value held through the walk (spilled to vector lanes and read back with lane
// reads in every pass).
template <class T>
__device__ __forceinline__ T in_vgpr(T x)
{
    asm volatile("" : "+v"(x));
    return x;
}

template <class T>
__device__ __forceinline__ T* in_vgpr(T* p)
{
    unsigned long long v = (unsigned long long)p;
    asm volatile("" : "+v"(v));
    return as_global<T>(v);
}

// The rate of an E (isI false) or I unit of age xa: the hazard of its law.
// With both laws of one kind the E/I choice only selects parameters, so one
// hazard evaluation serves a wavefront holding both.  hz points to device
// memory (StepArgs::hz_dev): read where a hazard is evaluated, the laws'
// parameters and the tests on their kinds are not held through the walk.
__device__ __forceinline__ float unit_hazard(const HazardDev* hz, int32_t same_kind, float xa, bool isI)
{
    hz = opaque_uniform(hz);
    if (same_kind) {
        HazardDev hd = hz[0];
        if (isI) hd = hz[1];
        hd.kind = hz[0].kind;
        return fsd::hazard(hd, xa);
    }
    return isI ? fsd::hazard(hz[1], xa) : fsd::hazard(hz[0], xa);
}

// Packed columns of uniform layouts with one replica: PB bits per column
// (enough for every node id of the graph), a row's columns concatenated into
// one bit stream, column j at bits [PB j, PB j + PB) of the row's words.
// Words of a row holding d columns (PB = 0: plain 32-bit columns).
template <int PB>
__host__ __device__ constexpr uint32_t words_per_row(uint32_t d)
{
    return PB ? (d * (uint32_t)PB + 31u) >> 5 : d;
}

// The first D columns of a row from its loaded words (a copy for PB = 0).
// Every offset and shift is a compile-time constant: a field within one
// word is one bit-field extract, one that spans two words a funnel shift
// and a mask.
template <int PB, int D>
__device__ __forceinline__ void unpack_columns(const int32_t (&w)[UMAX], uint32_t (&c)[D])
{
#pragma unroll
    for (int j = 0; j < D; ++j) {
        if (PB == 0) {
            c[j] = (uint32_t)w[j];
        } else {
            const int o = PB * j, lo = o >> 5, sh = o & 31;
            if (sh + PB <= 32)
                c[j] = __builtin_amdgcn_ubfe((uint32_t)w[lo], (uint32_t)sh, (uint32_t)PB);
            else
                c[j] = __builtin_amdgcn_alignbit((uint32_t)w[lo + 1], (uint32_t)w[lo], (uint32_t)sh) &
                       ((1u << PB) - 1u);
        }
    }
}

// The loads of one pass, as issued: chunk numbers and metadata are
// wave-uniform; xr, agw and dgr are the raw state, age and degree words
// (0 for lanes past the chunk's valid units), used only after the pass's
// wait.
template <class age_t>
struct Pass {
    uint32_t chk[CU], base[CU], ud[CU], nvalid[CU];
    bool live[CU];
    uint32_t xr[CU], agw[CU], dgr[CU], org[CU];
    int32_t c[CU][UMAX];
    float tab[CU][3]; // hazard-table entry of the lane's age (issue_table)
    uint32_t ht[CU], hd[CU]; // pushed pressure of a binned unit: count of the last step, delta
};

// The first D columns of chunk u of a pass: unpacked from its words, or
// (PB = 0, or a chunk of a mixed layout deeper than UMAX, which keeps 32-bit
// columns) copied.
template <int PB, int UD, int D = (UD != 0 ? UD : UMAX), class age_t>
__device__ __forceinline__ void pass_columns(const Pass<age_t>& P, int u, uint32_t (&col)[D])
{
    if (PB && UD == 0 && P.ud[u] > (uint32_t)UMAX)
        unpack_columns<0, D>(P.c[u], col);
    else
        unpack_columns<PB, D>(P.c[u], col);
}

// Pushed pressure of binned rows (StepArgs::hub_T) within one step launch:
// the slots of this step (offsets in units of the hub arrays), and the
// wavefront's queue of units that enter or leave I, whose pushes are made
// after its walk (so no dependent load waits inside a pass, where it would
// also wait for the next pass's prefetched loads).
constexpr uint32_t PUSHQ = 128;
struct HubCtx {
    bool on;
    rsrc_t tr; // hub_T and hub_D, which follows it (2 * hub_units on)
    uint32_t t_prev, t_cur, d_cur, d_clr, d_next; // element offsets of the slots from hub_T
    uint32_t* q;   // LDS queue: unit | (0x80000000 when leaving I), PUSHQ entries
    uint32_t* pb;  // LDS: 64 list starts (flush)
    uint32_t* px;  // LDS: 64 exclusive prefix sums (flush)
    uint32_t n;    // queued entries (wave-uniform)
    uint32_t base; // the first binned unit, hub_base << lgR (in a vector register)
};

// The pushes of the queued units: +1 (entering I) or -1 (leaving I) into the
// next step's delta of every binned row listing the unit's node, once per
// occurrence.  The lists of up to 64 queued units are flattened over the
// wavefront: lane l takes list entry f = f0 + l, finds its unit by a binary
// search of the lists' prefix sums, and adds to the row it names.
__device__ __forceinline__ void flush_pushes(const StepArgs& a, HubCtx& H, uint32_t lane)
{
    // (the queue was written by other lanes of this wavefront)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int32_t* __restrict__ optr = opaque_uniform(a.hub_out_ptr);
    const int32_t* __restrict__ oidx = opaque_uniform(a.hub_out_idx);
    uint32_t* hub = opaque_uniform(a.hub_T);
    for (uint32_t i0 = 0; i0 < H.n; i0 += 64) {
        const uint32_t m = min(64u, H.n - i0);
        const bool has = lane < m;
        const uint32_t e = has ? H.q[i0 + lane] : 0u;
        const uint32_t node = (e & 0x7FFFFFFFu) >> a.lgR;
        const uint32_t b = has ? (uint32_t)optr[node] : 0u;
        const uint32_t len0 = has ? (uint32_t)optr[node + 1] - b : 0u;
        // a list of more than 64 entries (a hub's own, which can run to
        // thousands) goes by itself below; the others are flattened over the
        // wavefront
        const bool lng = len0 > 64u;
        const uint32_t len = lng ? 0u : len0;
        // inclusive prefix sum of the list lengths over the wavefront
        uint32_t inc = len;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t v = __shfl_up(inc, off, 64);
            if (lane >= (uint32_t)off) inc += v;
        }
        const uint32_t total = __shfl(inc, 63, 64);
        H.px[lane] = has ? inc - len : total;
        H.pb[lane] = b;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (uint32_t f0 = 0; f0 < total; f0 += 64) {
            const uint32_t f = f0 + lane;
            if (f < total) {
                // the last list whose prefix is <= f (lists of length 0 share
                // their prefix with the next one, which is then taken)
                uint32_t lo = 0, hi = 64;
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (H.px[mid] <= f) lo = mid;
                    else hi = mid;
                }
                const uint32_t eo = H.q[i0 + lo];
                const uint32_t row = (uint32_t)oidx[H.pb[lo] + (f - H.px[lo])];
                const uint32_t rep = (eo & 0x7FFFFFFFu) & ((1u << a.lgR) - 1u);
                __hip_atomic_fetch_add(hub + H.d_next + (row << a.lgR) + rep,
                                       (eo & 0x80000000u) ? 0xFFFFFFFFu : 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        // the long lists, one at a time: rounds of LU x 64 entries whose
        // (coalesced) list loads are all issued before their pushes
        constexpr uint32_t LU = 8;
        for (unsigned long long lm = __ballot(lng); lm != 0ull; lm &= lm - 1ull) {
            const int l = __builtin_ctzll(lm);
            const uint32_t lb = (uint32_t)__shfl((int)b, l, 64), ll = (uint32_t)__shfl((int)len0, l, 64);
            const uint32_t le = (uint32_t)__shfl((int)e, l, 64);
            const uint32_t slot = H.d_next + ((le & 0x7FFFFFFFu) & ((1u << a.lgR) - 1u));
            const uint32_t v = (le & 0x80000000u) ? 0xFFFFFFFFu : 1u;
            const rsrc_t lr = make_rsrc(oidx + lb, ll * 4u);
            for (uint32_t o = 0; o < ll; o += 64u * LU) {
                uint32_t row[LU];
#pragma unroll
                for (uint32_t k = 0; k < LU; ++k) row[k] = ld32(lr, (o + k * 64u + lane) << 2); // (past the list: 0)
#pragma unroll
                for (uint32_t k = 0; k < LU; ++k)
                    if (o + k * 64u + lane < ll)
                        __hip_atomic_fetch_add(hub + slot + (row[k] << a.lgR), v, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    H.n = 0;
}

// The hazard table (StepArgs::htab) as the kernels of mixed layouts read it:
// its address, scale and length held in vector registers (their walks hold
// more wave-uniform values than the scalar registers take), and no table as
// length 0.
struct TabRef {
    const float4* p;
    float inv, len;
};

// Hazard-table loads of a pass's E/I lanes (StepArgs::htab), issued once its
// state and age have arrived and before the next pass's loads, so that
// waiting for them never waits for a later pass.  Lanes without an entry
// read nothing: their age field holds 0 (uniform layouts) or NaN (mixed
// layouts, where it also stands for a missing table).
template <bool UNIFORM, class age_t>
__device__ __forceinline__ void issue_table(const StepArgs& a, const TabRef& tv, Pass<age_t>& P, uint32_t lane)
{
    const rsrc_t tr = make_rsrc(a.htab, a.htab ? a.htab_len * 16u : 0u);
#pragma unroll
    for (int u = 0; u < CU; ++u) {
        const int x = lane < P.nvalid[u] ? (int)P.xr[u] : ST_R;
        const float af = age_units(age_from_raw<age_t>(P.agw[u]));
        if (UNIFORM) {
            const float mf = rintf(af * a.htab_inv);
            const bool want = (x == ST_E || x == ST_I) && mf < (float)a.htab_len;
            const auto t = __builtin_amdgcn_raw_buffer_load_b128(tr, want ? (int)((uint32_t)mf << 4) : (int)OOB, 0, 0);
            P.tab[u][0] = __uint_as_float(t[0]);
            P.tab[u][1] = __uint_as_float(t[1]);
            P.tab[u][2] = __uint_as_float(t[2]);
        } else {
            const float mf = rintf(af * tv.inv);
            const bool want = (x == ST_E || x == ST_I) && mf < tv.len;
            float4 t = make_float4(__builtin_nanf(""), 0.0f, 0.0f, 0.0f);
            if (want) t = tv.p[(uint32_t)mf];
            P.tab[u][0] = t.x;
            P.tab[u][1] = t.y;
            P.tab[u][2] = t.z;
        }
    }
    // (keep the scheduler from moving the next pass's loads above these)
    __builtin_amdgcn_sched_barrier(0);
}

// Lookahead of the pass issues: the active-list entry (compaction) and the
// chunk metadata (mixed layouts) the next issue uses, loaded by this one.
struct Ahead {
    uint32_t chunk[CU];
    uint32_t mx[CU], my[CU];
    const uint2* meta; // StepArgs::chunk_meta, held in vector registers
};

// Issues every load of a pass that does not depend on the state: chunk
// metadata, state, age and light degree, and the edge
// slots of uniform chunks (whose rows are all present).  Each array is read
// through a descriptor covering only this chunk's valid entries, so no lane
// branches and a pass past the last chunk reads nothing.  `first` is a
// position in the walk of `walk` chunks: the chunk itself, or with
// compaction (EXTRA kernels with an active list) the list entry at that
// position, which the issue of the previous pass (or the walk's start)
// loaded into ah.chunk[u]; this issue loads the entry one stride further.  That
// load is a vector load (every lane reads the same word) issued before the
// pass's other loads: a scalar load would be waited for by the pass's first
// LDS wait (scalar and LDS results share one counter), a vector load only by
// the next issue, behind loads that are older anyway.  The metadata of a
// mixed layout's chunk comes the same way (without compaction): loaded in
// this pass's issue it would hold the issue up, the column loads depending
// on it, until every older load (the pass being processed) had arrived.
template <int STORAGE, int UD, bool EXTRA, int PB, class age_t>
__device__ __forceinline__ void issue_pass(const StepArgs& a, uint32_t first, uint32_t nwaves, uint32_t stride,
                                           uint32_t nchunks, uint32_t walk, uint32_t total, uint32_t lane,
                                           Pass<age_t>& P, Ahead& ah, const HubCtx& H)
{
    constexpr bool UNIFORM = UD != 0;
    constexpr int DEPTH = UNIFORM ? UD : UMAX;
    using state_t = typename Store<STORAGE>::state_t;
    const uint32_t rows = 64u >> a.lgR;
    const uint32_t q = lane >> a.lgR;
#pragma unroll
    for (int u = 0; u < CU; ++u) {
        const uint32_t pos = __builtin_amdgcn_readfirstlane(first + (uint32_t)u * nwaves);
        P.live[u] = pos < walk;
        uint32_t c = P.live[u] ? pos : nchunks - 1; // (a pass past the walk reads nothing)
        if (EXTRA && a.act) {
            if (P.live[u]) c = __builtin_amdgcn_readfirstlane(ah.chunk[u]);
            ah.chunk[u] = ld32(make_rsrc(a.act, (2u + walk) * 4u), (2u + pos + stride) << 2);
        }
        P.chk[u] = c;
        if (UNIFORM) {
            // (packed columns: a row holds words_per_row(udeg) words)
            P.base[u] = P.chk[u] * rows * words_per_row<PB>((uint32_t)a.udeg);
            P.ud[u] = P.live[u] ? (uint32_t)a.udeg : 0u;
        } else if (EXTRA && a.act) {
            const uint2 meta = a.chunk_meta[P.chk[u]];
            P.base[u] = meta.x;
            P.ud[u] = P.live[u] ? meta.y : 0u;
        } else {
            // (a pass past the walk takes its predecessor's clamped entry and
            // reads nothing)
            P.base[u] = __builtin_amdgcn_readfirstlane(ah.mx[u]);
            P.ud[u] = P.live[u] ? __builtin_amdgcn_readfirstlane(ah.my[u]) : 0u;
            const uint32_t nxt = min(pos + stride, nchunks - 1u);
            const uint2 m = ah.meta[nxt];
            ah.mx[u] = m.x;
            ah.my[u] = m.y;
        }
        const uint32_t u0 = P.chk[u] << 6;
        P.nvalid[u] = P.live[u] ? min(64u, total - u0) : 0u;
        const uint32_t n0 = u0 >> a.lgR;
        const uint32_t nrows = P.live[u] ? min(rows, (uint32_t)a.n - n0) : 0u;
        P.xr[u] = BufIO<state_t>::ld(make_rsrc((const state_t*)a.state + u0, P.nvalid[u] * sizeof(state_t)), lane);
        P.agw[u] = BufIO<age_t>::ld(make_rsrc((const age_t*)a.age + u0, P.nvalid[u] * sizeof(age_t)), lane);
        // (uniform layouts have no heavy rows and arithmetic metadata: the
        // degree array is not needed)
        P.dgr[u] = UNIFORM ? 0u : BufIO<uint16_t>::ld(make_rsrc(a.ldeg + n0, nrows * 2u), q);
        // graphs in a degree-sorted order (never uniform ones) key the draws
        // by the caller's node id
        P.org[u] = UNIFORM ? n0 + q : ld32(make_rsrc(a.orig_id + n0, nrows * 4u), q << 2);
        // binned rows with pushed pressure are the nodes from hub_base on:
        // their last count and this step's delta come with the pass
        if (!UNIFORM && H.on) {
            // (unit u0 + lane belongs to a binned row exactly when it is at
            // least the first binned unit)
            const bool hub = lane < P.nvalid[u] && u0 + lane >= H.base;
            const uint32_t h = hub ? u0 + lane - H.base : 0u;
            P.ht[u] = ld32(H.tr, hub ? (H.t_prev + h) << 2 : OOB);
            P.hd[u] = ld32(H.tr, hub ? (H.d_cur + h) << 2 : OOB);
        }
        // every uniform chunk preloads its first UMAX slots, or with packed
        // columns the words that hold its first DEPTH columns (slots and
        // words past its degree are out of range).  In a mixed layout, the
        // chunks deeper than UMAX keep 32-bit columns.
        const bool pre = P.ud[u] != MIXED_CHUNK;
        constexpr int LW = UNIFORM ? (int)words_per_row<PB>((uint32_t)DEPTH) : DEPTH;
        const uint32_t rw = (PB && P.ud[u] <= (uint32_t)UMAX) ? words_per_row<PB>(P.ud[u]) : P.ud[u];
        const rsrc_t cr = make_rsrc(a.col_t + P.base[u], pre ? rw * rows * 4u : 0u);
        if (UNIFORM) {
#pragma unroll
            for (int j = 0; j < LW; ++j) P.c[u][j] = (int32_t)ld32(cr, ((uint32_t)j * rows + q) << 2);
#pragma unroll
            for (int j = LW; j < DEPTH; ++j) P.c[u][j] = 0;
        } else {
            // (mixed layouts: the loads in groups of four, as far as the
            // chunk's preloaded words reach; a wave-uniform choice)
            const uint32_t nw = pre ? min(rw, (uint32_t)UMAX) : 0u;
#pragma unroll
            for (int j = 0; j < 4; ++j) P.c[u][j] = (int32_t)ld32(cr, ((uint32_t)j * rows + q) << 2);
#pragma unroll
            for (int g = 4; g < UMAX; g += 4) {
                if (nw > (uint32_t)g) {
#pragma unroll
                    for (int j = g; j < g + 4; ++j) P.c[u][j] = (int32_t)ld32(cr, ((uint32_t)j * rows + q) << 2);
                } else {
#pragma unroll
                    for (int j = g; j < g + 4; ++j) P.c[u][j] = 0;
                }
            }
        }
    }
}

// Shedding values of the preloaded edge slots of a pass (resident variant):
// the LDS bit of every slot a susceptible light row uses, then, for set bits,
// the source's s(tau).  Issued before the next pass's loads, so the wait for
// these values leaves the next pass's loads in flight (loads complete in
// order).  Slots not used read nothing and hold 0.
struct ShedPre {
    float v[CU][UMAX];
};

template <int STORAGE, int UD, int PB, class age_t>
__device__ __forceinline__ void shed_pre(const StepArgs& a, const Pass<age_t>& P, uint32_t lane,
                                         const uint32_t* __restrict__ lds, rsrc_t shedr, ShedPre& S)
{
    constexpr bool UNIFORM = UD != 0;
    constexpr int DEPTH = UNIFORM ? UD : UMAX;
    const int32_t lgR = a.lgR;
    const uint32_t rep = lane & ((1u << lgR) - 1u);
#pragma unroll
    for (int u = 0; u < CU; ++u) {
        const bool valid = lane < P.nvalid[u];
        const int x = valid ? (int)P.xr[u] : ST_R;
        const uint32_t dg = valid ? P.dgr[u] : 0u;
        const bool want = x == ST_S && (UNIFORM || dg != HEAVY_ROW);
        const bool pre = UNIFORM || P.ud[u] != MIXED_CHUNK;
        // (every LDS word read first, then the value loads of the set bits)
        uint32_t src[DEPTH], wv[DEPTH], col[DEPTH];
        pass_columns<PB, UD>(P, u, col);
#pragma unroll
        for (int j = 0; j < DEPTH; ++j) {
            src[j] = (col[j] << lgR) + rep;
            wv[j] = lds[src[j] >> 5];
        }
#pragma unroll
        for (int j = 0; j < DEPTH; ++j) {
            const bool use = pre && (uint32_t)j < P.ud[u] && want;
            const uint32_t b = use ? __builtin_amdgcn_ubfe(wv[j], src[j] & 31u, 1) : 0u;
            S.v[u][j] = shed_at<STORAGE>(shedr, src[j], b != 0u);
        }
    }
}

// The preloaded slots of a light row (the first D of a uniform chunk's
// columns, col[]): their count of infectious sources (unit weights) or
// weighted sum.  In a mixed layout D is the smallest bucket that holds the
// chunk's degree, and slots past the degree read nothing.
template <int MODE, bool WEIGHTED, bool UNIFORM, int D, class age_t>
__device__ __forceinline__ void preloaded_slots(const StepArgs& a, const Pass<age_t>& P, int u, bool want,
                                                const uint32_t (&col)[D], const uint32_t* __restrict__ lds,
                                                rsrc_t gbits, rsrc_t wr, uint32_t rows, uint32_t q, uint32_t rep,
                                                int32_t lgR, uint32_t& pi, float& pw)
{
    // every slot's LDS word is read before any is used (one wait for
    // all); the global bitmap words, in the variants that need them,
    // are loaded only where the slot is used (and, with the summary,
    // its group holds an infectious unit), and not at all when no
    // lane of the wavefront needs one: a load consumed here would
    // also wait for the next pass's prefetched loads
    uint32_t src[D], bit[D];
    bool use[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        use[j] = (uint32_t)j < P.ud[u] && want;
        src[j] = (col[j] << lgR) + rep;
    }
    if (MODE == MODE_RESIDENT && !WEIGHTED) {
        // unit weights: the count of set bits, masked once (slots past
        // a mixed chunk's degree read nothing and hold 0; the bit
        // extract uses the low five bits of its offset)
        uint32_t wv[D];
#pragma unroll
        for (int j = 0; j < D; ++j) wv[j] = (UNIFORM || (uint32_t)j < P.ud[u]) ? lds[src[j] >> 5] : 0u;
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) sum += __builtin_amdgcn_ubfe(wv[j], src[j], 1);
        if (UNIFORM) {
            // the slots of a uniform chunk past its degree loaded no
            // column (out of range: 0), so they counted unit `rep`
            // (node 0 of this replica): take those counts back
            sum -= ((uint32_t)D - P.ud[u]) * __builtin_amdgcn_ubfe(lds[rep >> 5], rep, 1);
        }
#pragma unroll
        for (int j = 0; j < D; ++j) bit[j] = 0u;
        pi += want ? sum : 0u;
    } else if (MODE == MODE_RESIDENT) {
        uint32_t wv[D];
        // (a mixed layout's chunk reads only its degree's slots: a
        // wave-uniform test)
#pragma unroll
        for (int j = 0; j < D; ++j) wv[j] = (UNIFORM || (uint32_t)j < P.ud[u]) ? lds[src[j] >> 5] : 0u;
#pragma unroll
        for (int j = 0; j < D; ++j) bit[j] = __builtin_amdgcn_ubfe(wv[j], src[j] & 31u, 1) & (uint32_t)use[j];
    } else {
        bool go[D];
        if (MODE == MODE_SUMMARY) {
            uint32_t sw[D];
#pragma unroll
            for (int j = 0; j < D; ++j)
                sw[j] = (UNIFORM || (uint32_t)j < P.ud[u]) ? lds[src[j] >> (a.sum_shift + 10)] : 0u;
#pragma unroll
            for (int j = 0; j < D; ++j)
                go[j] = use[j] & (__builtin_amdgcn_ubfe(sw[j], src[j] >> (a.sum_shift + 5), 1) != 0u);
        } else {
#pragma unroll
            for (int j = 0; j < D; ++j) go[j] = use[j];
        }
        bool anyg = false;
#pragma unroll
        for (int j = 0; j < D; ++j) anyg = anyg | go[j];
#pragma unroll
        for (int j = 0; j < D; ++j) bit[j] = 0u;
        if (__ballot(anyg) != 0ull) {
            uint32_t w[D];
#pragma unroll
            for (int j = 0; j < D; ++j) w[j] = ld32(gbits, go[j] ? (src[j] >> 5) << 2 : OOB);
            // (slots not loaded read 0)
#pragma unroll
            for (int j = 0; j < D; ++j) bit[j] = __builtin_amdgcn_ubfe(w[j], src[j], 1);
        }
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
        if (WEIGHTED) {
            const float w = __uint_as_float(ld32(wr, use[j] ? ((uint32_t)j * rows + q) << 2 : OOB));
            pw = __builtin_fmaf(w, (float)bit[j], pw);
        } else {
            pi += bit[j];
        }
    }
}

// Pressure of one chunk's light row for this lane (Eq. (influence) without
// beta).  Uniform chunks use the preloaded slots (and load any further ones
// in batches of JT, each batch's loads issued together); mixed chunks find a row's
// position in run j as its rank among the rows with more than j edges (ballot
// prefix count), JB slots at a time.  With age-dependent shedding (SHED) a
// source whose bit is set contributes its s(tau) from `shedr`; the value load
// of every other slot is out of range and reads nothing.
template <int STORAGE, int MODE, bool WEIGHTED, int UD, bool SHED, int PB, class age_t>
__device__ __forceinline__ float pressure_row(const StepArgs& a, const Pass<age_t>& P, int u, bool want,
                                              uint32_t dg, const uint32_t* __restrict__ lds, rsrc_t gbits,
                                              rsrc_t shedr, const ShedPre& S, uint32_t lane)
{
    constexpr bool UNIFORM = UD != 0;
    constexpr int DEPTH = UNIFORM ? UD : UMAX;
    // shedding values of preloaded slots come from shed_pre (resident variant)
    constexpr bool SPLIT = SHED && MODE == MODE_RESIDENT;
    const int32_t lgR = a.lgR;
    const uint32_t R = 1u << lgR;
    const uint32_t rep = lane & (R - 1);
    const uint32_t d = dg == HEAVY_ROW ? 0u : dg;
    uint32_t pi = 0;
    float pw = 0.0f;
    if (UNIFORM || P.ud[u] != MIXED_CHUNK) {
        // uniform chunk: slots past the degree hold 0 (a valid node) and are
        // not used; weights come through the same per-chunk range
        const uint32_t rows = 64u >> lgR;
        const uint32_t q = lane >> lgR;
        const rsrc_t wr = make_rsrc(WEIGHTED ? (const void*)(a.w_t + P.base[u]) : (const void*)a.w_t,
                                    WEIGHTED ? P.ud[u] * rows * 4u : 0u);
        if (!SHED) {
            if (UNIFORM) {
                uint32_t col[DEPTH];
                pass_columns<PB, UD, DEPTH>(P, u, col);
                preloaded_slots<MODE, WEIGHTED, UNIFORM, DEPTH>(a, P, u, want, col, lds, gbits, wr, rows, q, rep, lgR,
                                                                pi, pw);
            } else if (P.ud[u] <= 6u) {
                // (mixed layouts: the preloaded slots a chunk of this degree
                // uses, a wave-uniform choice)
                uint32_t col[6];
                pass_columns<PB, UD, 6>(P, u, col);
                preloaded_slots<MODE, WEIGHTED, UNIFORM, 6>(a, P, u, want, col, lds, gbits, wr, rows, q, rep, lgR, pi,
                                                            pw);
            } else if (P.ud[u] <= 9u) {
                uint32_t col[9];
                pass_columns<PB, UD, 9>(P, u, col);
                preloaded_slots<MODE, WEIGHTED, UNIFORM, 9>(a, P, u, want, col, lds, gbits, wr, rows, q, rep, lgR, pi,
                                                            pw);
            } else {
                uint32_t col[DEPTH];
                pass_columns<PB, UD, DEPTH>(P, u, col);
                preloaded_slots<MODE, WEIGHTED, UNIFORM, DEPTH>(a, P, u, want, col, lds, gbits, wr, rows, q, rep, lgR,
                                                                pi, pw);
            }
        } else {
            uint32_t col[DEPTH];
            pass_columns<PB, UD, DEPTH>(P, u, col);
#pragma unroll
            for (int j = 0; j < DEPTH; ++j) {
                const bool use = (uint32_t)j < P.ud[u] && want;
                float v;
                if (SPLIT) {
                    v = S.v[u][j];
                } else {
                    const uint32_t src = (col[j] << lgR) + rep;
                    const uint32_t b = fetch_bit<MODE>(lds, gbits, src, a.sum_shift, use);
                    v = shed_at<STORAGE>(shedr, src, b != 0u);
                }
                if (WEIGHTED) {
                    const float w = __uint_as_float(ld32(wr, use ? ((uint32_t)j * rows + q) << 2 : OOB));
                    pw = __builtin_fmaf(w, v, pw);
                } else {
                    pw += v;
                }
            }
        }
        // a uniform chunk deeper than the preload: its remaining slots, JT
        // per batch (same layout; slots past the degree are out of range)
        if (!UNIFORM && P.ud[u] > (uint32_t)UMAX) {
            const rsrc_t cr = make_rsrc(a.col_t + P.base[u], P.ud[u] * rows * 4u);
            for (uint32_t j0 = UMAX; j0 < P.ud[u]; j0 += JT) {
                int32_t c[JT];
                float wv[JT];
#pragma unroll
                for (int jj = 0; jj < JT; ++jj) {
                    const uint32_t off = want ? ((j0 + jj) * rows + q) << 2 : OOB;
                    c[jj] = (int32_t)ld32(cr, off);
                    wv[jj] = WEIGHTED ? __uint_as_float(ld32(wr, off)) : 0.0f;
                }
#pragma unroll
                for (int jj = 0; jj < JT; ++jj) {
                    const bool use = want && j0 + jj < P.ud[u];
                    const uint32_t src = ((uint32_t)c[jj] << lgR) + rep;
                    const uint32_t b = fetch_bit<MODE>(lds, gbits, src, a.sum_shift, use);
                    const float v = SHED ? shed_at<STORAGE>(shedr, src, b != 0u) : (float)b;
                    if (WEIGHTED) pw = __builtin_fmaf(wv[jj], v, pw);
                    else if (SHED) pw += v;
                    else pi += b;
                }
            }
        }
    } else {
        const unsigned long long below = (1ull << (lane & ~(R - 1))) - 1ull;
        uint32_t off = P.base[u];
        for (uint32_t j0 = 0;; j0 += JB) {
            if (__ballot(rep == 0 && d > j0) == 0ull) break;
            int32_t c[JB];
            float wv[JB];
#pragma unroll
            for (int jj = 0; jj < JB; ++jj) {
                const unsigned long long m = __ballot(rep == 0 && d > j0 + jj);
                c[jj] = 0;
                wv[jj] = 0.0f;
                if (want && d > j0 + jj) {
                    const uint32_t idx = off + (uint32_t)__popcll(m & below);
                    c[jj] = a.col_t[idx];
                    if (WEIGHTED) wv[jj] = a.w_t[idx];
                }
                off += (uint32_t)__popcll(m);
            }
#pragma unroll
            for (int jj = 0; jj < JB; ++jj) {
                if (want && d > j0 + jj) {
                    const uint32_t src = ((uint32_t)c[jj] << lgR) + rep;
                    const uint32_t b = fetch_bit<MODE>(lds, gbits, src, a.sum_shift, true);
                    const float v = SHED ? shed_at<STORAGE>(shedr, src, b != 0u) : (float)b;
                    if (WEIGHTED) pw = __builtin_fmaf(wv[jj], v, pw);
                    else if (SHED) pw += v;
                    else pi += b;
                }
            }
        }
    }
    return (WEIGHTED || SHED) ? pw : (float)pi;
}

// Pressure of a degree-binned row: its segment partials in segment order
// (float partials with weights or shedding values, else integer counts).
template <bool FLOATP>
__device__ __forceinline__ float pressure_heavy(const StepArgs& a, uint32_t node, uint32_t rep)
{
    const size_t R = (size_t)1 << a.lgR;
    // (the pointers and the segment length are read here, not held through
    // the walk)
    const int32_t* rp = opaque_uniform(a.row_ptr);
    const int32_t* hf = opaque_uniform(a.heavy_first);
    const void* spp = opaque_uniform(a.seg_part);
    int32_t se = __builtin_amdgcn_readfirstlane(a.seg_edges);
    asm volatile("" : "+s"(se));
    const int32_t dg = rp[node + 1] - rp[node];
    const int32_t first = hf[node];
    const int32_t nseg = (dg + se - 1) / se;
    if (FLOATP) {
        const float* sp = (const float*)spp;
        float p = 0.0f;
        for (int32_t j = 0; j < nseg; ++j) p += sp[(size_t)(first + j) * R + rep];
        return p;
    }
    const uint32_t* sp = (const uint32_t*)spp;
    uint32_t p = 0;
    for (int32_t j = 0; j < nseg; ++j) p += sp[(size_t)(first + j) * R + rep];
    return (float)p;
}

// Evaluates f on the flagged items of CU chunks with the items packed into
// consecutive lanes (64 per round), so a computation most lanes skip costs one
// wavefront pass per 64 items instead of one per chunk.  xch is this
// wavefront's 64-entry LDS exchange row; f maps a payload word to a result
// word.  Only flagged items receive a result.
template <int CU, class F>
__device__ __forceinline__ void compact_apply(uint32_t* xch, uint32_t lane, const bool* flag,
                                              const uint32_t* payload, uint32_t* result, F f)
{
    if constexpr (CU == 1) {
        // one chunk per pass holds at most 64 items: packing would still
        // evaluate f once, so evaluate it on the flagged lanes in place
        (void)xch;
        (void)lane;
        if (flag[0]) result[0] = f(payload[0]);
        return;
    }
    unsigned long long m[CU];
    uint32_t pre[CU + 1];
    pre[0] = 0;
#pragma unroll
    for (int u = 0; u < CU; ++u) {
        m[u] = __ballot(flag[u]);
        pre[u + 1] = pre[u] + (uint32_t)__popcll(m[u]);
    }
    const uint32_t total = pre[CU];
    const unsigned long long lt = (1ull << lane) - 1ull;
    uint32_t slot[CU];
#pragma unroll
    for (int u = 0; u < CU; ++u) slot[u] = pre[u] + (uint32_t)__popcll(m[u] & lt);
    for (uint32_t r0 = 0; r0 < total; r0 += 64) {
#pragma unroll
        for (int u = 0; u < CU; ++u)
            if (flag[u] && slot[u] >= r0 && slot[u] < r0 + 64) xch[slot[u] - r0] = payload[u];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (r0 + lane < total) xch[lane] = f(xch[lane]);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int u = 0; u < CU; ++u)
            if (flag[u] && slot[u] >= r0 && slot[u] < r0 + 64) result[u] = xch[slot[u] - r0];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Everything of one pass after its loads were issued: rates (gather,
// hazards), draws, stores, next-infectivity words (and, with SHED, the
// s(tau') values of the units infectious after the step), counts, and the
// chunk's live flag for compaction.
template <int STORAGE, bool WEIGHTED, int MODE, int UD, bool SHED, bool EXTRA, int PB, class age_t>
__device__ __forceinline__ void process_pass(const StepArgs& a, const Pass<age_t>& P, uint32_t lane,
                                             const uint32_t* __restrict__ s_bits, rsrc_t gbits, rsrc_t shedr,
                                             void* __restrict__ shed_out, const ShedPre& sv, const ShedDev& sdv,
                                             uint32_t* xch, unsigned long long k,
                                             unsigned long long* __restrict__ bits_out, uint32_t* s_cnt,
                                             uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, float dt,
                                             float& lmax, HubCtx& H)
{
    constexpr bool UNIFORM = UD != 0;
    using state_t = typename Store<STORAGE>::state_t;
    const uint32_t R = 1u << a.lgR;

    // the pass's loaded words; lanes past the chunk's valid units act as R
    bool valid[CU];
    int x[CU];
    age_t ag[CU];
    uint32_t dg[CU], unit[CU];
#pragma unroll
    for (int u = 0; u < CU; ++u) {
        valid[u] = lane < P.nvalid[u];
        unit[u] = (P.chk[u] << 6) + lane;
        x[u] = valid[u] ? (int)P.xr[u] : ST_R;
        ag[u] = valid[u] ? age_from_raw<age_t>(P.agw[u]) : (age_t)0;
        dg[u] = valid[u] ? P.dgr[u] : 0u;
    }

    // 1.-2. rate: beta * pressure for S; hazard at the start-of-step age for E/I; 0 for R
    float lam[CU];
#pragma unroll
    for (int u = 0; u < CU; ++u) {
        lam[u] = 0.0f;
        const bool heavy = !UNIFORM && dg[u] == HEAVY_ROW;
        const bool want = x[u] == ST_S && !heavy;
        const float p =
            pressure_row<STORAGE, MODE, WEIGHTED, UD, SHED, PB>(a, P, u, want, dg[u], s_bits, gbits, shedr, sv, lane);
        if (want) lam[u] = a.beta * p;
        if (!UNIFORM && !WEIGHTED && !SHED && H.on) {
            // pushed pressure: every binned unit, whatever its state, carries
            // its count into this step's slot and clears the delta slot that
            // the next step's pushes do not use
            if (__ballot(heavy) != 0ull) {
                const uint32_t h = heavy ? unit[u] - H.base : 0u;
                const uint32_t pp = P.ht[u] + P.hd[u];
                st32(H.tr, heavy ? (H.t_cur + h) << 2 : OOB, pp);
                st32(H.tr, heavy ? (H.d_clr + h) << 2 : OOB, 0u);
                if (heavy && x[u] == ST_S) lam[u] = a.beta * (float)pp;
            }
        } else if (!UNIFORM && heavy && x[u] == ST_S) {
            lam[u] = a.beta * pressure_heavy<WEIGHTED || SHED>(a, unit[u] >> a.lgR, unit[u] & (R - 1));
        }
    }

    // hazards of the E/I units of the pass, on compacted lanes; the payload
    // is the age bit pattern with bit 31 marking the I -> R law (ages are
    // non-negative, so bit 31 is free)
    {
        bool need[CU];
        uint32_t pay[CU], res[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            need[u] = x[u] == ST_E || x[u] == ST_I;
            pay[u] = age_bits(ag[u]) | (x[u] == ST_I ? 0x80000000u : 0u);
            res[u] = 0;
        }
        // ages the table holds take their hazard from it
        bool hit[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            hit[u] = (!UNIFORM || a.htab != nullptr) && need[u] && P.tab[u][0] == age_units(ag[u]);
            if (hit[u]) lam[u] = x[u] == ST_I ? P.tab[u][2] : P.tab[u][1];
            need[u] = need[u] && !hit[u];
        }
        compact_apply<CU>(xch, lane, need, pay, res, [&](uint32_t w) {
            return __float_as_uint(
                unit_hazard(a.hz_dev, a.same_kind, age_from_bits<age_t>(w & 0x7FFFFFFFu), (w & 0x80000000u) != 0u));
        });
#pragma unroll
        for (int u = 0; u < CU; ++u)
            if (need[u]) lam[u] = __uint_as_float(res[u]);
    }

    // 3.-4. Bernoulli tau-leap: fire when u < 1 - exp(-lambda dt); no draw at
    // lambda = 0.  The Philox draws of the pass run on compacted lanes.
    bool fire[CU];
    {
        bool need[CU];
        uint32_t pay[CU], res[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            need[u] = lam[u] > 0.0f;
            pay[u] = (P.org[u] << a.lgR) | (lane & (R - 1)); // the caller's node id and the replica
            res[u] = 0;
        }
        const uint32_t kk = (uint32_t)k;
        compact_apply<CU>(xch, lane, need, pay, res, [&](uint32_t un) {
            // the key and step pass through an empty asm here, so the round
            // keys and the key-step terms are formed by scalar adds at each
            // draw instead of being hoisted out of the walk: held for the
            // whole walk they would take 20 scalar registers and be spilled
            // to vector lanes, each use a lane read
            // (all three are wave-uniform)
            uint32_t k0 = __builtin_amdgcn_readfirstlane(a.key0), k1 = __builtin_amdgcn_readfirstlane(a.key1),
                     ks = __builtin_amdgcn_readfirstlane(kk);
            asm volatile("" : "+s"(k0), "+s"(k1), "+s"(ks));
            return fsd::philox4x32_10(make_uint4(un >> a.lgR, ks, un & (R - 1), 0u), k0, k1).x >> 8;
        });
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            fire[u] = false;
            if (need[u]) {
                const float uu = (float)res[u] * 0x1p-24f;
                const float qq = -expm1f(-lam[u] * dt);
                fire[u] = uu < qq;
            }
        }
    }

    int xns[CU];
    age_t ans[CU];
#pragma unroll
    for (int u = 0; u < CU; ++u) {
        // 5.-6. advance state and age in place (the chunk's descriptors drop
        // the lanes past its valid units; the state only changes on a firing)
        const int xn = x[u] + (fire[u] ? 1 : 0);
        xns[u] = xn;
        ans[u] = fire[u] ? (age_t)0 : age_next(ag[u], dt);
        const uint32_t u0 = P.chk[u] << 6;
        BufIO<state_t>::st(make_rsrc((state_t*)a.state + u0, P.nvalid[u] * sizeof(state_t)),
                           fire[u] ? lane : OOB_ELEM, (uint32_t)xn);
        BufIO<age_t>::st(make_rsrc((age_t*)a.age + u0, P.nvalid[u] * sizeof(age_t)), lane, age_to_raw(ans[u]));
        lmax = fmaxf(lmax, lam[u]);
        if (!UNIFORM && !WEIGHTED && !SHED && H.on) {
            // a unit entering or leaving I is queued for its pushes into the
            // next step's deltas of the binned rows that list its node
            const bool push = fire[u] && (x[u] == ST_E || x[u] == ST_I);
            const unsigned long long pm = __ballot(push);
            if (pm != 0ull) {
                const uint32_t cnt = (uint32_t)__popcll(pm);
                if (H.n + cnt > PUSHQ) flush_pushes(a, H, lane);
                if (push)
                    H.q[H.n + (uint32_t)__popcll(pm & ((1ull << lane) - 1ull))] =
                        unit[u] | (x[u] == ST_I ? 0x80000000u : 0u);
                H.n += cnt;
            }
        }
        // the rates, when recorded (EXTRA kernels)
        if (EXTRA && a.rates) st32(make_rsrc(a.rates + u0, P.nvalid[u] * 4u), lane << 2, __float_as_uint(lam[u]));
        // 7. next-step infectivity bits (one 64-bit word per chunk, written by
        // lanes 0 and 1) and 8. counts
        const unsigned long long mI = __ballot(valid[u] && xn == ST_I);
        if (UNIFORM) {
            st32(make_rsrc(bits_out + P.chk[u], P.live[u] ? 8u : 0u), lane < 2 ? lane << 2 : OOB,
                 lane == 0 ? (uint32_t)mI : (uint32_t)(mI >> 32));
        } else if (P.live[u] && lane < 2) {
            // (mixed layouts: bits_out is held in vector registers)
            ((uint32_t*)bits_out)[2 * P.chk[u] + lane] = lane == 0 ? (uint32_t)mI : (uint32_t)(mI >> 32);
        }
        if (R == 1) {
            c0 += (uint32_t)__popcll(__ballot(valid[u] && xn == ST_S));
            c1 += (uint32_t)__popcll(__ballot(valid[u] && xn == ST_E));
            c2 += (uint32_t)__popcll(mI);
            c3 += (uint32_t)__popcll(__ballot(valid[u] && xn == ST_R));
        } else if (valid[u]) {
            atomicAdd(&s_cnt[(unit[u] & (R - 1)) * 4 + xn], 1u); // LDS
        }
        // compaction: whether the chunk held a unit that is not R at the start
        // of the step.  A chunk is dropped only after a step that began with
        // all its units in R, so both of its ping-pong bitmap words are 0
        // (it held no I unit before or after that step) and stay 0.
        if (EXTRA && a.live) {
            const bool alive = __ballot(valid[u] && x[u] != ST_R) != 0ull;
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(alive ? 1 : 0),
                                                 make_rsrc(a.live + P.chk[u], P.live[u] ? 1u : 0u),
                                                 lane == 0 ? 0 : (int)OOB, 0, 0);
        }
    }

    if (SHED) {
        // 7'. infectivity values s(tau') of the units infectious after the
        // step (Eq. (infectivity)), on compacted lanes (a separate round
        // measured faster than folding s(tau + dt) into the hazard round)
        bool need[CU];
        uint32_t pay[CU], res[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u) {
            need[u] = valid[u] && xns[u] == ST_I;
            pay[u] = age_bits(ans[u]);
            res[u] = 0;
        }
        compact_apply<CU>(xch, lane, need, pay, res, [&](uint32_t w) {
            return __float_as_uint(fsd::shed(sdv, age_from_bits<age_t>(w)));
        });
#pragma unroll
        for (int u = 0; u < CU; ++u)
            shed_put<STORAGE>(make_rsrc((char*)shed_out + (size_t)(P.chk[u] << 6) * Store<STORAGE>::shed_bytes,
                                        P.nvalid[u] * Store<STORAGE>::shed_bytes),
                              lane, need[u], __uint_as_float(res[u]));
    }
}

// One fused step.  Units are processed in chunks of 64 (one wavefront, one
// 64-bit word of the next infectivity bitmap); every wavefront walks its own
// chunks, CU per pass, with no workgroup barrier inside the walk.
//  MODE_RESIDENT: the whole start-of-step bitmap (units <= RESIDENT_BITS) is
//    copied into LDS once per workgroup (direct global-to-LDS loads, overlapped
//    with the first pass's loads) and every gather reads LDS;
//  MODE_SUMMARY: the bitmap's summary is copied into LDS the same way, and a
//    gather reads the global bitmap only where the summary bit is set (when
//    infection is sparse most neighbours fall in empty groups);
//  MODE_STREAM: gathers read the bitmap through the caches.
// The LDS variants run one workgroup of RESIDENT_TPB threads per compute unit.
template <int STORAGE, bool WEIGHTED, int MODE, int UD, bool SHED, bool EXTRA, int TPB, int PB = 0>
__device__ __forceinline__ void step_body(const StepArgs& a, uint32_t block, uint32_t nblocks)
{
    constexpr bool UNIFORM = UD != 0;
    constexpr bool USE_LDS = MODE != MODE_STREAM;
    using age_t = typename Store<STORAGE>::age_t;
    constexpr int NW = TPB / 64;
    static_assert(PB == 0 || !WEIGHTED, "packed columns: unit weights only");

    __shared__ uint32_t s_cnt[4 * 64];
    __shared__ __attribute__((aligned(16))) uint32_t s_bits[USE_LDS ? RESIDENT_BITS / 32 : 4];
    static_assert(SUMMARY_BITS <= RESIDENT_BITS, "the summary shares the LDS bitmap array");
    __shared__ uint32_t s_xch[NW][64];
    // pushed pressure of binned rows: per-wavefront push queue and flush tables
    constexpr bool HUBS = !UNIFORM && !WEIGHTED && !SHED;
    __shared__ uint32_t s_pq[HUBS ? NW : 1][HUBS ? PUSHQ : 1];
    __shared__ uint32_t s_pb[HUBS ? NW : 1][HUBS ? 64 : 1];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6); // wave-uniform, in a scalar register
    const uint32_t R = 1u << a.lgR;
    const unsigned long long k = a.ctl->step + a.step_off;
    const uint32_t* __restrict__ bits_in = (const uint32_t*)((k & 1) ? a.iota1 : a.iota0);
    unsigned long long* __restrict__ bits_out = (unsigned long long*)((k & 1) ? a.iota0 : a.iota1);
    const uint32_t total = (uint32_t)a.n << a.lgR;
    const uint32_t nchunks = (total + 63) >> 6;
    // the input bitmap: whole 512-unit tiles of 64 bytes
    const rsrc_t gbits = make_rsrc(bits_in, ((total + 511u) >> 9) << 6);
    // shedding values: read from the step's input, written to the other buffer
    const rsrc_t shedr = make_rsrc((k & 1) ? a.shed1 : a.shed0, SHED ? total * Store<STORAGE>::shed_bytes : 0u);
    void* __restrict__ shed_out = (k & 1) ? a.shed0 : a.shed1;
    // the chunks this launch walks: all, or the active list
    const uint32_t walk = (EXTRA && a.act) ? a.act[0] : nchunks;
    // this step's size: fixed, or (adaptive) from the largest rate of the
    // previous step, folded by every wave from the per-workgroup maxima
    float dt = a.dt;
    if (a.adaptive && k != a.ctl->adapt_from) {
        const float* prev = a.lam_part + (size_t)((k - 1) & 1) * nblocks;
        float m = 0.0f;
        for (uint32_t i = lane; i < nblocks; i += 64) m = fmaxf(m, prev[i]);
        for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
        dt = fminf(a.dt, a.eps / (m + a.delta));
    }
    float lmax = 0.0f;
    const uint32_t wave_id = block * NW + wave;
    const uint32_t nwaves = nblocks * NW;
    HubCtx H;
    H.on = HUBS && a.hub_T != nullptr;
    H.n = 0;
    H.q = s_pq[HUBS ? wave : 0];
    H.pb = s_pb[HUBS ? wave : 0];
    H.px = s_xch[wave];
    H.t_prev = H.t_cur = H.d_cur = H.d_clr = H.d_next = H.base = 0;
    if (H.on) {
        const uint32_t HU = a.hub_units;
        const uint32_t k2 = (uint32_t)(k & 1ull), k3 = (uint32_t)(k % 3ull);
        H.tr = make_rsrc(a.hub_T, 5u * HU * 4u);
        H.t_prev = in_vgpr((k2 ^ 1u) * HU);
        H.t_cur = in_vgpr(k2 * HU);
        H.d_cur = in_vgpr((2u + k3) * HU);
        H.d_next = in_vgpr((2u + (k3 + 1u) % 3u) * HU);
        H.d_clr = in_vgpr((2u + (k3 + 2u) % 3u) * HU);
        H.base = in_vgpr((uint32_t)a.hub_base << a.lgR);
    } else {
        H.tr = make_rsrc(nullptr, 0u);
    }

    // first pass loads, then the bitmap fill, then one wait for both
    Pass<age_t> P;
    uint32_t first = wave_id;
    const uint32_t stride = nwaves * CU;
    Ahead ahead;
    ahead.meta = UNIFORM ? a.chunk_meta : in_vgpr(a.chunk_meta);
#pragma unroll
    for (int u = 0; u < CU; ++u) {
        const uint32_t pos = first + (uint32_t)u * nwaves;
        ahead.chunk[u] = (EXTRA && a.act && pos < walk) ? a.act[2 + pos] : 0u;
        ahead.mx[u] = ahead.my[u] = 0u;
        if (!UNIFORM) {
            const uint2 m = ahead.meta[min(pos, nchunks - 1u)];
            ahead.mx[u] = m.x;
            ahead.my[u] = m.y;
        }
    }
    issue_pass<STORAGE, UD, EXTRA, PB>(a, first, nwaves, stride, nchunks, walk, total, lane, P, ahead, H);
    if (R > 1)
        for (uint32_t i = tid; i < 4 * R; i += TPB) s_cnt[i] = 0;
    if (USE_LDS) {
        // 16 bytes per lane straight into LDS: wave w fills the blocks of 64
        // uint4 it owns; lane l's block element lands at base + 16 l
        const uint32_t nbits = MODE == MODE_RESIDENT ? total : a.sum_bits;
        const uint32_t n4 = (((nbits + 31) >> 5) + 3) >> 2;
        const uint4* src = (const uint4*)(MODE == MODE_RESIDENT ? bits_in : a.summary);
        for (uint32_t b0 = wave * 64; b0 < n4; b0 += TPB) {
            if (b0 + lane < n4)
                __builtin_amdgcn_global_load_lds((const void*)(src + b0 + lane),
                                                 (__attribute__((address_space(3))) void*)((uint4*)s_bits + b0), 16, 0, 0);
        }
        __builtin_amdgcn_s_waitcnt(0);
    }
    if (R > 1 || USE_LDS) __syncthreads();
    TabRef tv{nullptr, 0.0f, 0.0f};
    if (!UNIFORM) {
        tv.p = in_vgpr(a.htab);
        tv.inv = in_vgpr(a.htab_inv);
        tv.len = in_vgpr(a.htab ? (float)a.htab_len : 0.0f);
    }
    unsigned long long* __restrict__ bo = UNIFORM ? bits_out : in_vgpr(bits_out);
    // the shedding profile (shedding kernels): read once, its parameters held
    // in vector registers for the walk (its kinds stay scalar); in scalar
    // registers they would be spilled and read back in every pass, and read
    // from memory where used, their loads would wait for the next pass's
    ShedDev sdv{};
    if (SHED) {
        sdv = *a.shed_dev;
        float* f[] = {&sdv.hz.K, &sdv.hz.c_hi, &sdv.hz.c_lo, &sdv.hz.g_hi, &sdv.hz.g_lo, &sdv.hz.x_hi,
                      &sdv.hz.x_lo, &sdv.s0, &sdv.m_hi, &sdv.m_lo, &sdv.lf_hi, &sdv.lf_lo};
#pragma unroll
        for (float* x : f) *x = in_vgpr(*x);
    }
    issue_table<UNIFORM>(a, tv, P, lane);

    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0; // per-wave counts (R == 1)

    // passes: the loads of the next pass are issued (always: a pass past the
    // end reads nothing) before the current pass is processed; two register
    // sets, unrolled by two
    Pass<age_t> P1;
    // resident variant with shedding: the pass's shedding values are loaded
    // before the next pass's loads are issued
    constexpr bool SPLIT = SHED && MODE == MODE_RESIDENT;
    ShedPre sv;
    for (;;) {
        if (first >= walk) break;
        if (SPLIT) shed_pre<STORAGE, UD, PB>(a, P, lane, s_bits, shedr, sv);
        if (PREFETCH)
            issue_pass<STORAGE, UD, EXTRA, PB>(a, first + stride, nwaves, stride, nchunks, walk, total, lane, P1,
                                                ahead, H);
        process_pass<STORAGE, WEIGHTED, MODE, UD, SHED, EXTRA, PB>(a, P, lane, s_bits, gbits, shedr, shed_out, sv,
                                                                    sdv, s_xch[wave], k, bo, s_cnt, c0, c1, c2,
                                                                    c3, dt, lmax, H);
        first += stride;
        if (first >= walk) break;
        if (!PREFETCH)
            issue_pass<STORAGE, UD, EXTRA, PB>(a, first, nwaves, stride, nchunks, walk, total, lane, P1, ahead, H);
        issue_table<UNIFORM>(a, tv, P1, lane);
        if (SPLIT) shed_pre<STORAGE, UD, PB>(a, P1, lane, s_bits, shedr, sv);
        if (PREFETCH)
            issue_pass<STORAGE, UD, EXTRA, PB>(a, first + stride, nwaves, stride, nchunks, walk, total, lane, P,
                                                ahead, H);
        process_pass<STORAGE, WEIGHTED, MODE, UD, SHED, EXTRA, PB>(a, P1, lane, s_bits, gbits, shedr, shed_out, sv,
                                                                    sdv, s_xch[wave], k, bo, s_cnt, c0, c1, c2,
                                                                    c3, dt, lmax, H);
        first += stride;
        if (!PREFETCH && first < walk)
            issue_pass<STORAGE, UD, EXTRA, PB>(a, first, nwaves, stride, nchunks, walk, total, lane, P, ahead, H);
        if (first < walk) issue_table<UNIFORM>(a, tv, P, lane);
    }

    // the queued pushes of binned rows, after the walk (no prefetched load is
    // in flight any more)
    if (H.on && H.n > 0) flush_pushes(a, H, lane);

    // one plain store of this workgroup's counts; the reduce kernel sums them
    // (workgroup 0 also counts the R units of the chunks compaction skipped)
    uint32_t* out = a.part + ((size_t)a.step_off * nblocks + block) * (4 * R);
    const uint32_t skipped = (EXTRA && a.act && block == 0) ? a.act[1] : 0u;
    if (R == 1) {
        if (lane == 0) {
            s_cnt[wave * 4 + 0] = c0;
            s_cnt[wave * 4 + 1] = c1;
            s_cnt[wave * 4 + 2] = c2;
            s_cnt[wave * 4 + 3] = c3;
        }
        __syncthreads();
        if (tid < 4) {
            uint32_t t = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) t += s_cnt[w * 4 + tid];
            out[tid] = t + (tid == ST_R ? skipped : 0u);
        }
    } else {
        __syncthreads();
        for (uint32_t i = tid; i < 4 * R; i += TPB) out[i] = s_cnt[i] + ((i & 3) == ST_R ? skipped : 0u);
    }
    if (a.adaptive) {
        // the workgroup's largest rate, for the next step's size; block 0
        // records this step's size
        __shared__ float s_lmax[NW];
        for (int off = 32; off > 0; off >>= 1) lmax = fmaxf(lmax, __shfl_xor(lmax, off, 64));
        if (lane == 0) s_lmax[wave] = lmax;
        __syncthreads();
        if (tid == 0) {
            float m = 0.0f;
#pragma unroll
            for (int w = 0; w < NW; ++w) m = fmaxf(m, s_lmax[w]);
            a.lam_part[(size_t)(k & 1) * nblocks + block] = m;
            if (block == 0) a.dt_hist[k % a.hist_len] = dt;
        }
    }
}

// EXTRA: the instantiation that records rates when StepArgs::rates is set
// and walks the active-chunk list when StepArgs::act is set; without it
// neither check is compiled in.
// UD: 0 for mixed layouts, else the preload depth of a uniform layout (the
// smallest of 8, 10, 12 that holds its degree: slots past the degree would
// cost an issued load and a gather each)
template <int STORAGE, bool WEIGHTED, int MODE, int UD, bool SHED, bool EXTRA, int TPB>
__global__ __launch_bounds__(TPB) void step_kernel(StepArgs a)
{
    step_body<STORAGE, WEIGHTED, MODE, UD, SHED, EXTRA, TPB>(a, blockIdx.x, gridDim.x);
}

// The plain step of a sim with one replica: the same body with R = 1 known
// at compile time, so replica shifts and masks, unit and node indices and
// the column offsets (slot j of lane q at j * 64 + q, a constant offset per
// slot) cost no instructions.
template <int STORAGE, bool WEIGHTED, int MODE, int UD, int TPB>
__global__ __launch_bounds__(TPB) void step_kernel_r1(StepArgs a)
{
    StepArgs b = a;
    b.lgR = 0;
    step_body<STORAGE, WEIGHTED, MODE, UD, false, false, TPB>(b, blockIdx.x, gridDim.x);
}

// The same with packed columns of PB bits (unit weights only), with
// constant or (SHED) age-dependent shedding, and (EXTRA) the rate recording
// and compaction checks.
template <int STORAGE, int MODE, int UD, int PB, bool SHED, bool EXTRA, int TPB>
__global__ __launch_bounds__(TPB) void step_kernel_r1p(StepArgs a)
{
    StepArgs b = a;
    b.lgR = 0;
    step_body<STORAGE, false, MODE, UD, SHED, EXTRA, TPB, PB>(b, blockIdx.x, gridDim.x);
}

template <int S, int U, int PB, bool SHED, bool EXTRA>
const void* step_kernel_r1p_sel(int mode)
{
    if (mode == MODE_RESIDENT)
        return (const void*)&step_kernel_r1p<S, MODE_RESIDENT, U, PB, SHED, EXTRA, RESIDENT_TPB>;
    if (mode == MODE_SUMMARY)
        return (const void*)&step_kernel_r1p<S, MODE_SUMMARY, U, PB, SHED, EXTRA, RESIDENT_TPB>;
    return (const void*)&step_kernel_r1p<S, MODE_STREAM, U, PB, SHED, EXTRA, STREAM_TPB>;
}

// udeg: the uniform layout's degree, or -1 for a mixed layout
template <int S, int PB, bool SHED, bool EXTRA>
const void* step_kernel_r1p_depth(int mode, int udeg)
{
    if (udeg < 0) return step_kernel_r1p_sel<S, 0, PB, SHED, EXTRA>(mode);
    if (udeg <= 8) return step_kernel_r1p_sel<S, 8, PB, SHED, EXTRA>(mode);
    if (udeg <= 10) return step_kernel_r1p_sel<S, 10, PB, SHED, EXTRA>(mode);
    return step_kernel_r1p_sel<S, 12, PB, SHED, EXTRA>(mode);
}

template <int S, bool W, int U>
const void* step_kernel_r1_sel(int mode)
{
    if (mode == MODE_RESIDENT) return (const void*)&step_kernel_r1<S, W, MODE_RESIDENT, U, RESIDENT_TPB>;
    if (mode == MODE_SUMMARY) return (const void*)&step_kernel_r1<S, W, MODE_SUMMARY, U, RESIDENT_TPB>;
    return (const void*)&step_kernel_r1<S, W, MODE_STREAM, U, STREAM_TPB>;
}

// udeg: the uniform layout's degree, or -1 for a mixed layout
template <int S, bool W>
const void* step_kernel_r1_depth(int mode, int udeg)
{
    if (udeg < 0) return step_kernel_r1_sel<S, W, 0>(mode);
    if (udeg <= 8) return step_kernel_r1_sel<S, W, 8>(mode);
    if (udeg <= 10) return step_kernel_r1_sel<S, W, 10>(mode);
    return step_kernel_r1_sel<S, W, 12>(mode);
}

// Plain step kernels of unit-weight sims with 16 replicas (the scenario
// server's replica count): the replica shift is a compile-time constant, which
// frees the scalar registers that the general kernel's walk spills.
template <int STORAGE, int MODE, int UD, int TPB>
__global__ __launch_bounds__(TPB) void step_kernel_r16(StepArgs a)
{
    StepArgs b = a;
    b.lgR = 4;
    step_body<STORAGE, false, MODE, UD, false, false, TPB>(b, blockIdx.x, gridDim.x);
}

template <int S, int U>
const void* step_kernel_r16_sel(int mode)
{
    if (mode == MODE_RESIDENT) return (const void*)&step_kernel_r16<S, MODE_RESIDENT, U, RESIDENT_TPB>;
    if (mode == MODE_SUMMARY) return (const void*)&step_kernel_r16<S, MODE_SUMMARY, U, RESIDENT_TPB>;
    return (const void*)&step_kernel_r16<S, MODE_STREAM, U, STREAM_TPB>;
}

// udeg: the uniform layout's degree, or -1 for a mixed layout
template <int S>
const void* step_kernel_r16_depth(int mode, int udeg)
{
    if (udeg < 0) return step_kernel_r16_sel<S, 0>(mode);
    if (udeg <= 8) return step_kernel_r16_sel<S, 8>(mode);
    if (udeg <= 10) return step_kernel_r16_sel<S, 10>(mode);
    return step_kernel_r16_sel<S, 12>(mode);
}

// Address of the step kernel of one configuration (each (SHED, EXTRA)
// combination is instantiated by a kernel source of its own).
template <bool SHED, bool EXTRA, int S, bool W, int U>
const void* step_kernel_sel(int mode)
{
    if (mode == MODE_RESIDENT) return (const void*)&step_kernel<S, W, MODE_RESIDENT, U, SHED, EXTRA, RESIDENT_TPB>;
    if (mode == MODE_SUMMARY) return (const void*)&step_kernel<S, W, MODE_SUMMARY, U, SHED, EXTRA, RESIDENT_TPB>;
    return (const void*)&step_kernel<S, W, MODE_STREAM, U, SHED, EXTRA, STREAM_TPB>;
}

template <bool SHED, bool EXTRA, int S, bool W>
const void* step_kernel_depth(int mode, int udeg)
{
    static_assert(UMAX == 12, "uniform preload depths 8, 10, 12");
    if (udeg < 0) return step_kernel_sel<SHED, EXTRA, S, W, 0>(mode);
    if (udeg <= 8) return step_kernel_sel<SHED, EXTRA, S, W, 8>(mode);
    if (udeg <= 10) return step_kernel_sel<SHED, EXTRA, S, W, 10>(mode);
    return step_kernel_sel<SHED, EXTRA, S, W, 12>(mode);
}

// udeg: the layout's uniform degree, or -1 for a mixed layout
template <bool SHED, bool EXTRA>
const void* step_kernel_pick(int storage, bool weighted, int mode, int udeg)
{
    if (storage == 0 && !weighted) return step_kernel_depth<SHED, EXTRA, 0, false>(mode, udeg);
    if (storage == 0 && weighted) return step_kernel_depth<SHED, EXTRA, 0, true>(mode, udeg);
    if (storage == 1 && !weighted) return step_kernel_depth<SHED, EXTRA, 1, false>(mode, udeg);
    if (storage == 1 && weighted) return step_kernel_depth<SHED, EXTRA, 1, true>(mode, udeg);
    return nullptr;
}

// Index of the table entry that owns workgroup b: first[m] <= b < first[m + 1]
// (a uniform binary search over the members' block ranges).
__device__ __forceinline__ uint32_t owner_of(const uint32_t* __restrict__ first, uint32_t members, uint32_t b)
{
    uint32_t lo = 0, hi = members;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (first[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// One fused step for every member of a batch of simulations (each with its
// own graph, laws, replicas and step index): member m owns the workgroups
// [first[m], first[m + 1]) and runs exactly the streaming step on them, so
// its results are those it gets alone.  step_off is the launch's position in
// its sequence (member m runs step table[m].ctl->step + step_off).
template <int STORAGE, bool WEIGHTED, bool EXTRA>
__global__ __launch_bounds__(STREAM_TPB) void step_batch_kernel(const StepArgs* __restrict__ table,
                                                                const uint32_t* __restrict__ first,
                                                                uint32_t members, uint32_t step_off)
{
    const uint32_t m = owner_of(first, members, blockIdx.x);
    StepArgs a = table[m];
    a.step_off = step_off;
    step_body<STORAGE, WEIGHTED, MODE_STREAM, false, false, EXTRA, STREAM_TPB>(a, blockIdx.x - first[m],
                                                                               first[m + 1] - first[m]);
}


// Pressure partials of heavy-row segments (degree-binned dispatch).  One
// wavefront per segment: lane l covers edge offset l / R and replica l % R,
// so the 64 lanes read 64 / R edges per pass; the per-replica totals are
// folded with a fixed shuffle tree (deterministic) and lanes 0..R-1 store
// them.  Reads the same start-of-step bitmap (and, with SHED, shedding
// values) as the step launch that follows.
template <bool WEIGHTED, bool SHED>
__device__ __forceinline__ void heavy_body(const HeavyArgs& h, uint32_t block, uint32_t nblocks)
{
    constexpr bool FLOATP = WEIGHTED || SHED;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t R = 1u << h.lgR;
    const uint32_t per = 64u >> h.lgR; // edges per pass
    const uint32_t eoff = lane >> h.lgR;
    const uint32_t rep = lane & (R - 1);
    const unsigned long long k = h.ctl->step + h.step_off;
    const uint32_t* __restrict__ bits = (const uint32_t*)((k & 1) ? h.iota1 : h.iota0);
    const void* __restrict__ shv = (k & 1) ? h.shed1 : h.shed0;
    const uint32_t nwaves = nblocks * (WG / 64);
    unsigned long long rmask = 1ull; // lanes of replica 0: every R-th lane
    for (uint32_t sh = R; sh < 64u; sh <<= 1) rmask |= rmask << sh;
    for (uint32_t s = block * (WG / 64) + (threadIdx.x >> 6); s < h.nseg; s += nwaves) {
        const Segment sg = h.segs[s];
        // only rows that are susceptible (in some replica) read their pressure
        const uint32_t ru = ((uint32_t)sg.row << h.lgR) + rep;
        const int x = h.storage ? (int)((const uint8_t*)h.state)[ru] : (int)((const int32_t*)h.state)[ru];
        if (__ballot(x == ST_S) == 0ull) continue;
        // integer counts by one ballot per edge pass and replica (lanes r,
        // r + R, ... hold replica r; lanes below R, at edge offset 0, take
        // part in every pass), float sums by a fixed shuffle tree
        uint32_t ci = 0;
        float cw = 0.0f;
        for (int32_t e = sg.e_begin + (int32_t)eoff; e < sg.e_end; e += (int32_t)per) {
            const uint32_t src = ((uint32_t)h.col_ind[e] << h.lgR) + rep;
            const uint32_t b = bit_at(bits, src);
            const float v = SHED ? (b ? (h.storage ? half_bits_to_float(((const uint16_t*)shv)[src])
                                                   : ((const float*)shv)[src])
                                      : 0.0f)
                                 : (float)b;
            if (WEIGHTED) cw = __builtin_fmaf(h.weights[e], v, cw);
            else if (SHED) cw += v;
            else ci += (uint32_t)__popcll(__ballot(b != 0u) & (rmask << rep));
        }
        if (FLOATP)
            for (uint32_t off = 32; off >= R && off > 0; off >>= 1) cw += __shfl_down(cw, off, 64);
        if (lane < R) {
            if (FLOATP) ((float*)h.seg_part)[(size_t)s * R + lane] = cw;
            else ((uint32_t*)h.seg_part)[(size_t)s * R + lane] = ci;
        }
    }
}

template <bool WEIGHTED, bool SHED>
__global__ __launch_bounds__(WG) void heavy_pressure_kernel(HeavyArgs h)
{
    heavy_body<WEIGHTED, SHED>(h, blockIdx.x, gridDim.x);
}

// Column slots of a heavy segment each lane loads ahead (HC * 64 / R edges),
// and segments whose loads are issued together (HB).
constexpr int HC = 4;
constexpr int HB = 8;

// The loads of one heavy segment, as issued.
struct HeavySeg {
    uint32_t seg, len;          // segment index, edge count (0: none)
    uint32_t x;                 // the row's state in this lane's replica
    int32_t c[HC];
    float w[HC];
};

// Heavy-row partials with the bitmap resident in LDS (sims whose step runs
// the resident variant): one RESIDENT_TPB-thread workgroup per CU copies the
// step's input bitmap into LDS as the step kernel does.  Wave v takes
// segments v, v + nwaves, ...; their descriptors come 64 at a time from one
// vector load (lane j: the group's j-th segment), and the state words and
// first HC column slots (and weights) of HB segments are issued together
// before any of them is gathered, so a wave waits about one memory latency
// per HB segments.  Per lane the edges are summed in the same order, and
// folded by the same shuffle tree, as in heavy_body.
template <bool WEIGHTED, bool SHED>
__device__ __forceinline__ void heavy_resident_body(const HeavyArgs& h, uint32_t block, uint32_t nblocks)
{
    constexpr bool FLOATP = WEIGHTED || SHED;
    constexpr uint32_t NW = RESIDENT_TPB / 64;
    __shared__ __attribute__((aligned(16))) uint32_t s_bits[RESIDENT_BITS / 32];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int32_t lgR = h.lgR;
    const uint32_t R = 1u << lgR;
    const uint32_t per = 64u >> lgR;
    const uint32_t eoff = lane >> lgR;
    const uint32_t rep = lane & (R - 1);
    const unsigned long long k = h.ctl->step + h.step_off;
    const uint32_t* __restrict__ bits = (const uint32_t*)((k & 1) ? h.iota1 : h.iota0);
    const rsrc_t shedr = make_rsrc((k & 1) ? h.shed1 : h.shed0, SHED ? h.units * (h.storage ? 2u : 4u) : 0u);
    const uint32_t nw = nblocks * NW;
    const uint32_t s0 = block * NW + wave;
    // lanes of replica 0: every R-th lane
    unsigned long long rmask = 1ull;
    for (uint32_t sh = R; sh < 64u; sh <<= 1) rmask |= rmask << sh;
    const uint32_t cnt = h.nseg > s0 ? (h.nseg - s0 + nw - 1) / nw : 0u;
    const rsrc_t segr = make_rsrc(h.segs, h.nseg * (uint32_t)sizeof(Segment));
    const rsrc_t str = make_rsrc(h.state, h.units * (h.storage ? 1u : 4u));

    // this wave's first descriptor group is loaded with the bitmap fill
    uint32_t dr = 0, db = 0, de = 0;
    auto load_group = [&](uint32_t i0) {
        const uint32_t off = i0 + lane < cnt ? (s0 + (i0 + lane) * nw) * (uint32_t)sizeof(Segment) : OOB;
        const auto d = __builtin_amdgcn_raw_buffer_load_b128(segr, (int)off, 0, 0);
        dr = d[0];
        db = d[1];
        de = d[2];
    };
    load_group(0);
    {
        const uint32_t n4 = (((h.units + 31) >> 5) + 3) >> 2;
        const uint4* src = (const uint4*)bits;
        for (uint32_t b0 = wave * 64; b0 < n4; b0 += RESIDENT_TPB) {
            if (b0 + lane < n4)
                __builtin_amdgcn_global_load_lds((const void*)(src + b0 + lane),
                                                 (__attribute__((address_space(3))) void*)((uint4*)s_bits + b0), 16, 0, 0);
        }
        __builtin_amdgcn_s_waitcnt(0);
    }
    __syncthreads();

    // the loads of the group's segment j (none past the group's end)
    auto issue = [&](uint32_t i0, uint32_t j, HeavySeg& S) {
        const bool has = j < 64u && i0 + j < cnt;
        const uint32_t jj = has ? j : 0u;
        const uint32_t row = __builtin_amdgcn_readlane(dr, jj);
        const uint32_t eb = __builtin_amdgcn_readlane(db, jj);
        const uint32_t ee = __builtin_amdgcn_readlane(de, jj);
        S.seg = s0 + (i0 + jj) * nw;
        S.len = has ? ee - eb : 0u;
        const uint32_t ru = (row << lgR) + rep;
        S.x = h.storage ? __builtin_amdgcn_raw_buffer_load_b8(str, has ? (int)ru : (int)OOB, 0, 0)
                        : ld32(str, has ? ru << 2 : OOB);
        const rsrc_t cr = make_rsrc(h.col_ind + eb, S.len * 4u);
        const rsrc_t wr = make_rsrc(WEIGHTED ? (const void*)(h.weights + eb) : (const void*)h.weights,
                                    WEIGHTED ? S.len * 4u : 0u);
#pragma unroll
        for (int i = 0; i < HC; ++i) {
            const uint32_t off = ((uint32_t)i * per + eoff) << 2;
            S.c[i] = (int32_t)ld32(cr, off);
            S.w[i] = WEIGHTED ? __uint_as_float(ld32(wr, off)) : 0.0f;
        }
    };
    auto process = [&](const HeavySeg& S) {
        // only rows that are susceptible (in some replica) read their pressure
        if (S.len == 0u || __ballot(S.x == (uint32_t)ST_S) == 0ull) return;
        // integer counts: each edge pass's bits are counted per replica with
        // one ballot (lanes r, r + R, ... hold replica r; lanes below R take
        // part in every pass, their edge offset being 0), which gives the
        // same totals as the shuffle tree without its LDS round trips
        uint32_t ci = 0;
        float cw = 0.0f;
        auto add = [&](int32_t c, float w) {
            const uint32_t src = ((uint32_t)c << lgR) + rep;
            const uint32_t b = lds_bit(s_bits, src);
            const float v = SHED ? (h.storage ? shed_at<1>(shedr, src, b != 0u) : shed_at<0>(shedr, src, b != 0u))
                                 : (float)b;
            if (WEIGHTED) cw = __builtin_fmaf(w, v, cw);
            else if (SHED) cw += v;
            else ci += (uint32_t)__popcll(__ballot(b != 0u) & (rmask << rep));
        };
#pragma unroll
        for (int i = 0; i < HC; ++i)
            if ((uint32_t)i * per + eoff < S.len) add(S.c[i], S.w[i]);
        if (S.len > (uint32_t)HC * per) {
            // the rest of a long segment, unprefetched
            const uint32_t eb = (uint32_t)h.segs[S.seg].e_begin;
            for (uint32_t e = HC * per + eoff; e < S.len; e += per)
                add(h.col_ind[eb + e], WEIGHTED ? h.weights[eb + e] : 0.0f);
        }
        if (FLOATP)
            for (uint32_t off = 32; off >= R && off > 0; off >>= 1) cw += __shfl_down(cw, off, 64);
        if (lane < R) {
            if (FLOATP) ((float*)h.seg_part)[(size_t)S.seg * R + lane] = cw;
            else ((uint32_t*)h.seg_part)[(size_t)S.seg * R + lane] = ci;
        }
    };

    for (uint32_t i0 = 0; i0 < cnt; i0 += 64) {
        if (i0 > 0) load_group(i0);
        const uint32_t m = min(64u, cnt - i0);
        for (uint32_t j0 = 0; j0 < m; j0 += HB) {
            HeavySeg S[HB];
#pragma unroll
            for (int b = 0; b < HB; ++b) issue(i0, j0 + b < m ? j0 + b : 64u, S[b]);
#pragma unroll
            for (int b = 0; b < HB; ++b) process(S[b]);
        }
    }
}

template <bool WEIGHTED, bool SHED>
__global__ __launch_bounds__(RESIDENT_TPB) void heavy_resident_kernel(HeavyArgs h)
{
    heavy_resident_body<WEIGHTED, SHED>(h, blockIdx.x, gridDim.x);
}

// Batched heavy-row partials: member m owns workgroups [first[m], first[m + 1]).
template <bool WEIGHTED>
__global__ __launch_bounds__(WG) void heavy_batch_kernel(const HeavyArgs* __restrict__ table,
                                                         const uint32_t* __restrict__ first, uint32_t members,
                                                         uint32_t step_off)
{
    const uint32_t m = owner_of(first, members, blockIdx.x);
    HeavyArgs h = table[m];
    h.step_off = step_off;
    heavy_body<WEIGHTED, false>(h, blockIdx.x - first[m], first[m + 1] - first[m]);
}


} // namespace fsk
