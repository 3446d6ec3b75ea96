// HIP kernels of the renewal tau-leap step (FlashSpread, arXiv 2604.22092,
// Algorithm 3 with Eq. (influence), Eq. (infectivity), Proposition 1 and the
// Bernoulli tau-leap rule), written for gfx950 (wave64).
//
// One launch performs one whole step for every (node, replica) unit:
//   pressure gather over the incoming CSR row (S units only: the rate of
//   E, I and R units does not depend on it), rate by state, Philox draw,
//   state/age advance in place, next-step infectivity into the other
//   ping-pong buffer, and exact per-step S/E/I/R counts.
// A sequence of r step launches (launch j runs step ctl->step + j) is
// followed by one reduce launch that sums the per-workgroup count partials of
// every step into the count history, and one single-thread launch that
// advances ctl->step by r.  No step kernel uses a global atomic.
#include <hip/hip_runtime.h>

#include "fs_device.hpp"
#include "fs_internal.hpp"
#include "fs_kernels.hpp"

namespace fsk {

using namespace fsi;

template <int STORAGE>
struct Store;
template <>
struct Store<0> {
    using state_t = int32_t;
    using age_t = float;
};
template <>
struct Store<1> {
    using state_t = uint8_t;
    using age_t = uint16_t;
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
template <int MODE>
__device__ __forceinline__ uint32_t fetch_bit(const uint32_t* __restrict__ lds, rsrc_t gbits, uint32_t b,
                                              int32_t lg_gran, bool use)
{
    if (MODE == MODE_RESIDENT) return use ? lds_bit(lds, b) : 0u;
    bool go = use;
    if (MODE == MODE_SUMMARY) go = go && lds_bit(lds, b >> lg_gran) != 0u;
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
};

// Issues every load of a pass that does not depend on the state: chunk
// metadata (one scalar load), state, age and light degree, and the edge
// slots of uniform chunks (whose rows are all present).  Each array is read
// through a descriptor covering only this chunk's valid entries, so no lane
// branches and a pass past the last chunk reads nothing.
template <int STORAGE, bool UNIFORM, class age_t>
__device__ __forceinline__ void issue_pass(const StepArgs& a, uint32_t first, uint32_t nwaves, uint32_t nchunks,
                                           uint32_t total, uint32_t lane, Pass<age_t>& P)
{
    using state_t = typename Store<STORAGE>::state_t;
    const uint32_t rows = 64u >> a.lgR;
    const uint32_t q = lane >> a.lgR;
#pragma unroll
    for (int u = 0; u < CU; ++u) {
        const uint32_t c = __builtin_amdgcn_readfirstlane(first + (uint32_t)u * nwaves);
        P.live[u] = c < nchunks;
        P.chk[u] = P.live[u] ? c : nchunks - 1;
        if (UNIFORM) {
            P.base[u] = P.chk[u] * rows * (uint32_t)a.udeg;
            P.ud[u] = P.live[u] ? (uint32_t)a.udeg : 0u;
        } else {
            const uint2 meta = a.chunk_meta[P.chk[u]];
            P.base[u] = meta.x;
            P.ud[u] = P.live[u] ? meta.y : 0u;
        }
        const uint32_t u0 = P.chk[u] << 6;
        P.nvalid[u] = P.live[u] ? min(64u, total - u0) : 0u;
        const uint32_t n0 = u0 >> a.lgR;
        const uint32_t nrows = P.live[u] ? min(rows, (uint32_t)a.n - n0) : 0u;
        P.xr[u] = BufIO<state_t>::ld(make_rsrc((const state_t*)a.state + u0, P.nvalid[u] * sizeof(state_t)), lane);
        P.agw[u] = BufIO<age_t>::ld(make_rsrc((const age_t*)a.age + u0, P.nvalid[u] * sizeof(age_t)), lane);
        P.dgr[u] = BufIO<uint16_t>::ld(make_rsrc(a.ldeg + n0, nrows * 2u), q);
        // graphs in a degree-sorted order (never uniform ones) key the draws
        // by the caller's node id
        P.org[u] = UNIFORM ? n0 + q : ld32(make_rsrc(a.orig_id + n0, nrows * 4u), q << 2);
        const bool pre = P.ud[u] <= (uint32_t)UMAX;
        const rsrc_t cr = make_rsrc(a.col_t + P.base[u], pre ? P.ud[u] * rows * 4u : 0u);
#pragma unroll
        for (int j = 0; j < UMAX; ++j) P.c[u][j] = (int32_t)ld32(cr, ((uint32_t)j * rows + q) << 2);
    }
}

// Pressure of one chunk's light row for this lane (Eq. (influence) without
// beta).  Uniform chunks use the preloaded slots; mixed chunks find a row's
// position in run j as its rank among the rows with more than j edges (ballot
// prefix count), JB slots at a time.
template <int MODE, bool WEIGHTED, bool UNIFORM, class age_t>
__device__ __forceinline__ float pressure_row(const StepArgs& a, const Pass<age_t>& P, int u, bool want,
                                              uint32_t dg, const uint32_t* __restrict__ lds, rsrc_t gbits,
                                              uint32_t lane)
{
    const int32_t lgR = a.lgR;
    const uint32_t R = 1u << lgR;
    const uint32_t rep = lane & (R - 1);
    const uint32_t d = dg == HEAVY_ROW ? 0u : dg;
    uint32_t pi = 0;
    float pw = 0.0f;
    if (UNIFORM || P.ud[u] <= (uint32_t)UMAX) {
        // uniform chunk: slots past the degree hold 0 (a valid node) and are
        // not used; weights come through the same per-chunk range
        const uint32_t rows = 64u >> lgR;
        const uint32_t q = lane >> lgR;
        const rsrc_t wr = make_rsrc(WEIGHTED ? (const void*)(a.w_t + P.base[u]) : (const void*)a.w_t,
                                    WEIGHTED ? P.ud[u] * rows * 4u : 0u);
#pragma unroll
        for (int j = 0; j < UMAX; ++j) {
            const bool use = (uint32_t)j < P.ud[u] && want;
            const uint32_t b = fetch_bit<MODE>(lds, gbits, ((uint32_t)P.c[u][j] << lgR) + rep, a.lg_gran, use);
            if (WEIGHTED) {
                const float w = __uint_as_float(ld32(wr, use ? ((uint32_t)j * rows + q) << 2 : OOB));
                pw = __builtin_fmaf(w, (float)b, pw);
            } else {
                pi += b;
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
                    const uint32_t b = fetch_bit<MODE>(lds, gbits, ((uint32_t)c[jj] << lgR) + rep, a.lg_gran, true);
                    if (WEIGHTED) pw = __builtin_fmaf(wv[jj], (float)b, pw);
                    else pi += b;
                }
            }
        }
    }
    return WEIGHTED ? pw : (float)pi;
}

// Pressure of a degree-binned row: its segment partials in segment order.
template <bool WEIGHTED>
__device__ __forceinline__ float pressure_heavy(const StepArgs& a, uint32_t node, uint32_t rep)
{
    const size_t R = (size_t)1 << a.lgR;
    const int32_t dg = a.row_ptr[node + 1] - a.row_ptr[node];
    const int32_t first = a.heavy_first[node];
    const int32_t nseg = (dg + a.seg_edges - 1) / a.seg_edges;
    if (WEIGHTED) {
        const float* sp = (const float*)a.seg_part;
        float p = 0.0f;
        for (int32_t j = 0; j < nseg; ++j) p += sp[(size_t)(first + j) * R + rep];
        return p;
    }
    const uint32_t* sp = (const uint32_t*)a.seg_part;
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
// hazards), draws, stores, next-infectivity words and counts.
template <int STORAGE, bool WEIGHTED, bool RATES, int MODE, bool UNIFORM, class age_t>
__device__ __forceinline__ void process_pass(const StepArgs& a, const Pass<age_t>& P, uint32_t lane,
                                             const uint32_t* __restrict__ s_bits, rsrc_t gbits, uint32_t* xch,
                                             unsigned long long k, unsigned long long* __restrict__ bits_out,
                                             uint32_t* s_cnt, uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                             uint32_t& c3, float dt, float& lmax)
{
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
        const float p = pressure_row<MODE, WEIGHTED, UNIFORM>(a, P, u, want, dg[u], s_bits, gbits, lane);
        if (want) lam[u] = a.beta * p;
        if (!UNIFORM && heavy && x[u] == ST_S)
            lam[u] = a.beta * pressure_heavy<WEIGHTED>(a, unit[u] >> a.lgR, unit[u] & (R - 1));
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
        compact_apply<CU>(xch, lane, need, pay, res, [&](uint32_t w) {
            const bool isI = (w & 0x80000000u) != 0u;
            const float xa = age_from_bits<age_t>(w & 0x7FFFFFFFu);
            float h;
            if (a.same_kind) {
                HazardDev hd = a.hz[0];
                if (isI) hd = a.hz[1];
                hd.kind = a.hz[0].kind;
                h = fsd::hazard(hd, xa);
            } else {
                h = isI ? fsd::hazard(a.hz[1], xa) : fsd::hazard(a.hz[0], xa);
            }
            return __float_as_uint(h);
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
            return fsd::philox4x32_10(make_uint4(un >> a.lgR, kk, un & (R - 1), 0u), a.key0, a.key1).x >> 8;
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

#pragma unroll
    for (int u = 0; u < CU; ++u) {
        // 5.-6. advance state and age in place (the chunk's descriptors drop
        // the lanes past its valid units; the state only changes on a firing)
        const int xn = x[u] + (fire[u] ? 1 : 0);
        const uint32_t u0 = P.chk[u] << 6;
        BufIO<state_t>::st(make_rsrc((state_t*)a.state + u0, P.nvalid[u] * sizeof(state_t)),
                           fire[u] ? lane : OOB_ELEM, (uint32_t)xn);
        BufIO<age_t>::st(make_rsrc((age_t*)a.age + u0, P.nvalid[u] * sizeof(age_t)), lane,
                         age_to_raw(fire[u] ? (age_t)0 : age_next(ag[u], dt)));
        lmax = fmaxf(lmax, lam[u]);
        if (RATES) st32(make_rsrc(a.rates + u0, P.nvalid[u] * 4u), lane << 2, __float_as_uint(lam[u]));
        // 7. next-step infectivity bits (one 64-bit word per chunk, written by
        // lanes 0 and 1) and 8. counts
        const unsigned long long mI = __ballot(valid[u] && xn == ST_I);
        st32(make_rsrc(bits_out + P.chk[u], P.live[u] ? 8u : 0u), lane < 2 ? lane << 2 : OOB,
             lane == 0 ? (uint32_t)mI : (uint32_t)(mI >> 32));
        if (R == 1) {
            c0 += (uint32_t)__popcll(__ballot(valid[u] && xn == ST_S));
            c1 += (uint32_t)__popcll(__ballot(valid[u] && xn == ST_E));
            c2 += (uint32_t)__popcll(mI);
            c3 += (uint32_t)__popcll(__ballot(valid[u] && xn == ST_R));
        } else if (valid[u]) {
            atomicAdd(&s_cnt[(unit[u] & (R - 1)) * 4 + xn], 1u); // LDS
        }
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
template <int STORAGE, bool WEIGHTED, bool RATES, int MODE, bool UNIFORM, int TPB>
__device__ __forceinline__ void step_body(const StepArgs& a, uint32_t block, uint32_t nblocks)
{
    constexpr bool USE_LDS = MODE != MODE_STREAM;
    using age_t = typename Store<STORAGE>::age_t;
    constexpr int NW = TPB / 64;

    __shared__ uint32_t s_cnt[4 * 64];
    __shared__ __attribute__((aligned(16))) uint32_t s_bits[USE_LDS ? RESIDENT_BITS / 32 : 4];
    static_assert(SUMMARY_BITS <= RESIDENT_BITS, "the summary shares the LDS bitmap array");
    __shared__ uint32_t s_xch[NW][64];

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

    // first pass loads, then the bitmap fill, then one wait for both
    Pass<age_t> P;
    uint32_t first = wave_id;
    issue_pass<STORAGE, UNIFORM>(a, first, nwaves, nchunks, total, lane, P);
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

    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0; // per-wave counts (R == 1)

    // passes: the loads of the next pass are issued (always: a pass past the
    // end reads nothing) before the current pass is processed; two register
    // sets, unrolled by two
    Pass<age_t> P1;
    const uint32_t stride = nwaves * CU;
    for (;;) {
        if (first >= nchunks) break;
        if (PREFETCH) issue_pass<STORAGE, UNIFORM>(a, first + stride, nwaves, nchunks, total, lane, P1);
        process_pass<STORAGE, WEIGHTED, RATES, MODE, UNIFORM>(a, P, lane, s_bits, gbits, s_xch[wave], k, bits_out,
                                                              s_cnt, c0, c1, c2, c3, dt, lmax);
        first += stride;
        if (first >= nchunks) break;
        if (!PREFETCH) issue_pass<STORAGE, UNIFORM>(a, first, nwaves, nchunks, total, lane, P1);
        if (PREFETCH) issue_pass<STORAGE, UNIFORM>(a, first + stride, nwaves, nchunks, total, lane, P);
        process_pass<STORAGE, WEIGHTED, RATES, MODE, UNIFORM>(a, P1, lane, s_bits, gbits, s_xch[wave], k, bits_out,
                                                              s_cnt, c0, c1, c2, c3, dt, lmax);
        first += stride;
        if (!PREFETCH && first < nchunks) issue_pass<STORAGE, UNIFORM>(a, first, nwaves, nchunks, total, lane, P);
    }

    // one plain store of this workgroup's counts; the reduce kernel sums them
    uint32_t* out = a.part + ((size_t)a.step_off * nblocks + block) * (4 * R);
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
            out[tid] = t;
        }
    } else {
        __syncthreads();
        for (uint32_t i = tid; i < 4 * R; i += TPB) out[i] = s_cnt[i];
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

template <int STORAGE, bool WEIGHTED, bool RATES, int MODE, bool UNIFORM, int TPB>
__global__ __launch_bounds__(TPB) void step_kernel(StepArgs a)
{
    step_body<STORAGE, WEIGHTED, RATES, MODE, UNIFORM, TPB>(a, blockIdx.x, gridDim.x);
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
template <int STORAGE, bool WEIGHTED, bool RATES>
__global__ __launch_bounds__(STREAM_TPB) void step_batch_kernel(const StepArgs* __restrict__ table,
                                                                const uint32_t* __restrict__ first,
                                                                uint32_t members, uint32_t step_off)
{
    const uint32_t m = owner_of(first, members, blockIdx.x);
    StepArgs a = table[m];
    a.step_off = step_off;
    step_body<STORAGE, WEIGHTED, RATES, MODE_STREAM, false, STREAM_TPB>(a, blockIdx.x - first[m],
                                                                        first[m + 1] - first[m]);
}

// Sums per-workgroup count partials.  Block j handles slot j: rows of C
// counters from G workgroups, part[j][g][c]; the totals go to
// out[((base + j) mod H)][c] where base = ctl->step (0 without ctl).
// Requires C <= WG and WG % C == 0 (C = 4R with R a power of two <= 64).
__device__ __forceinline__ void reduce_body(const Ctl* ctl, const uint32_t* part, uint32_t G, uint32_t C,
                                            uint32_t* out, uint32_t H, uint32_t j, uint32_t r)
{
    __shared__ uint32_t s[WG];
    const uint32_t t = threadIdx.x;
    // of a sequence longer than the ring only the last H steps are kept, so
    // no two blocks write one slot
    if ((size_t)j + H < (size_t)r) return;
    const uint32_t groups = WG / C;
    const uint32_t c = t % C;
    const uint32_t* p = part + (size_t)j * G * C;
    uint32_t sum = 0;
    for (uint32_t g = t / C; g < G; g += groups) sum += p[(size_t)g * C + c];
    s[t] = sum;
    __syncthreads();
    if (t < C) {
        uint32_t tot = 0;
        for (uint32_t i = 0; i < groups; ++i) tot += s[i * C + t];
        const unsigned long long base = ctl ? ctl->step : 0ull;
        out[(size_t)((base + j) % H) * C + t] = tot;
    }
}

__global__ __launch_bounds__(WG) void reduce_kernel(const Ctl* ctl, const uint32_t* part, uint32_t G,
                                                     uint32_t C, uint32_t* out, uint32_t H)
{
    reduce_body(ctl, part, G, C, out, H, blockIdx.x, gridDim.x);
}

// Batched reduce: block (j, m) sums slot j of member m (grid r x members).
__global__ __launch_bounds__(WG) void reduce_batch_kernel(const RedArgs* __restrict__ table)
{
    const RedArgs q = table[blockIdx.y];
    reduce_body(q.ctl, q.part, q.G, q.C, q.hist, q.H, blockIdx.x, gridDim.x);
}

__global__ void advance_kernel(Ctl* ctl, uint32_t r)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->step = ctl->step + r;
}

// Batched advance: thread m adds r to member m's step index.
__global__ void advance_batch_kernel(Ctl* const* __restrict__ ctls, uint32_t members, uint32_t r)
{
    const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < members) ctls[m]->step = ctls[m]->step + r;
}

// Summary of an infectivity bitmap: bit s is set when any of the 2^lg_gran
// units of group s is infectious, i.e. when one of its 2^(lg_gran - 6) bitmap
// words is nonzero.  One thread per summary bit, one summary word per wave.
__global__ __launch_bounds__(WG) void summary_kernel(SumArgs q)
{
    const unsigned long long k = q.ctl->step + q.step_off + q.after;
    const unsigned long long* __restrict__ bits = (k & 1) ? q.iota1 : q.iota0;
    const uint32_t s = blockIdx.x * WG + threadIdx.x;
    const uint32_t gw = 1u << (q.lg_gran - 6);
    const uint64_t w0 = (uint64_t)s * gw;
    bool any = false;
    for (uint32_t i = 0; i < gw; ++i)
        if (w0 + i < q.words && bits[w0 + i] != 0ull) any = true;
    const unsigned long long m = __ballot(any);
    if ((threadIdx.x & 63) == 0 && (s >> 6) < q.sum_words) q.summary[s >> 6] = m;
}

// Pressure partials of heavy-row segments (degree-binned dispatch).  One
// wavefront per segment: lane l covers edge offset l / R and replica l % R,
// so the 64 lanes read 64 / R edges per pass; the per-replica totals are
// folded with a fixed shuffle tree (deterministic) and lanes 0..R-1 store
// them.  Reads the same start-of-step bitmap as the step launch that follows.
template <bool WEIGHTED>
__device__ __forceinline__ void heavy_body(const HeavyArgs& h, uint32_t block, uint32_t nblocks)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t R = 1u << h.lgR;
    const uint32_t per = 64u >> h.lgR; // edges per pass
    const uint32_t eoff = lane >> h.lgR;
    const uint32_t rep = lane & (R - 1);
    const unsigned long long k = h.ctl->step + h.step_off;
    const uint32_t* __restrict__ bits = (const uint32_t*)((k & 1) ? h.iota1 : h.iota0);
    const uint32_t nwaves = nblocks * (WG / 64);
    for (uint32_t s = block * (WG / 64) + (threadIdx.x >> 6); s < h.nseg; s += nwaves) {
        const Segment sg = h.segs[s];
        uint32_t ci = 0;
        float cw = 0.0f;
        for (int32_t e = sg.e_begin + (int32_t)eoff; e < sg.e_end; e += (int32_t)per) {
            const uint32_t b = bit_at(bits, ((uint32_t)h.col_ind[e] << h.lgR) + rep);
            if (WEIGHTED) cw = __builtin_fmaf(h.weights[e], (float)b, cw);
            else ci += b;
        }
        for (uint32_t off = 32; off >= R && off > 0; off >>= 1) {
            if (WEIGHTED) cw += __shfl_down(cw, off, 64);
            else ci += __shfl_down(ci, off, 64);
        }
        if (lane < R) {
            if (WEIGHTED) ((float*)h.seg_part)[(size_t)s * R + lane] = cw;
            else ((uint32_t*)h.seg_part)[(size_t)s * R + lane] = ci;
        }
    }
}

template <bool WEIGHTED>
__global__ __launch_bounds__(WG) void heavy_pressure_kernel(HeavyArgs h)
{
    heavy_body<WEIGHTED>(h, blockIdx.x, gridDim.x);
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
    heavy_body<WEIGHTED>(h, blockIdx.x - first[m], first[m + 1] - first[m]);
}

template <int STORAGE>
__global__ __launch_bounds__(WG) void recount_kernel(const void* state_v, int32_t n, int32_t lgR,
                                                     int32_t replica, uint32_t* part)
{
    using state_t = typename Store<STORAGE>::state_t;
    const state_t* state = (const state_t*)state_v;
    __shared__ uint32_t s[4 * (WG / 64)];
    uint32_t c[4] = {0, 0, 0, 0};
    for (uint32_t tile = blockIdx.x; (size_t)tile * WG < (size_t)n; tile += gridDim.x) {
        const uint32_t i = tile * WG + threadIdx.x;
        const bool valid = i < (uint32_t)n;
        const int x = valid ? (int)state[((size_t)i << lgR) + replica] : -1;
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] += (uint32_t)__popcll(__ballot(x == q));
    }
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 4; ++q) s[(threadIdx.x >> 6) * 4 + q] = c[q];
    __syncthreads();
    if (threadIdx.x < 4) {
        uint32_t tot = 0;
        for (int w = 0; w < WG / 64; ++w) tot += s[w * 4 + threadIdx.x];
        part[blockIdx.x * 4 + threadIdx.x] = tot;
    }
}

// Writes one replica's contiguous state/age into the interleaved layout.
template <int STORAGE>
__global__ void put_replica_kernel(void* state_v, void* age_v, const int32_t* src_state, const void* src_age,
                                   int32_t n, int32_t lgR, int32_t replica)
{
    using S = Store<STORAGE>;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)n) return;
    const size_t u = ((size_t)i << lgR) + replica;
    ((typename S::state_t*)state_v)[u] = (typename S::state_t)src_state[i];
    ((typename S::age_t*)age_v)[u] = ((const typename S::age_t*)src_age)[i];
}

// Rebuilds an infectivity bitmap from the states: one 64-bit word per wave.
template <int STORAGE>
__global__ __launch_bounds__(WG) void rebuild_bits_kernel(const void* state_v, uint32_t total,
                                                          unsigned long long* bits, uint32_t words)
{
    using state_t = typename Store<STORAGE>::state_t;
    const uint32_t unit = blockIdx.x * WG + threadIdx.x;
    const bool valid = unit < total;
    const int x = valid ? (int)((const state_t*)state_v)[unit] : -1;
    const unsigned long long m = __ballot(x == ST_I);
    const uint32_t w = unit >> 6;
    if ((threadIdx.x & 63) == 0 && w < words) bits[w] = m;
}

template <int STORAGE>
__global__ void get_replica_kernel(const void* state_v, const void* age_v, int32_t* dst_state,
                                   void* dst_age, int32_t n, int32_t lgR, int32_t replica)
{
    using S = Store<STORAGE>;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)n) return;
    const size_t u = ((size_t)i << lgR) + replica;
    dst_state[i] = (int32_t)((const typename S::state_t*)state_v)[u];
    ((typename S::age_t*)dst_age)[i] = ((const typename S::age_t*)age_v)[u];
}

template <int STORAGE>
__global__ void get_rates_kernel(const float* rates, float* dst, int32_t n, int32_t lgR, int32_t replica)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint32_t)n) return;
    dst[i] = rates[((size_t)i << lgR) + replica];
}

// Seeds listed nodes of one replica (or all replicas) into `comp` at age 0.
template <int STORAGE>
__global__ void seed_kernel(void* state_v, void* age_v, const int64_t* nodes, int64_t count, int32_t lgR,
                            int32_t replica, int32_t comp)
{
    using S = Store<STORAGE>;
    const uint32_t R = 1u << lgR;
    const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= (uint64_t)count * (replica < 0 ? R : 1u)) return;
    const uint64_t idx = replica < 0 ? j / R : j;
    const uint32_t r = replica < 0 ? (uint32_t)(j % R) : (uint32_t)replica;
    const size_t u = ((size_t)nodes[idx] << lgR) + r;
    ((typename S::state_t*)state_v)[u] = (typename S::state_t)comp;
    ((typename S::age_t*)age_v)[u] = (typename S::age_t)0;
}

__global__ void clear_u32_kernel(uint32_t* p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void set_ctl_kernel(Ctl* ctl, unsigned long long step)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->step = step;
        ctl->adapt_from = step;
    }
}

__global__ void eval_hazard_kernel(HazardDev h, int32_t storage, const void* ages, float* out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = storage == 0 ? ((const float*)ages)[i] : (float)((const uint16_t*)ages)[i];
    out[i] = fsd::hazard(h, x);
}

__global__ void eval_philox_kernel(const uint4* ctr, uint32_t k0, uint32_t k1, uint4* out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = fsd::philox4x32_10(ctr[i], k0, k1);
}

// ---------------------------------------------------------------- launchers

template <int S, bool W, bool RT, bool U>
const void* step_kernel_sel(int mode)
{
    if (mode == MODE_RESIDENT) return (const void*)&step_kernel<S, W, RT, MODE_RESIDENT, U, RESIDENT_TPB>;
    if (mode == MODE_SUMMARY) return (const void*)&step_kernel<S, W, RT, MODE_SUMMARY, U, RESIDENT_TPB>;
    return (const void*)&step_kernel<S, W, RT, MODE_STREAM, U, STREAM_TPB>;
}

const void* step_kernel_fn(int storage, bool weighted, bool rates, int mode, bool uniform)
{
#define FS_SEL(S, W, RT)                                                                         \
    if (storage == S && weighted == W && rates == RT)                                            \
        return uniform ? step_kernel_sel<S, W, RT, true>(mode) : step_kernel_sel<S, W, RT, false>(mode);
    FS_SEL(0, false, false) FS_SEL(0, false, true) FS_SEL(0, true, false) FS_SEL(0, true, true)
    FS_SEL(1, false, false) FS_SEL(1, false, true) FS_SEL(1, true, false) FS_SEL(1, true, true)
#undef FS_SEL
    return nullptr;
}

static unsigned grid_for(size_t n, unsigned block) { return (unsigned)((n + block - 1) / block); }

hipError_t launch_recount(int storage, const void* state, int32_t n, int32_t lgR, int32_t replica,
                          uint32_t* part, uint32_t max_grid, uint32_t* out4, hipStream_t s)
{
    unsigned g = grid_for((size_t)n, WG);
    if (g > max_grid) g = max_grid;
    if (g == 0) g = 1;
    if (storage == 0)
        hipLaunchKernelGGL(recount_kernel<0>, dim3(g), dim3(WG), 0, s, state, n, lgR, replica, part);
    else
        hipLaunchKernelGGL(recount_kernel<1>, dim3(g), dim3(WG), 0, s, state, n, lgR, replica, part);
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(WG), 0, s, (const Ctl*)nullptr, (const uint32_t*)part,
                       (uint32_t)g, 4u, out4, 1u);
    return hipGetLastError();
}

const void* reduce_kernel_fn() { return (const void*)&reduce_kernel; }
const void* heavy_kernel_fn(bool weighted)
{
    return weighted ? (const void*)&heavy_pressure_kernel<true> : (const void*)&heavy_pressure_kernel<false>;
}
const void* advance_kernel_fn() { return (const void*)&advance_kernel; }
const void* summary_kernel_fn() { return (const void*)&summary_kernel; }

const void* step_batch_kernel_fn(int storage, bool weighted, bool rates)
{
#define FS_SEL(S, W, RT)                                                                         \
    if (storage == S && weighted == W && rates == RT) return (const void*)&step_batch_kernel<S, W, RT>;
    FS_SEL(0, false, false) FS_SEL(0, false, true) FS_SEL(0, true, false) FS_SEL(0, true, true)
    FS_SEL(1, false, false) FS_SEL(1, false, true) FS_SEL(1, true, false) FS_SEL(1, true, true)
#undef FS_SEL
    return nullptr;
}
const void* heavy_batch_kernel_fn(bool weighted)
{
    return weighted ? (const void*)&heavy_batch_kernel<true> : (const void*)&heavy_batch_kernel<false>;
}
const void* reduce_batch_kernel_fn() { return (const void*)&reduce_batch_kernel; }
const void* advance_batch_kernel_fn() { return (const void*)&advance_batch_kernel; }

hipError_t launch_put_replica(int storage, void* state, void* age, const int32_t* src_state, const void* src_age,
                              int32_t n, int32_t lgR, int32_t replica, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    unsigned g = grid_for((size_t)n, 256);
    if (storage == 0)
        hipLaunchKernelGGL(put_replica_kernel<0>, dim3(g), dim3(256), 0, s, state, age, src_state, src_age, n, lgR,
                           replica);
    else
        hipLaunchKernelGGL(put_replica_kernel<1>, dim3(g), dim3(256), 0, s, state, age, src_state, src_age, n, lgR,
                           replica);
    return hipGetLastError();
}

hipError_t launch_rebuild_bits(int storage, const void* state, uint32_t total, unsigned long long* bits,
                               uint32_t words, hipStream_t s)
{
    unsigned g = grid_for((size_t)words * 64, WG);
    if (g == 0) return hipSuccess;
    if (storage == 0)
        hipLaunchKernelGGL(rebuild_bits_kernel<0>, dim3(g), dim3(WG), 0, s, state, total, bits, words);
    else
        hipLaunchKernelGGL(rebuild_bits_kernel<1>, dim3(g), dim3(WG), 0, s, state, total, bits, words);
    return hipGetLastError();
}

hipError_t launch_get_replica(int storage, const void* state, const void* age, int32_t* dst_state,
                              void* dst_age, int32_t n, int32_t lgR, int32_t replica, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    unsigned g = grid_for((size_t)n, 256);
    if (storage == 0)
        hipLaunchKernelGGL(get_replica_kernel<0>, dim3(g), dim3(256), 0, s, state, age, dst_state, dst_age,
                           n, lgR, replica);
    else
        hipLaunchKernelGGL(get_replica_kernel<1>, dim3(g), dim3(256), 0, s, state, age, dst_state, dst_age,
                           n, lgR, replica);
    return hipGetLastError();
}

hipError_t launch_get_rates(const float* rates, float* dst, int32_t n, int32_t lgR, int32_t replica,
                            hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(get_rates_kernel<0>, dim3(grid_for((size_t)n, 256)), dim3(256), 0, s, rates, dst, n,
                       lgR, replica);
    return hipGetLastError();
}

hipError_t launch_seed(int storage, void* state, void* age, const int64_t* nodes, int64_t count, int32_t lgR,
                       int32_t replica, int32_t comp, hipStream_t s)
{
    const size_t work = (size_t)count * (replica < 0 ? (1u << lgR) : 1u);
    if (work == 0) return hipSuccess;
    unsigned g = grid_for(work, 256);
    if (storage == 0)
        hipLaunchKernelGGL(seed_kernel<0>, dim3(g), dim3(256), 0, s, state, age, nodes, count, lgR, replica, comp);
    else
        hipLaunchKernelGGL(seed_kernel<1>, dim3(g), dim3(256), 0, s, state, age, nodes, count, lgR, replica, comp);
    return hipGetLastError();
}

hipError_t launch_clear_u32(uint32_t* p, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    unsigned g = grid_for(n, 256);
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(clear_u32_kernel, dim3(g), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_set_ctl(Ctl* ctl, unsigned long long step, hipStream_t s)
{
    hipLaunchKernelGGL(set_ctl_kernel, dim3(1), dim3(64), 0, s, ctl, step);
    return hipGetLastError();
}

hipError_t launch_eval_hazard(const HazardDev& h, int32_t storage, const void* ages, float* out, int64_t n,
                              hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(eval_hazard_kernel, dim3(grid_for((size_t)n, 256)), dim3(256), 0, s, h, storage, ages,
                       out, n);
    return hipGetLastError();
}

hipError_t launch_eval_philox(const uint4* ctr, uint32_t k0, uint32_t k1, uint4* out, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(eval_philox_kernel, dim3(grid_for((size_t)n, 256)), dim3(256), 0, s, ctr, k0, k1, out, n);
    return hipGetLastError();
}

} // namespace fsk
