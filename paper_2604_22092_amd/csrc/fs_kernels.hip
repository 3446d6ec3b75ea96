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

__device__ __forceinline__ float age_units(float a) { return a; }
__device__ __forceinline__ float age_units(uint16_t a) { return (float)a; }
__device__ __forceinline__ float age_next(float a, float dt) { return a + dt; }
__device__ __forceinline__ uint16_t age_next(uint16_t a, float) { return a == 65535 ? a : (uint16_t)(a + 1); }

// Infectivity is held as one bit per unit (bit u = 1{X_u = I}); with constant
// shedding s = 1 this is the exact value of Eq. (infectivity) without beta.
__device__ __forceinline__ uint32_t bit_at(const uint32_t* __restrict__ w, uint32_t b)
{
    return (w[b >> 5] >> (b & 31)) & 1u;
}

// Pressure of one row (Eq. (influence) without beta): the sum over its edges
// of w_e * bit[col_e * R + rep].  Columns are fetched PB at a time with
// clamped, unconditional loads so one round trip covers a whole batch (the
// surplus lanes re-read the row's last entry and are masked out).  Unit
// weights count bits exactly in an integer.
constexpr int PB = 16;

template <bool WEIGHTED>
__device__ __forceinline__ float pressure(const int32_t* __restrict__ col_ind, const float* __restrict__ w,
                                          int32_t e0, int32_t e1, const uint32_t* __restrict__ bits,
                                          int32_t lgR, uint32_t rep)
{
    uint32_t pi = 0;
    float pw = 0.0f;
    for (int32_t base = e0; base < e1; base += PB) {
        int32_t c[PB];
        float wv[PB];
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            const int32_t idx = min(base + j, e1 - 1);
            c[j] = col_ind[idx];
            if (WEIGHTED) wv[j] = w[idx];
        }
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            const uint32_t b = (base + j < e1) ? bit_at(bits, ((uint32_t)c[j] << lgR) + rep) : 0u;
            if (WEIGHTED) pw = __builtin_fmaf(wv[j], (float)b, pw);
            else pi += b;
        }
    }
    return WEIGHTED ? pw : (float)pi;
}

// One fused step.  Units are processed in chunks of 64 (one wavefront, one
// 64-bit word of the next infectivity bitmap); every wavefront walks its own
// chunks with no workgroup barrier, so the memory latency of one wavefront
// overlaps the work of the others.
//  RESIDENT: the whole start-of-step bitmap (units <= RESIDENT_BITS) is copied
//    into LDS once per workgroup and every gather reads LDS; launched with one
//    workgroup of RESIDENT_TPB threads per compute unit.
//  otherwise: gathers read the bitmap through the caches.
template <int STORAGE, bool WEIGHTED, bool RATES, bool RESIDENT, int TPB>
__global__ __launch_bounds__(TPB) void step_kernel(StepArgs a)
{
    using S = Store<STORAGE>;
    using state_t = typename S::state_t;
    using age_t = typename S::age_t;
    constexpr int NW = TPB / 64;

    __shared__ uint32_t s_cnt[4 * 64];
    __shared__ uint32_t s_bits[RESIDENT ? RESIDENT_BITS / 32 : 1];

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63;
    const uint32_t R = 1u << a.lgR;
    const unsigned long long k = a.ctl->step + a.step_off;
    const uint32_t* __restrict__ bits_in = (const uint32_t*)((k & 1) ? a.iota1 : a.iota0);
    unsigned long long* __restrict__ bits_out = (unsigned long long*)((k & 1) ? a.iota0 : a.iota1);
    state_t* __restrict__ state = (state_t*)a.state;
    age_t* __restrict__ age = (age_t*)a.age;
    const uint32_t total = (uint32_t)a.n << a.lgR;
    const uint32_t nchunks = (total + 63) >> 6;

    if (R > 1)
        for (uint32_t i = tid; i < 4 * R; i += TPB) s_cnt[i] = 0;
    if (RESIDENT) {
        const uint32_t words = (total + 31) >> 5;
        const uint4* src = (const uint4*)bits_in;
        uint4* dst = (uint4*)s_bits;
        for (uint32_t i = tid; i < (words + 3) >> 2; i += TPB) dst[i] = src[i];
    }
    if (R > 1 || RESIDENT) __syncthreads();
    const uint32_t* __restrict__ gbits = RESIDENT ? s_bits : bits_in;

    uint32_t c0 = 0, c1 = 0, c2 = 0, c3 = 0; // per-wave counts (R == 1)

    for (uint32_t chunk = blockIdx.x * NW + (tid >> 6); chunk < nchunks; chunk += gridDim.x * NW) {
        const uint32_t unit = (chunk << 6) + lane;
        const bool valid = unit < total;
        const uint32_t node = unit >> a.lgR;
        const uint32_t rep = unit & (R - 1);

        int x = ST_R;
        age_t ag = 0;
        int32_t e0 = 0, e1 = 0;
        if (valid) {
            x = (int)state[unit];
            ag = age[unit];
            e0 = a.row_ptr[node];
            e1 = a.row_ptr[node + 1];
        }

        // 1.-2. rate: beta * pressure for S; hazard at the start-of-step age for E/I; 0 for R
        float lam = 0.0f;
        if (x == ST_S) lam = a.beta * pressure<WEIGHTED>(a.col_ind, a.weights, e0, e1, gbits, a.lgR, rep);
        if (a.same_kind) {
            if (x == ST_E || x == ST_I) {
                HazardDev h = a.hz[0];
                if (x == ST_I) h = a.hz[1];
                h.kind = a.hz[0].kind;
                lam = fsd::hazard(h, age_units(ag));
            }
        } else {
            if (x == ST_E) lam = fsd::hazard(a.hz[0], age_units(ag));
            if (x == ST_I) lam = fsd::hazard(a.hz[1], age_units(ag));
        }

        // 3.-4. Bernoulli tau-leap: fire when u < 1 - exp(-lambda dt); no draw at lambda = 0
        bool fire = false;
        if (lam > 0.0f) {
            const float u = fsd::step_uniform(node, (uint32_t)k, rep, a.key0, a.key1);
            const float q = -expm1f(-lam * a.dt);
            fire = u < q;
        }

        // 5.-6. advance state and age in place
        const int xn = x + (fire ? 1 : 0);
        if (valid) {
            if (fire) state[unit] = (state_t)xn;
            age[unit] = fire ? (age_t)0 : age_next(ag, a.dt);
            if (RATES) a.rates[unit] = lam;
        }

        // 7. next-step infectivity bits (one 64-bit word per chunk) and 8. counts
        const unsigned long long mI = __ballot(valid && xn == ST_I);
        if (lane == 0) bits_out[chunk] = mI;
        if (R == 1) {
            c0 += (uint32_t)__popcll(__ballot(valid && xn == ST_S));
            c1 += (uint32_t)__popcll(__ballot(valid && xn == ST_E));
            c2 += (uint32_t)__popcll(mI);
            c3 += (uint32_t)__popcll(__ballot(valid && xn == ST_R));
        } else if (valid) {
            atomicAdd(&s_cnt[rep * 4 + xn], 1u); // LDS
        }
    }

    // one plain store of this workgroup's counts; the reduce kernel sums them
    uint32_t* out = a.part + ((size_t)a.step_off * gridDim.x + blockIdx.x) * (4 * R);
    if (R == 1) {
        if (lane == 0) {
            const uint32_t w = tid >> 6;
            s_cnt[w * 4 + 0] = c0;
            s_cnt[w * 4 + 1] = c1;
            s_cnt[w * 4 + 2] = c2;
            s_cnt[w * 4 + 3] = c3;
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
}

// Sums per-workgroup count partials.  Block j handles slot j: rows of C
// counters from G workgroups, part[j][g][c]; the totals go to
// out[((base + j) mod H)][c] where base = ctl->step (0 without ctl).
// Requires C <= WG and WG % C == 0 (C = 4R with R a power of two <= 64).
__global__ __launch_bounds__(WG) void reduce_kernel(const Ctl* ctl, const uint32_t* part, uint32_t G,
                                                     uint32_t C, uint32_t* out, uint32_t H)
{
    __shared__ uint32_t s[WG];
    const uint32_t t = threadIdx.x;
    const uint32_t j = blockIdx.x;
    // of a sequence longer than the ring only the last H steps are kept, so
    // no two blocks write one slot
    if ((size_t)j + H < (size_t)gridDim.x) return;
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

__global__ void advance_kernel(Ctl* ctl, uint32_t r)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->step = ctl->step + r;
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
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->step = step;
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

const void* step_kernel_fn(int storage, bool weighted, bool rates, bool resident)
{
#define FS_SEL(S, W, RT)                                                                         \
    if (storage == S && weighted == W && rates == RT)                                            \
        return resident ? (const void*)&step_kernel<S, W, RT, true, RESIDENT_TPB>                \
                        : (const void*)&step_kernel<S, W, RT, false, STREAM_TPB>;
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
const void* advance_kernel_fn() { return (const void*)&advance_kernel; }

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
