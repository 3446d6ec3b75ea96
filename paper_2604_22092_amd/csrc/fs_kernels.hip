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

#include "fs_step.hpp"

namespace fsk {

// Sums per-workgroup count partials.  Block j handles slot j: rows of C
// counters from G workgroups, part[j][g][c]; the totals go to
// out[((base + j) mod H)][c] where base = ctl->step (0 without ctl).
// Requires C <= RED_TPB and RED_TPB % C == 0 (C = 4R with R a power of two
// <= 64).  Each thread keeps eight independent sums of the rows it reads (so
// eight loads are in flight), and the block's sums are folded by a tree in
// LDS (integer sums: the order does not change them).
// With a ctl, the r blocks of the launch end the launch sequence: each takes
// a ticket in ctl->done once its reads of ctl->step are done, and the last
// one adds r to ctl->step and clears the count (so the sequence needs no
// launch of its own for the advance).
__device__ __forceinline__ void reduce_body(Ctl* ctl, const uint32_t* part, uint32_t G, uint32_t C,
                                            uint32_t* out, uint32_t H, uint32_t j, uint32_t r)
{
    __shared__ uint32_t s[RED_TPB];
    const uint32_t t = threadIdx.x;
    // of a sequence longer than the ring only the last H steps are kept, so
    // no two blocks write one slot
    if ((size_t)j + H >= (size_t)r) {
        const uint32_t groups = RED_TPB / C;
        const uint32_t c = t % C;
        const uint32_t* p = part + (size_t)j * G * C + c;
        uint32_t acc[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
        uint32_t g = t / C;
        for (; g + 7u * groups < G; g += 8u * groups) {
#pragma unroll
            for (int i = 0; i < 8; ++i) acc[i] += p[(size_t)(g + (uint32_t)i * groups) * C];
        }
        for (; g < G; g += groups) acc[0] += p[(size_t)g * C];
        s[t] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
        __syncthreads();
        // (w is a multiple of C, so s[t] and s[t + w] hold the same counter)
        for (uint32_t w = RED_TPB / 2; w >= C; w >>= 1) {
            if (t < w) s[t] += s[t + w];
            __syncthreads();
        }
        if (t < C) {
            const unsigned long long base = ctl ? ctl->step : 0ull;
            out[(size_t)((base + j) % H) * C + t] = s[t];
        }
    }
    if (ctl) {
        __syncthreads();
        if (t == 0) {
            const uint32_t prior = __hip_atomic_fetch_add(&ctl->done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (prior + 1u == r) {
                __hip_atomic_store(&ctl->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&ctl->step, ctl->step + r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

__global__ __launch_bounds__(RED_TPB) void reduce_kernel(Ctl* ctl, const uint32_t* part, uint32_t G,
                                                     uint32_t C, uint32_t* out, uint32_t H)
{
    reduce_body(ctl, part, G, C, out, H, blockIdx.x, gridDim.x);
}

// Batched reduce: block (j, m) sums slot j of member m (grid r x members).
__global__ __launch_bounds__(RED_TPB) void reduce_batch_kernel(const RedArgs* __restrict__ table)
{
    const RedArgs q = table[blockIdx.y];
    reduce_body(q.ctl, q.part, q.G, q.C, q.hist, q.H, blockIdx.x, gridDim.x);
}

// Summary of an infectivity bitmap: bit s is set when any of the 32 w units
// of group s is infectious, i.e. when one of its w = 2^sum_shift 32-bit
// bitmap words is nonzero.  One thread per summary bit, one summary word per
// wave.
__global__ __launch_bounds__(WG) void summary_kernel(SumArgs q)
{
    const unsigned long long k = q.ctl->step + q.step_off + q.after;
    const uint32_t* __restrict__ bits = (const uint32_t*)((k & 1) ? q.iota1 : q.iota0);
    const uint32_t s = blockIdx.x * WG + threadIdx.x;
    const uint32_t gw = 1u << q.sum_shift;
    const uint64_t w0 = (uint64_t)s * gw, nw = 2ull * q.words;
    bool any = false;
    for (uint32_t i = 0; i < gw; ++i)
        if (w0 + i < nw && bits[w0 + i] != 0u) any = true;
    const unsigned long long m = __ballot(any);
    if ((threadIdx.x & 63) == 0 && (s >> 6) < q.sum_words) q.summary[s >> 6] = m;
}

// Pushed pressure of the binned rows recounted from a bitmap (after a change
// of states from the host): out[h] for hub unit h = (row - hub_base) * R + r
// is the number of infectious in-neighbours of the row in replica r, counted
// with multiplicity.  One wavefront per row: lane l takes edge offset l / R
// and replica l % R, and each edge pass's bits are counted per replica by a
// ballot, as the heavy-row kernels count integer partials.
__global__ __launch_bounds__(WG) void hub_recount_kernel(const int32_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col_ind, int32_t hub_base,
                                                         uint32_t hubs, int32_t lgR,
                                                         const uint32_t* __restrict__ bits,
                                                         uint32_t* __restrict__ out)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t R = 1u << lgR;
    const uint32_t per = 64u >> lgR;
    const uint32_t eoff = lane >> lgR;
    const uint32_t rep = lane & (R - 1);
    unsigned long long rmask = 1ull; // lanes of replica 0: every R-th lane
    for (uint32_t sh = R; sh < 64u; sh <<= 1) rmask |= rmask << sh;
    const uint32_t nw = gridDim.x * (WG / 64);
    for (uint32_t h = blockIdx.x * (WG / 64) + (threadIdx.x >> 6); h < hubs; h += nw) {
        const int32_t row = hub_base + (int32_t)h;
        const int32_t e1 = row_ptr[row + 1];
        uint32_t c = 0;
        for (int32_t e = row_ptr[row] + (int32_t)eoff;; e += (int32_t)per) {
            const bool in = e < e1;
            if (__ballot(in) == 0ull) break;
            const uint32_t b = in ? bit_at(bits, ((uint32_t)col_ind[e] << lgR) + rep) : 0u;
            c += (uint32_t)__popcll(__ballot(b != 0u) & (rmask << rep));
        }
        if (lane < R) out[(size_t)h * R + lane] = c;
    }
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

// Evaluates the shedding profile at n ages (checks of the device arithmetic).
__global__ void eval_shed_kernel(ShedDev sd, int32_t storage, const void* ages, float* out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = storage == 0 ? ((const float*)ages)[i] : (float)((const uint16_t*)ages)[i];
    out[i] = fsd::shed(sd, x);
}

// Shedding values s(tau) of every infectious unit from the state and age
// (after seeding or a state load); other units are left as they are.
template <int STORAGE>
__global__ void rebuild_shed_kernel(const void* state_v, const void* age_v, uint32_t total, ShedDev sd, void* out)
{
    using S = Store<STORAGE>;
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= total) return;
    if ((int)((const typename S::state_t*)state_v)[u] != ST_I) return;
    const float v = fsd::shed(sd, age_units(((const typename S::age_t*)age_v)[u]));
    if (STORAGE == 0) ((float*)out)[u] = v;
    else ((uint16_t*)out)[u] = (uint16_t)float_to_half_bits(v);
}

// Live flags of every chunk from the state: 1 when the chunk holds a unit
// that is not R.  One wavefront per chunk.
template <int STORAGE>
__global__ __launch_bounds__(WG) void chunk_live_kernel(const void* state_v, uint32_t total, uint8_t* live,
                                                        uint32_t nchunks)
{
    using state_t = typename Store<STORAGE>::state_t;
    const uint32_t unit = blockIdx.x * WG + threadIdx.x;
    const int x = unit < total ? (int)((const state_t*)state_v)[unit] : ST_R;
    const bool alive = __ballot(x != ST_R) != 0ull;
    const uint32_t c = unit >> 6;
    if ((threadIdx.x & 63) == 0 && c < nchunks) live[c] = alive ? 1 : 0;
}

// Active-chunk list from the live flags (one workgroup of WG_REFRESH threads):
// act[2 ..] = the chunks whose flag is set, ascending; act[0] = their number;
// act[1] = the nodes of the other chunks (all their units are R, in every
// replica).  Each thread takes 16 consecutive flags per tile; `live` is
// padded with zeros to whole tiles.  rows = nodes per chunk.
__global__ __launch_bounds__(WG_REFRESH) void compact_refresh_kernel(const uint8_t* __restrict__ live,
                                                                     uint32_t nchunks, uint32_t rows, uint32_t n,
                                                                     uint32_t* __restrict__ act)
{
    constexpr uint32_t NWR = WG_REFRESH / 64;
    __shared__ uint32_t s_wave[NWR];
    __shared__ uint32_t s_nodes[NWR];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    uint32_t base = 0, nodes = 0;
    for (uint32_t c0 = 0; c0 < nchunks; c0 += 16 * WG_REFRESH) {
        const uint32_t cf = c0 + 16 * tid;
        const uint4 w = *(const uint4*)(live + cf); // within the padded tile
        const uint32_t words[4] = {w.x, w.y, w.z, w.w};
        uint32_t mask = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const bool f = ((words[i >> 2] >> (8 * (i & 3))) & 0xFFu) != 0u && cf + i < nchunks;
            mask |= (f ? 1u : 0u) << i;
        }
        const uint32_t cnt = __popc(mask);
        // inclusive scan of the counts over the wave, then over the waves
        uint32_t inc = cnt;
        for (uint32_t off = 1; off < 64; off <<= 1) {
            const uint32_t v = __shfl_up(inc, off, 64);
            if (lane >= off) inc += v;
        }
        if (lane == 63) s_wave[wave] = inc;
        __syncthreads();
        uint32_t before = 0, tile = 0;
        for (uint32_t v = 0; v < NWR; ++v) {
            before += v < wave ? s_wave[v] : 0u;
            tile += s_wave[v];
        }
        uint32_t pos = base + before + inc - cnt;
        for (int i = 0; i < 16; ++i) {
            if ((mask >> i) & 1u) {
                const uint32_t c = cf + (uint32_t)i;
                act[2 + pos++] = c;
                nodes += min(rows, n - c * rows);
            }
        }
        base += tile;
        __syncthreads();
    }
    for (int off = 32; off > 0; off >>= 1) nodes += __shfl_xor(nodes, off, 64);
    if (lane == 0) s_nodes[wave] = nodes;
    __syncthreads();
    if (tid == 0) {
        uint32_t t = 0;
        for (uint32_t v = 0; v < NWR; ++v) t += s_nodes[v];
        act[0] = base;
        act[1] = n - t;
    }
}

// ---------------------------------------------------------------- launchers

const void* step_kernel_fn(int storage, bool weighted, int mode, int udeg, bool shed, bool extra, int lgR,
                           int pbits)
{
    if (pbits != 0) {
        if (weighted || lgR != 0 || (shed && extra)) return nullptr;
        if (pbits == 20)
            return shed ? step_kernel_fn_shed_r1p20(storage, mode, udeg)
                        : extra ? step_kernel_fn_extra_r1p20(storage, mode, udeg) : step_kernel_fn_r1p20(storage, mode, udeg);
        if (pbits == 24)
            return shed ? step_kernel_fn_shed_r1p24(storage, mode, udeg)
                        : extra ? step_kernel_fn_extra_r1p24(storage, mode, udeg) : step_kernel_fn_r1p24(storage, mode, udeg);
        if (pbits == 27)
            return shed ? step_kernel_fn_shed_r1p27(storage, mode, udeg)
                        : extra ? step_kernel_fn_extra_r1p27(storage, mode, udeg) : step_kernel_fn_r1p27(storage, mode, udeg);
        return nullptr;
    }
    if (!shed && !extra && lgR == 0) return step_kernel_fn_r1(storage, weighted, mode, udeg);
    if (!shed && !extra && !weighted && lgR == 4) return step_kernel_fn_r16(storage, mode, udeg);
    if (shed) return extra ? step_kernel_fn_shed_extra(storage, weighted, mode, udeg)
                           : step_kernel_fn_shed(storage, weighted, mode, udeg);
    if (extra) return step_kernel_fn_extra(storage, weighted, mode, udeg);
    return step_kernel_pick<false, false>(storage, weighted, mode, udeg);
}

static unsigned grid_for(size_t n, unsigned block) { return (unsigned)((n + block - 1) / block); }

hipError_t launch_hub_recount(const int32_t* row_ptr, const int32_t* col_ind, int32_t hub_base, uint32_t hubs,
                              int32_t lgR, const uint32_t* bits, uint32_t* out, hipStream_t s)
{
    if (hubs == 0) return hipSuccess;
    unsigned g = grid_for((size_t)hubs, WG / 64);
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(hub_recount_kernel, dim3(g), dim3(WG), 0, s, row_ptr, col_ind, hub_base, hubs, lgR, bits,
                       out);
    return hipGetLastError();
}

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
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(RED_TPB), 0, s, (Ctl*)nullptr, (const uint32_t*)part,
                       (uint32_t)g, 4u, out4, 1u);
    return hipGetLastError();
}

const void* reduce_kernel_fn() { return (const void*)&reduce_kernel; }
const void* heavy_kernel_fn(bool weighted, bool shed, bool resident)
{
    if (shed) return heavy_kernel_fn_shed(weighted, resident);
    if (resident)
        return weighted ? (const void*)&heavy_resident_kernel<true, false> : (const void*)&heavy_resident_kernel<false, false>;
    return weighted ? (const void*)&heavy_pressure_kernel<true, false> : (const void*)&heavy_pressure_kernel<false, false>;
}
const void* summary_kernel_fn() { return (const void*)&summary_kernel; }

const void* step_batch_kernel_fn(int storage, bool weighted, bool extra)
{
    if (extra) {
        if (storage == 0)
            return weighted ? (const void*)&step_batch_kernel<0, true, true> : (const void*)&step_batch_kernel<0, false, true>;
        return weighted ? (const void*)&step_batch_kernel<1, true, true> : (const void*)&step_batch_kernel<1, false, true>;
    }
    if (storage == 0)
        return weighted ? (const void*)&step_batch_kernel<0, true, false> : (const void*)&step_batch_kernel<0, false, false>;
    return weighted ? (const void*)&step_batch_kernel<1, true, false> : (const void*)&step_batch_kernel<1, false, false>;
}
const void* heavy_batch_kernel_fn(bool weighted)
{
    return weighted ? (const void*)&heavy_batch_kernel<true> : (const void*)&heavy_batch_kernel<false>;
}
const void* reduce_batch_kernel_fn() { return (const void*)&reduce_batch_kernel; }

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

// Hazard table of a fixed-step sim (StepArgs::htab): entry m holds the age
// a_m (written by the host) and receives the hazards of both laws at a_m,
// evaluated by the step's own code.
__global__ void hazard_table_kernel(const HazardDev* hz, int32_t same_kind, float4* tab, uint32_t n)
{
    const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const float x = tab[m].x;
    tab[m].y = unit_hazard(hz, same_kind, x, false);
    tab[m].z = unit_hazard(hz, same_kind, x, true);
    tab[m].w = 0.0f;
}

hipError_t launch_hazard_table(const HazardDev* hz, int32_t same_kind, float4* tab, uint32_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(hazard_table_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, hz, same_kind, tab, n);
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

hipError_t launch_eval_shed(const ShedDev& sd, int32_t storage, const void* ages, float* out, int64_t n,
                            hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(eval_shed_kernel, dim3(grid_for((size_t)n, 256)), dim3(256), 0, s, sd, storage, ages, out, n);
    return hipGetLastError();
}

hipError_t launch_rebuild_shed(int storage, const void* state, const void* age, uint32_t total, const ShedDev& sd,
                               void* out, hipStream_t s)
{
    if (total == 0) return hipSuccess;
    const unsigned g = grid_for(total, 256);
    if (storage == 0)
        hipLaunchKernelGGL(rebuild_shed_kernel<0>, dim3(g), dim3(256), 0, s, state, age, total, sd, out);
    else
        hipLaunchKernelGGL(rebuild_shed_kernel<1>, dim3(g), dim3(256), 0, s, state, age, total, sd, out);
    return hipGetLastError();
}

hipError_t launch_chunk_live(int storage, const void* state, uint32_t total, uint8_t* live, uint32_t nchunks,
                             hipStream_t s)
{
    const unsigned g = grid_for((size_t)nchunks * 64, WG);
    if (g == 0) return hipSuccess;
    if (storage == 0)
        hipLaunchKernelGGL(chunk_live_kernel<0>, dim3(g), dim3(WG), 0, s, state, total, live, nchunks);
    else
        hipLaunchKernelGGL(chunk_live_kernel<1>, dim3(g), dim3(WG), 0, s, state, total, live, nchunks);
    return hipGetLastError();
}

const void* compact_refresh_kernel_fn() { return (const void*)&compact_refresh_kernel; }
const void* clear_u32_kernel_fn() { return (const void*)&clear_u32_kernel; }

hipError_t launch_eval_philox(const uint4* ctr, uint32_t k0, uint32_t k1, uint4* out, int64_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(eval_philox_kernel, dim3(grid_for((size_t)n, 256)), dim3(256), 0, s, ctr, k0, k1, out, n);
    return hipGetLastError();
}

} // namespace fsk
