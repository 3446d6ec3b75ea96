// The Markovian engine (FlashSpread, arXiv 2604.22092, Section "Markovian
// engine", Algorithm "Markovian Engine: One Tau-Leaping Step") for gfx950.
//
// Rates are piecewise constant: S nodes beta * I_i (I_i: infectious
// in-neighbours, unit weights), E nodes sigma, I nodes gamma, R nodes 0.
// One step is three launches, all inside a captured graph:
//   draw   (dense): one wavefront per workgroup folds the per-workgroup rate
//          partials of the previous launch into Lambda and max lambda (exact integers),
//          takes tau = min(theta N / Lambda, p_max / max lambda, tau_max),
//          draws every node with a positive rate and applies the transitions;
//          a node whose infectiousness changed is appended to its
//          workgroup's event region (no global counter);
//   push   (sparse, Inertial Mode): when the step's events are few, each
//          event adds +-1 to the influence of its out-neighbours (integer
//          atomics on the outgoing CSR: exact and order-independent), the
//          events spread over every lane of the grid; otherwise it exits.
//          Without I -> S (SEIR, SIR) only susceptible targets are updated:
//          no other node reads its influence again;
//   rates  (dense): when the events were many (Control Mode) it recounts
//          every influence from the incoming CSR, then writes per-workgroup
//          (sum of S influences, max S influence, #E, #I) for the next draw;
//          after a step without transitions it keeps the old partials.
// Both modes give the same integer influences on every node that can still
// read them (every susceptible node; every node under SIS), so results do not
// depend on which ran.  Per-step counts, tau and event totals go to rings on the
// device; a launch sequence ends with the count reduce, which also advances
// the step index.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fs_device.hpp"
#include "fs_runtime.hpp"

namespace fsm {

using namespace fsi;

constexpr int MTPB = 1024; // threads per workgroup of the dense kernels
constexpr int PTPB = 256;  // threads per workgroup of the push kernel
constexpr uint32_t EV_LEAVE = 0x80000000u;

struct MkArgs {
    uint8_t* state;
    int32_t* infl;
    const int32_t* row_ptr; // incoming CSR (internal order)
    const int32_t* col_ind;
    const int32_t* out_ptr; // outgoing CSR (internal order)
    const int32_t* out_ind;
    const int32_t* orig_id; // caller's id of each node: the draws are keyed by it
    uint32_t* events;       // [G][span]: node | EV_LEAVE when it stopped being infectious
    uint32_t* ev_cnt;       // [G] events of the current step per region
    uint32_t* fired;        // [G] transitions of the current step per region (events or not);
                            // fired[G] receives their total (written by the push launch)
    uint4* rpart;           // [G]: (sum of S influences, max S influence, #E, #I)
    uint32_t* part;         // count partials [slot][G][4]
    float* tau_hist;        // [H]
    uint32_t* ev_hist;      // [H]
    double* elapsed;        // one value: the simulated time
    const Ctl* ctl;
    uint32_t n, G, span, H;
    uint32_t step_off;
    int32_t model;          // FS_MARKOV_*
    float beta, sigma, gamma;
    double theta, p_max, tau_max;
    uint32_t key0, key1;
    uint32_t inertial_max;  // events per step up to which pushes update the influence
    int32_t force_control;  // rates launch after a state change: recount everything
};

__device__ __forceinline__ int next_state(int model, int x)
{
    if (x == ST_S) return model == FS_MARKOV_SEIR ? ST_E : ST_I;
    if (x == ST_E) return ST_I;
    if (x == ST_I) return model == FS_MARKOV_SIS ? ST_S : ST_R;
    return x;
}

// tau of Algorithm "Markovian Engine" from the per-workgroup partials of the
// rates launch (every wave folds them in the same order, so every wave gets
// the same value).
__device__ double markov_tau(const MkArgs& a, uint32_t lane)
{
    unsigned long long A = 0, nE = 0, nI = 0;
    uint32_t M = 0;
    for (uint32_t g = lane; g < a.G; g += 64) {
        const uint4 v = a.rpart[g];
        A += v.x;
        M = max(M, v.y);
        nE += v.z;
        nI += v.w;
    }
    for (int off = 32; off > 0; off >>= 1) {
        A += __shfl_xor(A, off, 64);
        M = max(M, (uint32_t)__shfl_xor((int)M, off, 64));
        nE += __shfl_xor(nE, off, 64);
        nI += __shfl_xor(nI, off, 64);
    }
    const double L = (double)a.beta * (double)A + (double)a.sigma * (double)nE + (double)a.gamma * (double)nI;
    double mx = (double)a.beta * (double)M;
    if (nE > 0) mx = fmax(mx, (double)a.sigma);
    if (nI > 0) mx = fmax(mx, (double)a.gamma);
    double tau = a.tau_max;
    if (L > 0.0) tau = fmin(tau, a.theta * (double)a.n / L);
    if (mx > 0.0) tau = fmin(tau, a.p_max / mx);
    return tau;
}

__global__ __launch_bounds__(MTPB) void mk_draw_kernel(MkArgs a)
{
    constexpr int NW = MTPB / 64;
    __shared__ uint32_t s_ev, s_fired;
    __shared__ uint32_t s_cnt[NW][4];
    __shared__ double s_tau;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long k = a.ctl->step + a.step_off;
    // one wave per workgroup folds the rate partials
    if (wave == 0) {
        const double t = markov_tau(a, lane);
        if (lane == 0) {
            s_tau = t;
            s_ev = 0;
            s_fired = 0;
        }
    }
    __syncthreads();
    const double tau = s_tau;
    const float tf = (float)tau;
    const uint32_t base = blockIdx.x * a.span;
    const uint32_t end = min(a.n, base + a.span);
    uint32_t c[4] = {0, 0, 0, 0};
    uint32_t nfire = 0;
    for (uint32_t i0 = base + wave * 64; i0 < end; i0 += MTPB) {
        const uint32_t i = i0 + lane;
        const bool valid = i < end;
        const int x = valid ? (int)a.state[i] : ST_R;
        const int f = x == ST_S ? a.infl[i] : 0;
        const float lam = x == ST_S ? a.beta * (float)f : x == ST_E ? a.sigma : x == ST_I ? a.gamma : 0.0f;
        bool fire = false;
        if (lam > 0.0f) {
            const uint4 w = fsd::philox4x32_10(make_uint4((uint32_t)a.orig_id[i], (uint32_t)k, 0u, 0u), a.key0, a.key1);
            const float u = (float)(w.x >> 8) * 0x1p-24f;
            fire = u < -expm1f(-lam * tf);
        }
        const int xn = fire ? next_state(a.model, x) : x;
        if (fire) a.state[i] = (uint8_t)xn;
        nfire += (uint32_t)__popcll(__ballot(fire));
        // a change of infectiousness is an event of this workgroup's region
        const bool ev = fire && ((xn == ST_I) != (x == ST_I));
        const unsigned long long m = __ballot(ev);
        if (m) {
            uint32_t pos = 0;
            if (lane == 0) pos = atomicAdd(&s_ev, (uint32_t)__popcll(m)); // LDS
            pos = __shfl(pos, 0, 64);
            if (ev) a.events[base + pos + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = i | (x == ST_I ? EV_LEAVE : 0u);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] += (uint32_t)__popcll(__ballot(valid && xn == q));
    }
    if (lane == 0) {
        for (int q = 0; q < 4; ++q) s_cnt[wave][q] = c[q];
        atomicAdd(&s_fired, nfire); // LDS
    }
    __syncthreads();
    if (tid < 4) {
        uint32_t t = 0;
        for (int w = 0; w < NW; ++w) t += s_cnt[w][tid];
        a.part[((size_t)a.step_off * a.G + blockIdx.x) * 4 + tid] = t;
    }
    if (tid == 0) {
        a.ev_cnt[blockIdx.x] = s_ev;
        a.fired[blockIdx.x] = s_fired;
        if (blockIdx.x == 0) {
            a.tau_hist[k % a.H] = tf;
            *a.elapsed += tau;
        }
    }
}

// Inertial Mode.  The events of all regions, taken in region order, are
// spread over every lane of the grid: each workgroup builds the exclusive
// prefix of the region counts in LDS and each lane finds the region of its
// event by binary search, then pushes +-1 to the event's out-neighbours
// (non-returning integer atomics).
constexpr uint32_t MAX_REGIONS = 1024;

__global__ __launch_bounds__(PTPB) void mk_push_kernel(MkArgs a)
{
    __shared__ uint32_t s_pre[MAX_REGIONS + 1];
    __shared__ uint32_t s_fire[PTPB / 64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long k = a.ctl->step + a.step_off;
    // region counts into LDS (all threads), transitions summed per wave
    uint32_t f = 0;
    for (uint32_t g = tid; g < a.G; g += PTPB) {
        s_pre[g] = a.ev_cnt[g];
        f += a.fired[g];
    }
    for (int off = 32; off > 0; off >>= 1) f += __shfl_xor(f, off, 64);
    if (lane == 0) s_fire[wave] = f;
    __syncthreads();
    // exclusive prefix of the counts by wave 0: lane l scans its block of
    // ceil(G / 64) regions, then the block sums are scanned across lanes
    if (wave == 0) {
        const uint32_t per = (a.G + 63) / 64;
        const uint32_t g0 = lane * per, g1 = min(a.G, g0 + per);
        uint32_t sum = 0;
        for (uint32_t g = g0; g < g1; ++g) sum += s_pre[g];
        uint32_t inc = sum;
        for (uint32_t off = 1; off < 64; off <<= 1) {
            const uint32_t v = __shfl_up(inc, off, 64);
            if (lane >= off) inc += v;
        }
        uint32_t run = inc - sum;
        for (uint32_t g = g0; g < g1; ++g) {
            const uint32_t c = s_pre[g];
            s_pre[g] = run;
            run += c;
        }
        if (lane == 63) s_pre[a.G] = inc;
    }
    __syncthreads();
    if (blockIdx.x == 0 && tid == 0) {
        a.ev_hist[k % a.H] = s_pre[a.G];
        uint32_t t = 0;
        for (int w = 0; w < PTPB / 64; ++w) t += s_fire[w];
        a.fired[a.G] = t;
    }
    const uint32_t total = s_pre[a.G];
    if (total > a.inertial_max) return;
    const int32_t* __restrict__ out_ind = a.out_ind;
    const uint8_t* __restrict__ state = a.state;
    for (uint32_t j = blockIdx.x * PTPB + tid; j < total; j += gridDim.x * PTPB) {
        uint32_t lo = 0, hi = a.G; // s_pre[lo] <= j < s_pre[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_pre[mid] <= j) lo = mid;
            else hi = mid;
        }
        const uint32_t e = a.events[(size_t)lo * a.span + (j - s_pre[lo])];
        const uint32_t node = e & ~EV_LEAVE;
        const int d = (e & EV_LEAVE) ? -1 : 1;
        // without I -> S, a node that is not susceptible never reads its
        // influence again: only susceptible targets are updated.  Targets go
        // eight at a time: their ids, then their states, then the atomics,
        // so a lane waits for two loads per eight targets, not per target.
        const bool all = a.model == FS_MARKOV_SIS;
        const int32_t t1 = a.out_ptr[node + 1];
        for (int32_t t = a.out_ptr[node]; t < t1; t += 8) {
            int32_t tg[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) tg[q] = t + q < t1 ? out_ind[t + q] : -1;
            bool go[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) go[q] = tg[q] >= 0 && (all || state[tg[q]] == ST_S);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (go[q]) atomicAdd(&a.infl[tg[q]], d);
        }
    }
}

// Control Mode recount (when the step's events were many, or after a state
// change) and the rate partials of the current state.
__global__ __launch_bounds__(MTPB) void mk_rates_kernel(MkArgs a)
{
    constexpr int NW = MTPB / 64;
    __shared__ uint4 s_p[NW];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned long long k = a.ctl->step + a.step_off;
    const uint32_t events = a.ev_hist[k % a.H];
    // a step without transitions changed nothing: the partials still hold
    if (!a.force_control && a.fired[a.G] == 0) return;
    const bool control = a.force_control || events > a.inertial_max;
    const uint32_t base = blockIdx.x * a.span;
    const uint32_t end = min(a.n, base + a.span);
    uint32_t A = 0, M = 0, nE = 0, nI = 0;
    for (uint32_t i0 = base + wave * 64; i0 < end; i0 += MTPB) {
        const uint32_t i = i0 + lane;
        const bool valid = i < end;
        const int x = valid ? (int)a.state[i] : ST_R;
        int f = 0;
        if (valid) {
            if (control) {
                for (int32_t e = a.row_ptr[i]; e < a.row_ptr[i + 1]; ++e) f += a.state[a.col_ind[e]] == ST_I;
                a.infl[i] = f;
            } else if (x == ST_S) {
                f = a.infl[i];
            }
        }
        if (x == ST_S) {
            A += (uint32_t)f;
            M = max(M, (uint32_t)f);
        }
        nE += x == ST_E;
        nI += x == ST_I;
    }
    for (int off = 32; off > 0; off >>= 1) {
        A += __shfl_xor(A, off, 64);
        M = max(M, (uint32_t)__shfl_xor((int)M, off, 64));
        nE += __shfl_xor(nE, off, 64);
        nI += __shfl_xor(nI, off, 64);
    }
    if (lane == 0) s_p[wave] = make_uint4(A, M, nE, nI);
    __syncthreads();
    if (tid == 0) {
        uint4 t = make_uint4(0, 0, 0, 0);
        for (int w = 0; w < NW; ++w) {
            t.x += s_p[w].x;
            t.y = max(t.y, s_p[w].y);
            t.z += s_p[w].z;
            t.w += s_p[w].w;
        }
        a.rpart[blockIdx.x] = t;
    }
}

__global__ void mk_seed_kernel(uint8_t* state, const int64_t* nodes, int64_t count, int32_t comp)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < count) state[nodes[j]] = (uint8_t)comp;
}

__global__ void mk_put_kernel(uint8_t* state, const int32_t* src, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) state[i] = (uint8_t)src[i];
}

__global__ void mk_clear_kernel(double* elapsed, double value)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *elapsed = value;
}

} // namespace fsm

using namespace fsr;
using fsm::MkArgs;

struct fs_markov {
    fs_graph* g = nullptr;
    fs_markov_params p{};
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint8_t* d_state = nullptr;
    int32_t* d_infl = nullptr;
    uint32_t* d_events = nullptr;
    uint32_t* d_ev_cnt = nullptr;
    uint32_t* d_fired = nullptr;
    uint4* d_rpart = nullptr;
    uint32_t* d_part = nullptr;
    uint32_t* d_hist = nullptr;
    float* d_tau = nullptr;
    uint32_t* d_evh = nullptr;
    double* d_elapsed = nullptr;
    fsi::Ctl* d_ctl = nullptr;
    uint32_t G = 0, span = 0, H = 1024, chunk = 64;
    int64_t step = 0, hist_from = 0;
    MkArgs args{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

// The outgoing CSR of a graph's internal order, built on first use and kept
// with the graph (the transpose of its incoming rows).
fs_status ensure_out_csr(fs_graph* g)
{
    std::lock_guard<std::mutex> lk(g->layout_mu);
    if (g->d_out_ptr) return FS_OK;
    const int64_t n = g->n;
    std::vector<int32_t> ptr((size_t)n + 1, 0), ind((size_t)g->nnz);
    for (int64_t e = 0; e < g->nnz; ++e) ptr[(size_t)g->h_col_ind[(size_t)e] + 1] += 1;
    for (int64_t j = 0; j < n; ++j) ptr[(size_t)j + 1] += ptr[(size_t)j];
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        for (int32_t e = g->h_row_ptr[(size_t)i]; e < g->h_row_ptr[(size_t)i + 1]; ++e)
            ind[(size_t)fill[(size_t)g->h_col_ind[(size_t)e]]++] = (int32_t)i;
    int32_t *dp = nullptr, *di = nullptr;
    hipError_t e;
    if ((e = dev_alloc((void**)&dp, ptr.size() * 4)) != hipSuccess ||
        (e = dev_alloc((void**)&di, std::max<size_t>(ind.size(), 1) * 4)) != hipSuccess) {
        dev_free(dp);
        return fail(FS_ERR_OUT_OF_MEMORY, std::string("outgoing CSR: ") + hipGetErrorString(e));
    }
    if ((e = hipMemcpy(dp, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
        (!ind.empty() && (e = hipMemcpy(di, ind.data(), ind.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)) {
        dev_free(dp);
        dev_free(di);
        return fail(FS_ERR_DEVICE, std::string("outgoing CSR upload: ") + hipGetErrorString(e));
    }
    g->d_out_ptr = dp;
    g->d_out_ind = di;
    return FS_OK;
}

void release_markov(fs_markov* m)
{
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream); // (blocks may return to a caller's allocator)
    if (m->exec) (void)hipGraphExecDestroy(m->exec);
    if (m->graph) (void)hipGraphDestroy(m->graph);
    for (void* p : {(void*)m->d_state, (void*)m->d_infl, (void*)m->d_events, (void*)m->d_ev_cnt, (void*)m->d_fired,
                    (void*)m->d_rpart,
                    (void*)m->d_part, (void*)m->d_hist, (void*)m->d_tau, (void*)m->d_evh, (void*)m->d_elapsed,
                    (void*)m->d_ctl})
        dev_free(p);
    if (m->own_stream && m->stream) (void)hipStreamDestroy(m->stream);
    if (m->g) m->g->users.fetch_sub(1);
    delete m;
}

// After a change of states from the host: recount every influence and the
// rate partials the next draw folds.
hipError_t refresh(fs_markov* m)
{
    MkArgs a = m->args;
    a.force_control = 1;
    a.step_off = 0;
    void* argv[] = {&a};
    return hipLaunchKernel((const void*)&fsm::mk_rates_kernel, dim3(m->G), dim3(fsm::MTPB), argv, 0, m->stream);
}

struct MkSeq {
    std::vector<MkArgs> step;
    fsi::Ctl* ctl;
    const uint32_t* part;
    uint32_t G, C, H, r;
    uint32_t* hist;
};

void make_seq(fs_markov* m, uint32_t r, MkSeq& q)
{
    q.step.assign(r, m->args);
    for (uint32_t j = 0; j < r; ++j) q.step[j].step_off = j;
    q.ctl = m->d_ctl;
    q.part = m->d_part;
    q.G = m->G;
    q.C = 4;
    q.H = m->H;
    q.r = r;
    q.hist = m->d_hist;
}

uint32_t push_grid(const fs_markov* m) { return std::max(1u, std::min((m->G + 3) / 4, 1024u)); }

fs_status build_exec(fs_markov* m, uint32_t b)
{
    MkSeq q;
    make_seq(m, b, q);
    FS_HIP(hipGraphCreate(&m->graph, 0));
    hipGraphNode_t prev = nullptr;
    auto add = [&](const void* fn, dim3 grid, dim3 block, void** argv) -> fs_status {
        hipKernelNodeParams kp{};
        kp.func = const_cast<void*>(fn);
        kp.gridDim = grid;
        kp.blockDim = block;
        kp.kernelParams = argv;
        hipGraphNode_t node;
        FS_HIP(hipGraphAddKernelNode(&node, m->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
        prev = node;
        return FS_OK;
    };
    fs_status st;
    for (uint32_t j = 0; j < b; ++j) {
        void* argv[] = {&q.step[j]};
        if ((st = add((const void*)&fsm::mk_draw_kernel, dim3(m->G), dim3(fsm::MTPB), argv)) != FS_OK) return st;
        if ((st = add((const void*)&fsm::mk_push_kernel, dim3(push_grid(m)), dim3(fsm::PTPB), argv)) != FS_OK) return st;
        if ((st = add((const void*)&fsm::mk_rates_kernel, dim3(m->G), dim3(fsm::MTPB), argv)) != FS_OK) return st;
    }
    void* rargv[] = {&q.ctl, &q.part, &q.G, &q.C, &q.hist, &q.H};
    if ((st = add(fsk::reduce_kernel_fn(), dim3(q.r), dim3(fsi::RED_TPB), rargv)) != FS_OK) return st;
    FS_HIP(hipGraphInstantiate(&m->exec, m->graph, nullptr, nullptr, 0));
    return FS_OK;
}

fs_status launch_seq(fs_markov* m, uint32_t r)
{
    MkSeq q;
    make_seq(m, r, q);
    for (uint32_t j = 0; j < r; ++j) {
        void* argv[] = {&q.step[j]};
        FS_HIP(hipLaunchKernel((const void*)&fsm::mk_draw_kernel, dim3(m->G), dim3(fsm::MTPB), argv, 0, m->stream));
        FS_HIP(hipLaunchKernel((const void*)&fsm::mk_push_kernel, dim3(push_grid(m)), dim3(fsm::PTPB), argv, 0,
                               m->stream));
        FS_HIP(hipLaunchKernel((const void*)&fsm::mk_rates_kernel, dim3(m->G), dim3(fsm::MTPB), argv, 0, m->stream));
    }
    void* rargv[] = {&q.ctl, &q.part, &q.G, &q.C, &q.hist, &q.H};
    FS_HIP(hipLaunchKernel(fsk::reduce_kernel_fn(), dim3(r), dim3(fsi::RED_TPB), rargv, 0, m->stream));
    return FS_OK;
}

} // namespace

#define FS_GUARD_BEGIN try {
#define FS_GUARD_END                                                                            \
    }                                                                                           \
    catch (const std::bad_alloc&) { return fail(FS_ERR_OUT_OF_MEMORY, "host allocation failed"); } \
    catch (const std::exception& e) { return fail(FS_ERR_DEVICE, e.what()); }                   \
    catch (...) { return fail(FS_ERR_DEVICE, "unknown exception"); }

extern "C" {

fs_status fs_markov_create(fs_graph* g, const fs_markov_params* p, fs_markov** out)
{
    FS_GUARD_BEGIN
    if (!out) return fail(FS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!g || !p) return fail(FS_ERR_INVALID_ARG, "NULL graph or params");
    if (g->d_weights) return fail(FS_ERR_INVALID_ARG, "the Markovian engine runs unit-weight graphs");
    if (p->model != FS_MARKOV_SEIR && p->model != FS_MARKOV_SIR && p->model != FS_MARKOV_SIS)
        return fail(FS_ERR_INVALID_ARG, "model must be FS_MARKOV_SEIR, FS_MARKOV_SIR or FS_MARKOV_SIS");
    auto finite_ge0 = [](double v) { return v >= 0.0 && std::isfinite(v); };
    if (!finite_ge0(p->beta) || !finite_ge0(p->gamma) || (p->model == FS_MARKOV_SEIR && !finite_ge0(p->sigma)))
        return fail(FS_ERR_INVALID_ARG, "rates must be finite and >= 0");
    if (!(p->theta > 0.0) || !(p->p_max > 0.0) || !(p->tau_max > 0.0) || !std::isfinite(p->theta) ||
        !std::isfinite(p->p_max) || !std::isfinite(p->tau_max))
        return fail(FS_ERR_INVALID_ARG, "theta, p_max and tau_max must be finite and > 0");
    if (p->history_len < 0 || p->history_len == 1) return fail(FS_ERR_INVALID_ARG, "history_len must be 0 or >= 2");
    if (p->steps_per_graph < 0 || p->steps_per_graph > 100000)
        return fail(FS_ERR_INVALID_ARG, "steps_per_graph out of range");
    if (p->inertial_max < -1) return fail(FS_ERR_INVALID_ARG, "inertial_max must be -1, 0 or positive");
    DeviceGuard dg(g->device);
    fs_status st = ensure_out_csr(g);
    if (st != FS_OK) return st;
    fs_markov* m = new fs_markov();
    m->g = g;
    g->users.fetch_add(1);
    m->p = *p;
    m->device = g->device;
    m->H = p->history_len ? (uint32_t)p->history_len : 1024u;
    m->chunk = (uint32_t)std::max(p->steps_per_graph, 64);
    const uint32_t n = (uint32_t)g->n;
    int cus = 0;
    hipError_t e;
    auto bad = [&](hipError_t err, const char* what) {
        release_markov(m);
        return fail(err == hipErrorOutOfMemory ? FS_ERR_OUT_OF_MEMORY : FS_ERR_DEVICE,
                    std::string(what) + ": " + hipGetErrorString(err));
    };
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m->device)) != hipSuccess)
        return bad(e, "device attribute");
    // one workgroup region per compute unit, in whole wavefronts
    m->G = (uint32_t)std::max<int64_t>(1, std::min<int64_t>({(int64_t)cus, (int64_t)fsm::MAX_REGIONS,
                                                              ((int64_t)n + 63) / 64}));
    m->span = (((n + m->G - 1) / m->G) + 63) / 64 * 64;
    m->G = (n + m->span - 1) / m->span;
    if (p->stream) {
        m->stream = (hipStream_t)p->stream;
    } else {
        if ((e = hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking)) != hipSuccess) return bad(e, "stream");
        m->own_stream = true;
    }
    const size_t part_words = (size_t)m->chunk * m->G * 4;
    if ((e = dev_alloc((void**)&m->d_state, n)) != hipSuccess ||
        (e = dev_alloc((void**)&m->d_infl, (size_t)n * 4)) != hipSuccess ||
        (e = dev_alloc((void**)&m->d_events, (size_t)m->G * m->span * 4)) != hipSuccess ||
        (e = dev_alloc((void**)&m->d_ev_cnt, (size_t)m->G * 4)) != hipSuccess ||
        (e = dev_alloc((void**)&m->d_fired, ((size_t)m->G + 1) * 4)) != hipSuccess ||
        (e = dev_alloc((void**)&m->d_rpart, (size_t)m->G * sizeof(uint4))) != hipSuccess ||
        (e = dev_alloc((void**)&m->d_part, part_words * 4)) != hipSuccess ||
        (e = dev_alloc((void**)&m->d_hist, (size_t)m->H * 16)) != hipSuccess ||
        (e = dev_alloc((void**)&m->d_tau, (size_t)m->H * 4)) != hipSuccess ||
        (e = dev_alloc((void**)&m->d_evh, (size_t)m->H * 4)) != hipSuccess ||
        (e = dev_alloc((void**)&m->d_elapsed, 8)) != hipSuccess ||
        (e = dev_alloc((void**)&m->d_ctl, sizeof(fsi::Ctl))) != hipSuccess)
        return bad(e, "device allocation");
    if ((e = hipMemsetAsync(m->d_state, 0, n, m->stream)) != hipSuccess ||
        (e = hipMemsetAsync(m->d_infl, 0, (size_t)n * 4, m->stream)) != hipSuccess ||
        (e = hipMemsetAsync(m->d_ev_cnt, 0, (size_t)m->G * 4, m->stream)) != hipSuccess ||
        (e = hipMemsetAsync(m->d_fired, 0, ((size_t)m->G + 1) * 4, m->stream)) != hipSuccess ||
        (e = hipMemsetAsync(m->d_hist, 0, (size_t)m->H * 16, m->stream)) != hipSuccess ||
        (e = hipMemsetAsync(m->d_tau, 0, (size_t)m->H * 4, m->stream)) != hipSuccess ||
        (e = hipMemsetAsync(m->d_evh, 0, (size_t)m->H * 4, m->stream)) != hipSuccess ||
        (e = hipMemsetAsync(m->d_elapsed, 0, 8, m->stream)) != hipSuccess ||
        (e = hipMemsetAsync(m->d_ctl, 0, sizeof(fsi::Ctl), m->stream)) != hipSuccess)
        return bad(e, "initialisation");
    MkArgs& a = m->args;
    a.state = m->d_state;
    a.infl = m->d_infl;
    a.row_ptr = g->d_row_ptr;
    a.col_ind = g->d_col_ind;
    a.out_ptr = g->d_out_ptr;
    a.out_ind = g->d_out_ind;
    a.orig_id = g->d_orig;
    a.events = m->d_events;
    a.ev_cnt = m->d_ev_cnt;
    a.fired = m->d_fired;
    a.rpart = m->d_rpart;
    a.part = m->d_part;
    a.tau_hist = m->d_tau;
    a.ev_hist = m->d_evh;
    a.elapsed = m->d_elapsed;
    a.ctl = m->d_ctl;
    a.n = n;
    a.G = m->G;
    a.span = m->span;
    a.H = m->H;
    a.model = p->model;
    a.beta = (float)p->beta;
    a.sigma = (float)p->sigma;
    a.gamma = (float)p->gamma;
    a.theta = p->theta;
    a.p_max = p->p_max;
    a.tau_max = p->tau_max;
    a.key0 = (uint32_t)p->seed;
    a.key1 = (uint32_t)(p->seed >> 32);
    // automatic threshold: pushes while the step's events touch fewer edges
    // than a recount reads (events * mean degree < nnz / 8)
    const double dmean = std::max(1.0, g->mean_degree);
    a.inertial_max = p->inertial_max == -1 ? 0u
                   : p->inertial_max > 0   ? (uint32_t)std::min<int64_t>(p->inertial_max, 0xFFFFFFFFll)
                                           : (uint32_t)std::max(1.0, (double)g->nnz / 8.0 / dmean);
    if ((e = refresh(m)) != hipSuccess || (e = hipStreamSynchronize(m->stream)) != hipSuccess)
        return bad(e, "initialisation");
    *out = m;
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_markov_destroy(fs_markov* m)
{
    FS_GUARD_BEGIN
    if (!m) return fail(FS_ERR_INVALID_ARG, "engine is NULL");
    DeviceGuard dg(m->device);
    hipError_t e = hipStreamSynchronize(m->stream);
    release_markov(m);
    if (e != hipSuccess) return fail(FS_ERR_DEVICE, std::string("pending work failed: ") + hipGetErrorString(e));
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_markov_seed(fs_markov* m, int64_t count, const int64_t* nodes, int32_t compartment)
{
    FS_GUARD_BEGIN
    if (!m) return fail(FS_ERR_INVALID_ARG, "engine is NULL");
    if (compartment < 0 || compartment > 3) return fail(FS_ERR_INVALID_ARG, "compartment must be in [0, 3]");
    if (count < 0) return fail(FS_ERR_INVALID_ARG, "count < 0");
    if (count == 0) return FS_OK;
    if (!nodes) return fail(FS_ERR_INVALID_ARG, "nodes is NULL");
    std::vector<int64_t> internal((size_t)count);
    for (int64_t j = 0; j < count; ++j) {
        if (nodes[j] < 0 || nodes[j] >= m->g->n) return fail(FS_ERR_INVALID_ARG, "seed node out of range");
        internal[(size_t)j] = m->g->h_inv.empty() ? nodes[j] : m->g->h_inv[(size_t)nodes[j]];
    }
    DeviceGuard dg(m->device);
    StreamBuf tmp(m->stream);
    FS_HIP(hipMallocAsync(&tmp.p, (size_t)count * 8, m->stream));
    FS_HIP(hipMemcpyAsync(tmp.p, internal.data(), (size_t)count * 8, hipMemcpyHostToDevice, m->stream));
    hipLaunchKernelGGL(fsm::mk_seed_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, m->stream,
                       m->d_state, (const int64_t*)tmp.p, count, compartment);
    FS_HIP(hipGetLastError());
    FS_HIP(refresh(m));
    FS_HIP(hipStreamSynchronize(m->stream));
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_markov_set_state(fs_markov* m, const int32_t* state, int64_t step_index, double elapsed)
{
    FS_GUARD_BEGIN
    if (!m || !state) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    if (step_index < -1) return fail(FS_ERR_INVALID_ARG, "step_index must be >= -1");
    if (!(elapsed >= 0.0) || !std::isfinite(elapsed)) return fail(FS_ERR_INVALID_ARG, "elapsed must be finite and >= 0");
    const size_t n = (size_t)m->g->n;
    std::vector<int32_t> st(n);
    for (size_t i = 0; i < n; ++i) {
        const int32_t v = m->g->h_orig.empty() ? state[i] : state[(size_t)m->g->h_orig[i]];
        if (v < 0 || v > 3) return fail(FS_ERR_INVALID_ARG, "state values must lie in [0, 3]");
        st[i] = v;
    }
    DeviceGuard dg(m->device);
    const int64_t new_step = step_index >= 0 ? step_index : m->step;
    StreamBuf tmp(m->stream);
    FS_HIP(hipMallocAsync(&tmp.p, n * 4, m->stream));
    FS_HIP(hipMemcpyAsync(tmp.p, st.data(), n * 4, hipMemcpyHostToDevice, m->stream));
    hipLaunchKernelGGL(fsm::mk_put_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, m->stream, m->d_state,
                       (const int32_t*)tmp.p, (uint32_t)n);
    FS_HIP(hipGetLastError());
    hipLaunchKernelGGL(fsm::mk_clear_kernel, dim3(1), dim3(64), 0, m->stream, m->d_elapsed, elapsed);
    FS_HIP(hipGetLastError());
    FS_HIP(fsk::launch_set_ctl(m->d_ctl, (unsigned long long)new_step, m->stream));
    FS_HIP(refresh(m));
    FS_HIP(hipStreamSynchronize(m->stream));
    if (step_index >= 0) {
        m->step = step_index;
        m->hist_from = step_index;
    }
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_markov_step(fs_markov* m, int64_t n_steps)
{
    FS_GUARD_BEGIN
    if (!m) return fail(FS_ERR_INVALID_ARG, "engine is NULL");
    if (n_steps < 0) return fail(FS_ERR_INVALID_ARG, "n_steps < 0");
    DeviceGuard dg(m->device);
    const int b = m->p.steps_per_graph;
    int64_t left = n_steps;
    if (b > 0) {
        if (!m->exec) {
            fs_status st = build_exec(m, (uint32_t)b);
            if (st != FS_OK) return st;
        }
        for (; left >= b; left -= b) FS_HIP(hipGraphLaunch(m->exec, m->stream));
    }
    while (left > 0) {
        const uint32_t r = (uint32_t)std::min<int64_t>(left, m->chunk);
        fs_status st = launch_seq(m, r);
        if (st != FS_OK) return st;
        left -= r;
    }
    m->step += n_steps;
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_markov_sync(fs_markov* m)
{
    if (!m) return fail(FS_ERR_INVALID_ARG, "engine is NULL");
    DeviceGuard dg(m->device);
    FS_HIP(hipStreamSynchronize(m->stream));
    return FS_OK;
}

fs_status fs_markov_get_state(fs_markov* m, int32_t* state, int32_t* influence, int64_t* step_index, double* elapsed)
{
    FS_GUARD_BEGIN
    if (!m) return fail(FS_ERR_INVALID_ARG, "engine is NULL");
    DeviceGuard dg(m->device);
    const size_t n = (size_t)m->g->n;
    std::vector<uint8_t> st(n);
    std::vector<int32_t> inf(n);
    double el = 0.0;
    FS_HIP(hipMemcpyAsync(st.data(), m->d_state, n, hipMemcpyDeviceToHost, m->stream));
    FS_HIP(hipMemcpyAsync(inf.data(), m->d_infl, n * 4, hipMemcpyDeviceToHost, m->stream));
    FS_HIP(hipMemcpyAsync(&el, m->d_elapsed, 8, hipMemcpyDeviceToHost, m->stream));
    FS_HIP(hipStreamSynchronize(m->stream));
    for (size_t i = 0; i < n; ++i) {
        const size_t c = m->g->h_orig.empty() ? i : (size_t)m->g->h_orig[i];
        if (state) state[c] = st[i];
        if (influence) influence[c] = inf[i];
    }
    if (step_index) *step_index = m->step;
    if (elapsed) *elapsed = el;
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_markov_history(fs_markov* m, int64_t first_step, int64_t n, int64_t* counts, double* taus, int64_t* events)
{
    FS_GUARD_BEGIN
    if (!m) return fail(FS_ERR_INVALID_ARG, "engine is NULL");
    if (n < 0) return fail(FS_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return FS_OK;
    if (first_step < m->hist_from || first_step + n > m->step || m->step - first_step > (int64_t)m->H)
        return fail(FS_ERR_INVALID_ARG, "steps outside the recorded window");
    DeviceGuard dg(m->device);
    std::vector<uint32_t> h((size_t)m->H * 4), ev(m->H);
    std::vector<float> t(m->H);
    FS_HIP(hipMemcpyAsync(h.data(), m->d_hist, h.size() * 4, hipMemcpyDeviceToHost, m->stream));
    FS_HIP(hipMemcpyAsync(t.data(), m->d_tau, t.size() * 4, hipMemcpyDeviceToHost, m->stream));
    FS_HIP(hipMemcpyAsync(ev.data(), m->d_evh, ev.size() * 4, hipMemcpyDeviceToHost, m->stream));
    FS_HIP(hipStreamSynchronize(m->stream));
    for (int64_t j = 0; j < n; ++j) {
        const size_t slot = (size_t)((first_step + j) % m->H);
        if (counts)
            for (int q = 0; q < 4; ++q) counts[4 * j + q] = h[slot * 4 + (size_t)q];
        if (taus) taus[j] = t[slot];
        if (events) events[j] = ev[slot];
    }
    return FS_OK;
    FS_GUARD_END
}

} // extern "C"
