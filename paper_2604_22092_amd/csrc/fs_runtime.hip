// Host runtime of the C ABI declared in include/fs.h: validation, device
// memory, the device-resident step index, eager and hipGraph step loops,
// state transfer and counts.  No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <new>
#include <string>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "fs_runtime.hpp"

namespace fsr {

thread_local std::string g_err;

fs_status fail(fs_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

// The caller's device allocator (fs_set_allocator), and the release path of
// every block it gave out: a block is returned to whoever allocated it, also
// after the hook has changed.
struct Hook {
    fs_alloc_fn alloc = nullptr;
    fs_free_fn free = nullptr;
    void* ctx = nullptr;
};
std::mutex g_hook_mu;
Hook g_hook;
std::unordered_map<void*, Hook> g_hooked;

hipError_t hook_alloc(void** p, size_t bytes, bool* used)
{
    Hook h;
    {
        std::lock_guard<std::mutex> lk(g_hook_mu);
        h = g_hook;
    }
    *used = h.alloc != nullptr;
    if (!*used) return hipSuccess;
    *p = h.alloc(bytes, h.ctx);
    if (!*p) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> lk(g_hook_mu);
    g_hooked[*p] = h;
    return hipSuccess;
}

// Returns true when p came from a caller's allocator (and releases it).
bool hook_free(void* p)
{
    Hook h;
    {
        std::lock_guard<std::mutex> lk(g_hook_mu);
        auto it = g_hooked.find(p);
        if (it == g_hooked.end()) return false;
        h = it->second;
        g_hooked.erase(it);
    }
    h.free(p, h.ctx);
    return true;
}

hipError_t dev_alloc(void** p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    bool used = false;
    hipError_t e = hook_alloc(p, bytes, &used);
    if (used) return e;
    return hipMalloc(p, bytes);
}

void dev_free(void* p)
{
    if (p && !hook_free(p)) (void)hipFree(p);
}

// Per-sim buffers are stream-ordered allocations on the sim's stream: making
// and releasing a sim never waits for work queued on other streams.  The
// device's default pool keeps freed memory for reuse.
void keep_pool(int device)
{
    static std::mutex mu;
    static std::vector<int> done;
    std::lock_guard<std::mutex> lk(mu);
    if (std::find(done.begin(), done.end(), device) != done.end()) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    done.push_back(device);
}

hipError_t sim_alloc(fs_sim* s, void** p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    bool used = false;
    hipError_t e = hook_alloc(p, bytes, &used);
    if (used) return e;
    return hipMallocAsync(p, bytes, s->stream);
}

// A block from the caller's allocator is released once the sim's stream has
// finished with it; the library's own blocks are freed in stream order.
void sim_free(fs_sim* s, void* p)
{
    if (!p) return;
    bool hooked;
    {
        std::lock_guard<std::mutex> lk(g_hook_mu);
        hooked = g_hooked.count(p) != 0;
    }
    if (hooked) {
        (void)hipStreamSynchronize(s->stream);
        hook_free(p);
    } else {
        (void)hipFreeAsync(p, s->stream);
    }
}

// Per-node arrays between the caller's node order and a graph's internal
// order (no copy when the graph keeps the caller's order).
template <class T>
const T* to_internal(const fs_graph* g, const T* in, std::vector<T>& tmp)
{
    if (g->h_orig.empty()) return in;
    tmp.resize(g->h_orig.size());
    for (size_t j = 0; j < tmp.size(); ++j) tmp[j] = in[g->h_orig[j]];
    return tmp.data();
}

template <class T>
void to_caller(const fs_graph* g, const T* in, T* out)
{
    for (size_t j = 0; j < g->h_orig.size(); ++j) out[g->h_orig[j]] = in[j];
}


void split(double v, float& hi, float& lo)
{
    hi = (float)v;
    lo = (float)(v - (double)hi);
}

fs_status prep_hazard(const fs_dist& d, int storage, double dt, HazardDev* h, const char* which)
{
    std::memset(h, 0, sizeof *h);
    const double unit = storage == FS_STORAGE_COMPACT ? dt : 1.0;
    h->kind = d.kind;
    h->k = d.k;
    switch (d.kind) {
    case FS_DIST_EXP:
        if (!(d.a >= 0.0) || !std::isfinite(d.a))
            return fail(FS_ERR_INVALID_ARG, std::string(which) + ": exponential rate must be finite and >= 0");
        h->K = (float)d.a;
        return FS_OK;
    case FS_DIST_LOGNORMAL:
        if (!std::isfinite(d.a) || !(d.b > 0.0) || !std::isfinite(d.b))
            return fail(FS_ERR_INVALID_ARG, std::string(which) + ": log-normal needs finite mu and sigma > 0");
        h->K = (float)(std::sqrt(2.0 / M_PI) / (d.b * unit));
        split(std::log(unit) - d.a, h->c_hi, h->c_lo);
        split(1.0 / (d.b * std::sqrt(2.0)), h->g_hi, h->g_lo);
        return FS_OK;
    case FS_DIST_WEIBULL:
        if (!(d.a >= 1.0) || !std::isfinite(d.a) || !(d.b > 0.0) || !std::isfinite(d.b))
            return fail(FS_ERR_INVALID_ARG, std::string(which) + ": Weibull needs shape >= 1 and scale > 0");
        h->K = (float)(d.a / d.b);
        split(std::log(unit / d.b), h->c_hi, h->c_lo);
        split(d.a - 1.0, h->g_hi, h->g_lo);
        return FS_OK;
    case FS_DIST_ERLANG:
        if (d.k < 1 || d.k > 64 || !(d.a > 0.0) || !std::isfinite(d.a))
            return fail(FS_ERR_INVALID_ARG, std::string(which) + ": Erlang needs k in [1, 64] and rate > 0");
        h->K = (float)d.a;
        split(d.a * unit, h->x_hi, h->x_lo);
        return FS_OK;
    default:
        return fail(FS_ERR_INVALID_ARG, std::string(which) + ": unknown holding-time law");
    }
}

// Shedding profile of Eq. (infectivity) for the device (see fsi::ShedDev):
// the law's hazard parameters, then the constant K and the extra terms of
// the chosen form, in double precision, rounded once.
fs_status prep_shed(int32_t form, const fs_dist& d, double A, int storage, double dt, fsi::ShedDev* sd)
{
    std::memset(sd, 0, sizeof *sd);
    if (form == FS_SHED_CONSTANT) return FS_OK;
    if (form != FS_SHED_DENSITY && form != FS_SHED_HAZARD)
        return fail(FS_ERR_INVALID_ARG, "shedding must be FS_SHED_CONSTANT, FS_SHED_DENSITY or FS_SHED_HAZARD");
    if (!(A >= 0.0) || !std::isfinite(A)) return fail(FS_ERR_INVALID_ARG, "shed_scale must be finite and >= 0");
    fs_status st = prep_hazard(d, storage, dt, &sd->hz, "shed_law");
    if (st != FS_OK) return st;
    const double unit = storage == FS_STORAGE_COMPACT ? dt : 1.0;
    const double sq2pi = std::sqrt(2.0 * M_PI);
    if (form == FS_SHED_HAZARD) {
        double K = d.a; // exponential, Erlang: the rate
        if (d.kind == FS_DIST_LOGNORMAL) K = std::sqrt(2.0 / M_PI) / (d.b * unit);
        if (d.kind == FS_DIST_WEIBULL) K = d.a / d.b;
        sd->hz.K = (float)(A * K);
        return FS_OK;
    }
    sd->density = 1;
    switch (d.kind) {
    case FS_DIST_LOGNORMAL:
        sd->hz.K = (float)(A / (d.b * sq2pi * unit));
        sd->s0 = 0.0f;
        break;
    case FS_DIST_WEIBULL:
        sd->hz.K = (float)(A * d.a / d.b);
        split(d.a, sd->m_hi, sd->m_lo);
        sd->s0 = d.a == 1.0 ? (float)(A / d.b) : 0.0f;
        break;
    case FS_DIST_ERLANG:
        sd->hz.K = (float)(A * d.a);
        split(std::lgamma((double)d.k), sd->lf_hi, sd->lf_lo);
        sd->s0 = d.k == 1 ? (float)(A * d.a) : 0.0f;
        break;
    default: // exponential
        sd->hz.K = (float)(A * d.a);
        split(d.a * unit, sd->hz.x_hi, sd->hz.x_lo);
        sd->s0 = (float)(A * d.a);
        break;
    }
    return FS_OK;
}

size_t state_bytes(int storage) { return storage == FS_STORAGE_FP32 ? 4 : 1; }
size_t age_bytes(int storage) { return storage == FS_STORAGE_FP32 ? 4 : 2; }
// bytes of a stored shedding value: float32, or binary16 with compact storage
size_t shed_bytes(int storage) { return storage == FS_STORAGE_FP32 ? 4 : 2; }
// 64-bit words of an infectivity bitmap of `units` bits, in whole tiles.
size_t bitmap_words(size_t units) { return (units + fsi::BITMAP_TILE - 1) / fsi::BITMAP_TILE * (fsi::BITMAP_TILE / 64); }

void release_sim(fs_sim* s)
{
    if (!s) return;
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    s->exec = nullptr;
    s->graph = nullptr;
    if (s->stream) {
        for (void* p : {s->d_state, s->d_age, s->d_iota[0], s->d_iota[1], (void*)s->d_rates, (void*)s->d_ctl,
                        (void*)s->d_hist, (void*)s->d_part, (void*)s->d_rc_part, (void*)s->d_cnt4,
                        (void*)s->d_summary, s->d_seg_part, (void*)s->d_lam_part, (void*)s->d_dt_hist,
                        (void*)s->d_shed[0], (void*)s->d_shed[1], (void*)s->d_live, (void*)s->d_act,
                        (void*)s->d_htab, (void*)s->d_laws, (void*)s->d_hub})
            sim_free(s, p);
    }
    s->layout.reset();
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    if (s->g) s->g->users.fetch_sub(1);
    delete s;
}

fs_status check_replica(const fs_sim* s, int32_t replica, bool allow_all)
{
    if (replica >= 0 && replica < s->R) return FS_OK;
    if (allow_all && replica == -1) return FS_OK;
    return fail(FS_ERR_INVALID_ARG, "replica index out of range");
}

constexpr uint32_t RC_GRID = 1024;

// Launch sequence of r steps: (with compaction: a rates clear when rates are
// recorded, and the active-list refresh) r step launches, and one reduce,
// which also advances the device step index.
struct SeqArgs {
    std::vector<StepArgs> step;
    std::vector<fsi::HeavyArgs> heavy;
    std::vector<fsi::SumArgs> sum;
    fsi::Ctl* ctl;
    const uint32_t* part;
    uint32_t G, C, H, r;
    uint32_t* hist;
    // compaction refresh
    const uint8_t* live;
    uint32_t nchunks, rows, n;
    uint32_t* act;
    uint32_t* rates;
    size_t rates_words;
};

uint32_t clear_grid(size_t words) { return (uint32_t)std::max<size_t>(1, std::min<size_t>((words + 255) / 256, 4096)); }

uint32_t heavy_grid(const fs_sim* s)
{
    const uint32_t per_wg = WG / 64;
    return std::max(1u, std::min((s->nseg + per_wg - 1) / per_wg, 8192u));
}

// The sim's own heavy-row launch: with the resident step, the LDS-resident
// kernel (at most one workgroup per CU), else heavy_grid WG-thread workgroups.
uint32_t sim_heavy_block(const fs_sim* s) { return s->mode == fsi::MODE_RESIDENT ? fsi::RESIDENT_TPB : WG; }

uint32_t sim_heavy_grid(const fs_sim* s)
{
    if (s->mode != fsi::MODE_RESIDENT) return heavy_grid(s);
    const uint32_t per_wg = fsi::RESIDENT_TPB / 64;
    return std::max(1u, std::min((s->nseg + per_wg - 1) / per_wg, std::max(s->cus, 1u)));
}

void drop_graph_exec(fs_sim* s)
{
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    s->exec = nullptr;
    s->graph = nullptr;
}

// (Re)builds the degree bins: rows with degree > heavy_deg (and any row of
// 65535 or more edges) are cut into segments of at most seg_edges edges for
// the heavy-row kernel; the other rows are laid out wavefront-transposed for
// the step kernel (see StepArgs::col_t).
Layout::~Layout()
{
    dev_free(d_heavy_first);
    dev_free(d_segs);
    dev_free(d_ldeg);
    dev_free(d_chunk_meta);
    dev_free(d_col_t);
    dev_free(d_w_t);
    dev_free(d_hub_out_ptr);
    dev_free(d_hub_out_idx);
}

// Builds the layout of graph g for R replicas (Q = 64/R nodes per chunk).
// Bits per packed column for a graph of n nodes (ids below n), or 0 when
// 27 bits do not hold them.
int32_t packed_bits(int64_t n)
{
    if (n <= ((int64_t)1 << 20)) return 20;
    if (n <= ((int64_t)1 << 24)) return 24;
    if (n <= ((int64_t)1 << 27)) return 27;
    return 0;
}

fs_status build_layout(const fs_graph* g, int32_t R, int32_t limit, int32_t seg_edges, bool pack,
                       std::shared_ptr<Layout>& out)
{
    auto L = std::make_shared<Layout>();
    L->limit = limit;
    L->seg_edges = seg_edges;
    const int64_t n = g->n;
    const std::vector<int32_t>& rp = g->h_row_ptr;
    std::vector<int32_t> first;
    std::vector<fsi::Segment> segs;
    std::vector<uint16_t> ldeg((size_t)n);
    if (g->max_degree > limit) first.assign((size_t)n, -1);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t b = rp[i], e = rp[i + 1];
        if (e - b <= limit) {
            ldeg[i] = (uint16_t)(e - b);
            continue;
        }
        ldeg[i] = fsi::HEAVY_ROW;
        first[i] = (int32_t)segs.size();
        for (int32_t x = b; x < e; x += seg_edges) segs.push_back({(int32_t)i, x, std::min(e, x + seg_edges), 0});
    }
    // wavefront-transposed light layout: Q nodes per 64-unit chunk
    const int64_t Q = 64 / R;
    const int64_t nch = (n + Q - 1) / Q;
    // uniform graph: no heavy row and one light degree <= UNIFORM_MAX_DEG; the
    // last chunk's missing rows are then padded with column 0 (their lanes
    // are past the last unit and never use them)
    int32_t ud_all = segs.empty() && n > 0 ? (int32_t)ldeg[0] : -1;
    for (int64_t i = 0; i < n && ud_all >= 0; ++i)
        if ((int32_t)ldeg[i] != ud_all) ud_all = -1;
    if (ud_all > fsi::UNIFORM_MAX_DEG) ud_all = -1;
    L->udeg = ud_all;
    // packed columns (unweighted layouts of one replica): every chunk whose
    // rows share one degree d <= UNIFORM_MAX_DEG (all of a uniform layout's,
    // the last one padded with rows of columns 0) stores PB bits per column,
    // a row's columns one bit stream of W = ceil(d PB / 32) words, word w of
    // row q at the chunk's base + w * Q + q; other chunks keep 32-bit columns
    const int32_t PB = (pack && R == 1 && g->d_weights == nullptr) ? packed_bits(n) : 0;
    L->pbits = PB;
    std::vector<uint32_t> cbase((size_t)nch + 1);
    std::vector<int32_t> colt;
    std::vector<float> wt;
    colt.reserve((size_t)g->nnz);
    const bool weighted = g->d_weights != nullptr;
    std::vector<uint8_t> cdeg((size_t)nch);
    for (int64_t c = 0; c < nch; ++c) {
        cbase[c] = (uint32_t)colt.size();
        const int64_t n0 = c * Q, n1 = std::min(n, n0 + Q);
        int32_t pd = ud_all; // the packed chunk's degree, or -1
        if (PB && pd < 0) {
            pd = n1 - n0 == Q ? (int32_t)ldeg[n0] : -1;
            for (int64_t i = n0; i < n1 && pd >= 0; ++i)
                if (ldeg[i] == fsi::HEAVY_ROW || (int32_t)ldeg[i] != pd) pd = -1;
            if (pd > fsi::UNIFORM_MAX_DEG) pd = -1;
        }
        if (PB && pd >= 0) {
            const int32_t W = (pd * PB + 31) / 32;
            std::vector<uint32_t> words((size_t)W * (size_t)Q, 0u);
            for (int64_t i = n0; i < n1; ++i)
                for (int32_t j = 0; j < pd; ++j) {
                    const uint64_t v = (uint32_t)g->h_col_ind[rp[i] + j];
                    const int32_t o = PB * j, lo = o >> 5, sh = o & 31;
                    words[(size_t)lo * Q + (size_t)(i - n0)] |= (uint32_t)(v << sh);
                    if (sh + PB > 32) words[(size_t)(lo + 1) * Q + (size_t)(i - n0)] |= (uint32_t)(v >> (32 - sh));
                }
            for (uint32_t x : words) colt.push_back((int32_t)x);
            cdeg[c] = (uint8_t)pd;
            continue;
        }
        int32_t maxd = 0;
        bool same = n1 - n0 == Q;
        for (int64_t i = n0; i < n1; ++i) {
            if (ldeg[i] != fsi::HEAVY_ROW) maxd = std::max<int32_t>(maxd, ldeg[i]);
            same = same && ldeg[i] != fsi::HEAVY_ROW && ldeg[i] == ldeg[n0];
        }
        cdeg[c] = (same && ldeg[n0] < 255) ? (uint8_t)ldeg[n0] : (uint8_t)255;
        if (ud_all >= 0 && n1 - n0 < Q) {
            cdeg[c] = (uint8_t)ud_all;
            for (int32_t j = 0; j < ud_all; ++j)
                for (int64_t i = n0; i < n0 + Q; ++i) colt.push_back(i < n1 ? g->h_col_ind[rp[i] + j] : 0);
            if (weighted)
                for (int32_t j = 0; j < ud_all; ++j)
                    for (int64_t i = n0; i < n0 + Q; ++i) wt.push_back(i < n1 ? g->h_weights[rp[i] + j] : 0.0f);
            continue;
        }
        if (same) {
            // every row has the same light degree: slot j of row q at j*Q + q
            const int32_t d = ldeg[n0];
            for (int32_t j = 0; j < d; ++j)
                for (int64_t i = n0; i < n1; ++i) colt.push_back(g->h_col_ind[rp[i] + j]);
            if (weighted)
                for (int32_t j = 0; j < d; ++j)
                    for (int64_t i = n0; i < n1; ++i) wt.push_back(g->h_weights[rp[i] + j]);
            continue;
        }
        for (int32_t j = 0; j < maxd; ++j)
            for (int64_t i = n0; i < n1; ++i)
                if (ldeg[i] != fsi::HEAVY_ROW && ldeg[i] > j) {
                    colt.push_back(g->h_col_ind[rp[i] + j]);
                    if (weighted) wt.push_back(g->h_weights[rp[i] + j]);
                }
    }
    cbase[nch] = (uint32_t)colt.size();
    L->nseg = (uint32_t)segs.size();
    if (L->nseg) {
        FS_HIP(dev_alloc((void**)&L->d_heavy_first, first.size() * sizeof(int32_t)));
        FS_HIP(dev_alloc((void**)&L->d_segs, segs.size() * sizeof(fsi::Segment)));
        FS_HIP(hipMemcpy(L->d_heavy_first, first.data(), first.size() * sizeof(int32_t), hipMemcpyHostToDevice));
        FS_HIP(hipMemcpy(L->d_segs, segs.data(), segs.size() * sizeof(fsi::Segment), hipMemcpyHostToDevice));
    }
    FS_HIP(dev_alloc((void**)&L->d_ldeg, ldeg.size() * sizeof(uint16_t)));
    std::vector<uint2> meta(cbase.size());
    for (size_t c = 0; c < cbase.size(); ++c) meta[c] = make_uint2(cbase[c], c < cdeg.size() ? cdeg[c] : 255u);
    FS_HIP(dev_alloc((void**)&L->d_chunk_meta, meta.size() * sizeof(uint2)));
    FS_HIP(dev_alloc((void**)&L->d_col_t, colt.size() * sizeof(int32_t)));
    FS_HIP(hipMemcpy(L->d_chunk_meta, meta.data(), meta.size() * sizeof(uint2), hipMemcpyHostToDevice));
    FS_HIP(hipMemcpy(L->d_ldeg, ldeg.data(), ldeg.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    if (!colt.empty())
        FS_HIP(hipMemcpy(L->d_col_t, colt.data(), colt.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if (weighted) {
        FS_HIP(dev_alloc((void**)&L->d_w_t, wt.size() * sizeof(float)));
        if (!wt.empty()) FS_HIP(hipMemcpy(L->d_w_t, wt.data(), wt.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    // pushes into binned rows (unit weights): the rows are the last nodes of
    // the degree-sorted order; per node, the rows listing it
    size_t hub_bytes = 0;
    if (!segs.empty() && !weighted) {
        int64_t hb = n;
        while (hb > 0 && ldeg[(size_t)hb - 1] == fsi::HEAVY_ROW) --hb;
        bool tail = true;
        for (int64_t i = 0; i < hb && tail; ++i) tail = ldeg[(size_t)i] != fsi::HEAVY_ROW;
        if (tail) {
            std::vector<int32_t> optr((size_t)n + 1, 0);
            for (int64_t i = hb; i < n; ++i)
                for (int32_t e = rp[i]; e < rp[i + 1]; ++e) ++optr[(size_t)g->h_col_ind[e] + 1];
            for (int64_t j = 0; j < n; ++j) optr[(size_t)j + 1] += optr[(size_t)j];
            std::vector<int32_t> oidx((size_t)optr[(size_t)n]);
            std::vector<int32_t> fill(optr.begin(), optr.end() - 1);
            for (int64_t i = hb; i < n; ++i)
                for (int32_t e = rp[i]; e < rp[i + 1]; ++e)
                    oidx[(size_t)fill[(size_t)g->h_col_ind[e]]++] = (int32_t)(i - hb);
            FS_HIP(dev_alloc((void**)&L->d_hub_out_ptr, optr.size() * sizeof(int32_t)));
            FS_HIP(dev_alloc((void**)&L->d_hub_out_idx, oidx.size() * sizeof(int32_t)));
            FS_HIP(hipMemcpy(L->d_hub_out_ptr, optr.data(), optr.size() * sizeof(int32_t), hipMemcpyHostToDevice));
            if (!oidx.empty())
                FS_HIP(hipMemcpy(L->d_hub_out_idx, oidx.data(), oidx.size() * sizeof(int32_t), hipMemcpyHostToDevice));
            L->hub_base = (int32_t)hb;
            L->hubs = (uint32_t)(n - hb);
            hub_bytes = optr.size() * 4 + oidx.size() * 4;
        }
    }
    L->bytes = first.size() * 4 + segs.size() * sizeof(fsi::Segment) + ldeg.size() * 2 + cbase.size() * 4 +
               cdeg.size() + colt.size() * 4 + wt.size() * 4 + hub_bytes;
    out = std::move(L);
    return FS_OK;
}

int32_t light_limit(int32_t heavy_deg)
{
    const int32_t cap = 65534; // largest light degree a uint16 entry holds
    return heavy_deg < 0 ? cap : std::min(heavy_deg, cap);
}

bool layout_cached(fs_graph* g, int32_t R, int32_t heavy_deg, int32_t seg_edges, bool pack)
{
    std::lock_guard<std::mutex> lk(g->layout_mu);
    return g->layouts.count(LayoutKey(R, light_limit(heavy_deg), seg_edges, pack ? 1 : 0)) != 0;
}

// Whether a sim of these parameters may take packed columns: the
// single-replica step of an unweighted graph (not age-dependent shedding
// together with rate recording or compaction), unless the caller asks for
// 32-bit columns.
bool packing_allowed(const fs_graph* g, const fs_sim_params* p)
{
    return p->columns == FS_COLUMNS_AUTO && std::max(p->n_replicas, 1) == 1 && g->d_weights == nullptr &&
           !(p->shedding != FS_SHED_CONSTANT && (p->record_rates || p->compaction));
}

size_t sim_footprint(fs_graph* g, const fs_sim_params* p)
{
    const size_t R = (size_t)std::max(p->n_replicas, 1);
    const size_t units = (size_t)g->n * R;
    const size_t H = p->history_len ? (size_t)p->history_len : 1024;
    const size_t chunk = (size_t)std::max(p->steps_per_graph, 64);
    const size_t grid = std::min<size_t>((units + 255) / 256, fsi::max_step_grid((int)R));
    size_t b = units * (state_bytes(p->storage) + age_bytes(p->storage));
    b += 2 * bitmap_words(units) * 8;                   // infectivity ping-pong
    b += H * R * 16 + chunk * grid * R * 16;            // history ring, count partials
    const int32_t hd = p->heavy_degree == 0 ? 64 : p->heavy_degree;
    const int32_t se = p->segment_edges == 0 ? 512 : p->segment_edges;
    const bool pk = packing_allowed(g, p);
    if (!layout_cached(g, (int32_t)R, hd, se, pk)) {
        b += (size_t)g->nnz * 4 * (g->d_weights ? 2 : 1);   // transposed light rows (+ weights)
        b += (size_t)g->n * 2 + ((size_t)g->n * R / 64 + 1) * 5; // degrees, chunk metadata
        b += (size_t)g->nnz / 64 * 16 + (size_t)g->n * 4;   // heavy segments (upper bound)
    }
    b += (size_t)g->nnz / 64 * 4 * R;                       // heavy-segment partials (upper bound)
    if (g->max_degree > hd && hd > 0) {
        // pushed pressure of binned rows: at most nnz / (hd + 1) rows
        const size_t hubs = std::min<size_t>((size_t)g->n, (size_t)g->nnz / ((size_t)hd + 1));
        b += 5 * hubs * R * 4;
        if (!layout_cached(g, (int32_t)R, hd, se, pk)) b += ((size_t)g->n + 1) * 4 + (size_t)g->nnz * 4;
    }
    if (p->record_rates) b += units * 4;
    if (p->shedding != FS_SHED_CONSTANT) b += units * 2 * shed_bytes(p->storage);
    if (p->compaction) b += (units / 64 + 1) * 5 + fsi::LIVE_TILE;
    return b + ((size_t)1 << 20);
}

// Pushed pressure of the binned rows (StepArgs::hub_T) recounted from the
// bitmap step `step` reads, with every delta slot cleared: the state the
// steps maintain, rebuilt after a change of states from the host.
hipError_t refresh_hubs(fs_sim* s, int64_t step)
{
    if (!s->hub_push) return hipSuccess;
    const Layout& L = *s->layout;
    const uint32_t HU = L.hubs * (uint32_t)s->R;
    hipError_t e = fsk::launch_hub_recount(s->g->d_row_ptr, s->g->d_col_ind, L.hub_base, L.hubs, s->lgR,
                                           (const uint32_t*)s->d_iota[step & 1],
                                           s->d_hub + (size_t)((step - 1) & 1) * HU, s->stream);
    if (e != hipSuccess) return e;
    return fsk::launch_clear_u32(s->d_hub + 2 * (size_t)HU, 3 * (size_t)HU, s->stream);
}

// Points sim s at the layout of its graph for (R, heavy_deg, seg_edges),
// building it on first use, and gives s its own heavy-segment partials.
// Cached layouts no sim uses any more, other than this one, are released.
fs_status apply_bins(fs_sim* s, int32_t heavy_deg, int32_t seg_edges)
{
    fs_graph* g = s->g;
    if (seg_edges < 64 || seg_edges > (1 << 20)) return fail(FS_ERR_INVALID_ARG, "segment_edges must be in [64, 2^20]");
    const int32_t limit = light_limit(heavy_deg);
    const LayoutKey key(s->R, limit, seg_edges, s->pack ? 1 : 0);
    std::shared_ptr<Layout> L;
    {
        std::lock_guard<std::mutex> lk(g->layout_mu);
        auto it = g->layouts.find(key);
        if (it != g->layouts.end()) {
            L = it->second;
        } else {
            fs_status st = build_layout(g, s->R, limit, seg_edges, s->pack, L);
            if (st != FS_OK) return st;
            g->layouts[key] = L;
        }
    }
    drop_graph_exec(s);
    sim_free(s, s->d_seg_part);
    s->d_seg_part = nullptr;
    sim_free(s, s->d_hub);
    s->d_hub = nullptr;
    s->hub_push = false;
    s->args.hub_T = s->args.hub_D = nullptr;
    s->layout = L;
    {
        std::lock_guard<std::mutex> lk(g->layout_mu);
        for (auto it = g->layouts.begin(); it != g->layouts.end();) {
            if (it->first != key && it->second.use_count() == 1) it = g->layouts.erase(it);
            else ++it;
        }
    }
    s->nseg = L->nseg;
    s->d_segs = L->d_segs;
    s->heavy_deg = heavy_deg;
    s->seg_edges = seg_edges;
    // binned rows of an unweighted graph with constant shedding take pushed
    // pressure; the others (and batches of such sims) read segment partials
    s->hub_push = L->hubs > 0 && s->d_shed[0] == nullptr;
    if (s->nseg && !s->hub_push)
        FS_HIP(sim_alloc(s, &s->d_seg_part, (size_t)s->nseg * (size_t)s->R * sizeof(uint32_t)));
    if (s->hub_push) {
        const size_t HU = (size_t)L->hubs * (size_t)s->R;
        FS_HIP(sim_alloc(s, (void**)&s->d_hub, 5 * HU * sizeof(uint32_t)));
        s->args.hub_T = s->d_hub;
        s->args.hub_D = s->d_hub + 2 * HU;
        s->args.hub_out_ptr = L->d_hub_out_ptr;
        s->args.hub_out_idx = L->d_hub_out_idx;
        s->args.hub_base = L->hub_base;
        s->args.hub_units = (uint32_t)HU;
        FS_HIP(refresh_hubs(s, s->step));
    }
    s->args.heavy_first = L->d_heavy_first;
    s->args.seg_part = s->d_seg_part;
    s->args.heavy_deg = limit;
    s->args.seg_edges = seg_edges;
    s->args.ldeg = L->d_ldeg;
    s->args.chunk_meta = L->d_chunk_meta;
    s->args.orig_id = g->d_orig;
    s->args.udeg = L->udeg;
    s->args.pbits = L->pbits;
    s->kfn = fsk::step_kernel_fn(s->storage, g->d_weights != nullptr, s->mode, L->udeg, s->d_shed[0] != nullptr,
                                 s->d_rates != nullptr || s->d_act != nullptr, s->lgR, L->pbits);
    if (!s->kfn) return fail(FS_ERR_DEVICE, "no step kernel for this configuration");
    s->args.col_t = L->d_col_t;
    s->args.w_t = L->d_w_t;
    return FS_OK;
}

fs_status use_plain_columns(fs_sim* s)
{
    if (!s->pack) return FS_OK;
    s->pack = false;
    if (!s->layout || s->layout->pbits == 0) return FS_OK;
    return apply_bins(s, s->heavy_deg, s->seg_edges);
}

fsi::SumArgs summary_args(const fs_sim* s, uint32_t after)
{
    fsi::SumArgs a{};
    a.iota0 = (const unsigned long long*)s->d_iota[0];
    a.iota1 = (const unsigned long long*)s->d_iota[1];
    a.ctl = s->d_ctl;
    a.summary = s->d_summary;
    a.words = s->bit_words;
    a.sum_words = s->sum_words;
    a.sum_shift = s->sum_shift;
    a.step_off = 0;
    a.after = after;
    return a;
}

uint32_t summary_grid(const fs_sim* s) { return (s->sum_words * 64u + WG - 1) / WG; }

// Rebuilds the summary of the current bitmap (after seeding or a state load;
// ctl->step must already hold the sim's step index).
hipError_t refresh_summary(fs_sim* s)
{
    if (s->mode != fsi::MODE_SUMMARY) return hipSuccess;
    fsi::SumArgs a = summary_args(s, 0);
    void* argv[] = {&a};
    return hipLaunchKernel(fsk::summary_kernel_fn(), dim3(summary_grid(s)), dim3(WG), argv, 0, s->stream);
}

// After a change of states from the host (seeding, a state load): the
// shedding values s(tau) of the infectious units, read by step `step`, and
// the live flags of every chunk for compaction.
hipError_t refresh_derived(fs_sim* s, int64_t step)
{
    const uint32_t total = (uint32_t)(s->g->n * s->R);
    hipError_t e = hipSuccess;
    // compaction: a chunk the next refresh drops is never written again, so
    // the other bitmap must hold its (all-R, zero) words too
    if (s->d_live &&
        (e = fsk::launch_rebuild_bits(s->storage, s->d_state, total, (unsigned long long*)s->d_iota[(step + 1) & 1],
                                      s->bit_words, s->stream)) != hipSuccess)
        return e;
    if (s->d_shed[0] &&
        (e = fsk::launch_rebuild_shed(s->storage, s->d_state, s->d_age, total, s->shed, s->d_shed[step & 1],
                                      s->stream)) != hipSuccess)
        return e;
    if (s->d_live &&
        (e = fsk::launch_chunk_live(s->storage, s->d_state, total, s->d_live, s->nchunks, s->stream)) != hipSuccess)
        return e;
    return refresh_hubs(s, step);
}

fsi::HeavyArgs heavy_args(const fs_sim* s)
{
    fsi::HeavyArgs h{};
    h.col_ind = s->g->d_col_ind;
    h.weights = s->g->d_weights;
    h.segs = s->d_segs;
    h.seg_part = s->d_seg_part;
    h.iota0 = s->d_iota[0];
    h.iota1 = s->d_iota[1];
    h.ctl = s->d_ctl;
    h.nseg = s->nseg;
    h.lgR = s->lgR;
    h.shed0 = s->d_shed[0];
    h.shed1 = s->d_shed[1];
    h.state = s->d_state;
    h.storage = s->storage;
    h.units = (uint32_t)((size_t)s->g->n << s->lgR);
    return h;
}


void make_seq(fs_sim* s, uint32_t r, SeqArgs& q)
{
    q.step.assign(r, s->args);
    for (uint32_t j = 0; j < r; ++j) q.step[j].step_off = j;
    // compaction: only the sequence's last step records the live flags the
    // next refresh reads
    for (uint32_t j = 0; j + 1 < r; ++j) q.step[j].live = nullptr;
    q.heavy.clear();
    if (s->nseg && !s->hub_push) {
        q.heavy.assign(r, heavy_args(s));
        for (uint32_t j = 0; j < r; ++j) q.heavy[j].step_off = j;
    }
    q.sum.clear();
    if (s->mode == fsi::MODE_SUMMARY) {
        q.sum.assign(r, summary_args(s, 1));
        for (uint32_t j = 0; j < r; ++j) q.sum[j].step_off = j;
    }
    q.ctl = s->d_ctl;
    q.part = s->d_part;
    q.G = s->G;
    q.C = 4u * (uint32_t)s->R;
    q.H = (uint32_t)s->H;
    q.r = r;
    q.hist = s->d_hist;
    q.live = s->d_live;
    q.nchunks = s->nchunks;
    q.rows = 64u >> s->lgR;
    q.n = (uint32_t)s->g->n;
    q.act = s->d_act;
    q.rates = (uint32_t*)s->d_rates;
    q.rates_words = (size_t)s->g->n * (size_t)s->R;
}

fs_status build_graph_exec(fs_sim* s, int b)
{
    SeqArgs q;
    make_seq(s, (uint32_t)b, q);
    FS_HIP(hipGraphCreate(&s->graph, 0));
    hipGraphNode_t prev = nullptr;
    auto add = [&](const void* fn, dim3 grid, dim3 block, void** argv) -> fs_status {
        hipKernelNodeParams kp{};
        kp.func = const_cast<void*>(fn);
        kp.gridDim = grid;
        kp.blockDim = block;
        kp.sharedMemBytes = 0;
        kp.kernelParams = argv;
        kp.extra = nullptr;
        hipGraphNode_t node;
        FS_HIP(hipGraphAddKernelNode(&node, s->graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp));
        prev = node;
        return FS_OK;
    };
    fs_status st;
    if (s->d_act) {
        if (q.rates) {
            void* cargv[] = {&q.rates, &q.rates_words};
            if ((st = add(fsk::clear_u32_kernel_fn(), dim3(clear_grid(q.rates_words)), dim3(256), cargv)) != FS_OK)
                return st;
        }
        void* fargv[] = {&q.live, &q.nchunks, &q.rows, &q.n, &q.act};
        if ((st = add(fsk::compact_refresh_kernel_fn(), dim3(1), dim3(fsi::WG_REFRESH), fargv)) != FS_OK) return st;
    }
    for (int j = 0; j < b; ++j) {
        if (!q.heavy.empty()) {
            void* hargv[] = {&q.heavy[j]};
            if ((st = add(s->hfn, dim3(sim_heavy_grid(s)), dim3(sim_heavy_block(s)), hargv)) != FS_OK) return st;
        }
        void* argv[] = {&q.step[j]};
        if ((st = add(s->kfn, dim3(s->G), dim3(s->tpb), argv)) != FS_OK) return st;
        if (!q.sum.empty()) {
            void* sargv[] = {&q.sum[j]};
            if ((st = add(fsk::summary_kernel_fn(), dim3(summary_grid(s)), dim3(WG), sargv)) != FS_OK) return st;
        }
    }
    void* rargv[] = {&q.ctl, &q.part, &q.G, &q.C, &q.hist, &q.H};
    if ((st = add(fsk::reduce_kernel_fn(), dim3(q.r), dim3(fsi::RED_TPB), rargv)) != FS_OK) return st;
    FS_HIP(hipGraphInstantiate(&s->exec, s->graph, nullptr, nullptr, 0));
    return FS_OK;
}

fs_status launch_sequence(fs_sim* s, uint32_t r)
{
    SeqArgs q;
    make_seq(s, r, q);
    if (s->d_act) {
        if (q.rates) {
            void* cargv[] = {&q.rates, &q.rates_words};
            FS_HIP(hipLaunchKernel(fsk::clear_u32_kernel_fn(), dim3(clear_grid(q.rates_words)), dim3(256), cargv, 0,
                                   s->stream));
        }
        void* fargv[] = {&q.live, &q.nchunks, &q.rows, &q.n, &q.act};
        FS_HIP(hipLaunchKernel(fsk::compact_refresh_kernel_fn(), dim3(1), dim3(fsi::WG_REFRESH), fargv, 0, s->stream));
    }
    for (uint32_t j = 0; j < r; ++j) {
        if (!q.heavy.empty()) {
            void* hargv[] = {&q.heavy[j]};
            FS_HIP(hipLaunchKernel(s->hfn, dim3(sim_heavy_grid(s)), dim3(sim_heavy_block(s)), hargv, 0, s->stream));
        }
        void* argv[] = {&q.step[j]};
        FS_HIP(hipLaunchKernel(s->kfn, dim3(s->G), dim3(s->tpb), argv, 0, s->stream));
        if (!q.sum.empty()) {
            void* sargv[] = {&q.sum[j]};
            FS_HIP(hipLaunchKernel(fsk::summary_kernel_fn(), dim3(summary_grid(s)), dim3(WG), sargv, 0, s->stream));
        }
    }
    void* rargv[] = {&q.ctl, &q.part, &q.G, &q.C, &q.hist, &q.H};
    FS_HIP(hipLaunchKernel(fsk::reduce_kernel_fn(), dim3(r), dim3(fsi::RED_TPB), rargv, 0, s->stream));
    return FS_OK;
}

fs_status check_seed(const fs_sim* s, int32_t replica, int64_t count, const int64_t* nodes, int32_t compartment)
{
    if (!s) return fail(FS_ERR_INVALID_ARG, "sim is NULL");
    fs_status st = check_replica(s, replica, true);
    if (st != FS_OK) return st;
    if (compartment < 0 || compartment > 3) return fail(FS_ERR_INVALID_ARG, "compartment must be in [0, 3]");
    if (count < 0) return fail(FS_ERR_INVALID_ARG, "count < 0");
    if (count == 0) return FS_OK;
    if (!nodes) return fail(FS_ERR_INVALID_ARG, "nodes is NULL");
    for (int64_t j = 0; j < count; ++j)
        if (nodes[j] < 0 || nodes[j] >= s->g->n) return fail(FS_ERR_INVALID_ARG, "seed node out of range");
    return FS_OK;
}

fs_status seed_staged(fs_sim* s, int32_t replica, const int64_t* d_nodes, int64_t count, int32_t compartment)
{
    FS_HIP(fsk::launch_seed(s->storage, s->d_state, s->d_age, d_nodes, count, s->lgR, replica, compartment,
                            s->stream));
    FS_HIP(fsk::launch_rebuild_bits(s->storage, s->d_state, (uint32_t)(s->g->n * s->R),
                                    (unsigned long long*)s->d_iota[s->step & 1], s->bit_words, s->stream));
    FS_HIP(refresh_derived(s, s->step));
    FS_HIP(refresh_summary(s));
    FS_HIP(hipStreamSynchronize(s->stream));
    return FS_OK;
}

// Switches sim s to another step variant (mode): workgroup shape and
// count, count partials, the summary buffer and the kernels.  Adaptive sims
// only move between the LDS variants, which share the workgroup count, so
// the per-workgroup rate maxima the next step folds keep their meaning.
fs_status apply_variant(fs_sim* s, int mode)
{
    if (mode == s->mode) return FS_OK;
    const size_t units = (size_t)s->g->n * (size_t)s->R;
    if (mode == fsi::MODE_RESIDENT && units > fsi::RESIDENT_BITS)
        return fail(FS_ERR_INVALID_ARG, "the resident variant holds at most 2^20 units");
    if (mode == fsi::MODE_STREAM && s->p.adaptive) return fail(FS_ERR_INVALID_ARG, "adaptive sims keep an LDS variant");
    const uint32_t tpb = mode == fsi::MODE_STREAM ? fsi::STREAM_TPB : fsi::RESIDENT_TPB;
    const size_t chunks = (units + 63) / 64;
    const size_t tiles = (chunks + tpb / 64 - 1) / (tpb / 64);
    uint32_t G;
    if (mode != fsi::MODE_STREAM) {
        int cus = 0;
        FS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device));
        s->cus = (uint32_t)std::max(cus, 1);
        G = (uint32_t)std::min<size_t>(tiles, s->cus);
    } else {
        G = (uint32_t)std::min<size_t>(tiles, fsi::max_step_grid(s->R));
    }
    drop_graph_exec(s);
    if (G != s->G) {
        // count partials are written and reduced within one launch sequence:
        // nothing of them outlives it
        sim_free(s, s->d_part);
        s->d_part = nullptr;
        FS_HIP(sim_alloc(s, (void**)&s->d_part, (size_t)s->chunk * G * (size_t)s->R * 4 * sizeof(uint32_t)));
    }
    if (mode == fsi::MODE_SUMMARY && !s->d_summary)
        FS_HIP(sim_alloc(s, (void**)&s->d_summary, ((size_t)s->sum_bits + 511) / 512 * 64));
    s->mode = mode;
    s->tpb = tpb;
    s->G = G;
    s->args.part = s->d_part;
    s->args.summary = (const uint32_t*)s->d_summary;
    const bool weighted = s->g->d_weights != nullptr, shed = s->d_shed[0] != nullptr;
    s->kfn = fsk::step_kernel_fn(s->storage, weighted, mode, s->layout ? s->layout->udeg : -1, shed,
                                 s->d_rates != nullptr || s->d_act != nullptr, s->lgR,
                                 s->layout ? s->layout->pbits : 0);
    s->hfn = fsk::heavy_kernel_fn(weighted, shed, mode == fsi::MODE_RESIDENT);
    if (!s->kfn || !s->hfn) return fail(FS_ERR_DEVICE, "no step kernel for this configuration");
    FS_HIP(refresh_summary(s));
    return FS_OK;
}

// FNV-1a over a run's signature: what the fastest configuration depends on.
struct Fnv {
    uint64_t h = 1469598103934665603ull;
    void add(const void* p, size_t n)
    {
        const unsigned char* b = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    }
    template <class T>
    void put(T v) { add(&v, sizeof v); }
};

uint64_t tune_signature(const fs_sim* s)
{
    const fs_graph* g = s->g;
    Fnv f;
    const char* ver = "flashspread-tune-1";
    f.add(ver, std::strlen(ver));
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device);
    f.put<int32_t>(cus);
    f.put<int64_t>(g->n);
    f.put<int64_t>(g->nnz);
    f.put<int32_t>(s->R);
    f.put<int32_t>(s->storage);
    f.put<int32_t>(g->d_weights != nullptr);
    f.put<int32_t>(s->p.shedding);
    f.put<int32_t>(s->p.adaptive != 0);
    f.put<int32_t>(s->d_act != nullptr);
    f.put<int32_t>(s->d_rates != nullptr);
    // degree histogram: (degree, count) for every degree present
    std::vector<int64_t> hist((size_t)g->max_degree + 1, 0);
    for (int64_t i = 0; i < g->n; ++i) ++hist[(size_t)(g->h_row_ptr[(size_t)i + 1] - g->h_row_ptr[(size_t)i])];
    for (size_t d = 0; d < hist.size(); ++d)
        if (hist[d]) {
            f.put<int64_t>((int64_t)d);
            f.put<int64_t>(hist[d]);
        }
    return f.h;
}

// A cached choice: the last line of the file with this signature.
bool cache_lookup(const char* path, uint64_t sig, int* mode, int32_t* hd, int32_t* se)
{
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char line[256];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        unsigned long long k = 0;
        int v = 0, h = 0, c = 0;
        if (std::sscanf(line, "%llx variant=%d heavy_degree=%d segment_edges=%d", &k, &v, &h, &c) == 4 && k == sig &&
            v >= 1 && v <= 3 && h >= -1 && c >= 64 && c <= (1 << 20)) {
            *mode = v - 1;
            *hd = h;
            *se = c;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

fs_status cache_store(const char* path, uint64_t sig, int mode, int32_t hd, int32_t se, double us)
{
    FILE* f = std::fopen(path, "a");
    if (!f) return fail(FS_ERR_INVALID_ARG, std::string("cannot append to the tune cache ") + path);
    std::fprintf(f, "%016llx variant=%d heavy_degree=%d segment_edges=%d us_per_step=%.3f\n",
                 (unsigned long long)sig, mode + 1, hd, se, us);
    const bool ok = std::fclose(f) == 0;
    return ok ? FS_OK : fail(FS_ERR_INVALID_ARG, std::string("cannot write the tune cache ") + path);
}

fs_status autotune(fs_sim* s, const fs_tune_params& tp, fs_tune_result* out)
{
    if (!s) return fail(FS_ERR_INVALID_ARG, "sim is NULL");
    if (s->batch) return fail(FS_ERR_BUSY, "sim belongs to a batch");
    const int32_t trial_steps = tp.trial_steps;
    if (trial_steps < 1 || trial_steps > 4096) return fail(FS_ERR_INVALID_ARG, "trial_steps must be in [1, 4096]");
    DeviceGuard dg(s->device);
    *out = fs_tune_result{};
    out->signature = tune_signature(s);
    if (tp.cache_path) {
        int mode = 0;
        int32_t hd = 0, se = 0;
        if (cache_lookup(tp.cache_path, out->signature, &mode, &hd, &se) && (tp.variants || mode == s->mode)) {
            FS_HIP(hipStreamSynchronize(s->stream));
            fs_status st = apply_variant(s, mode);
            if (st == FS_OK) st = apply_bins(s, hd, se);
            if (st != FS_OK) return st;
            FS_HIP(hipStreamSynchronize(s->stream));
            out->variant = s->mode + 1;
            out->heavy_degree = s->heavy_deg;
            out->segment_edges = s->seg_edges;
            out->from_cache = 1;
            return FS_OK;
        }
    }
    FS_HIP(hipStreamSynchronize(s->stream));
    const size_t units = (size_t)s->g->n * s->R;
    // snapshot everything a step changes (cf. Algorithm 2: snapshot, warm up, restore)
    struct Buf {
        void* live;
        size_t bytes;
        DevBuf copy;
    };
    Buf bufs[] = {{s->d_state, units * state_bytes(s->storage), {}},
                  {s->d_age, units * age_bytes(s->storage), {}},
                  {s->d_iota[0], (size_t)s->bit_words * 8, {}},
                  {s->d_iota[1], (size_t)s->bit_words * 8, {}},
                  {s->d_ctl, sizeof(fsi::Ctl), {}},
                  {s->d_hist, (size_t)s->H * s->R * 4 * sizeof(uint32_t), {}},
                  {s->d_lam_part, 2 * (size_t)s->G * sizeof(float), {}},
                  {s->d_shed[0], (size_t)s->g->n * s->R * shed_bytes(s->storage), {}},
                  {s->d_shed[1], (size_t)s->g->n * s->R * shed_bytes(s->storage), {}},
                  {s->d_live, s->live_bytes, {}},
                  {s->d_act, (2 + (size_t)s->nchunks) * sizeof(uint32_t), {}},
                  {s->d_dt_hist, (size_t)s->H * sizeof(float), {}}};
    for (auto& b : bufs) {
        if (!b.live) continue;
        FS_HIP(dev_alloc(&b.copy.p, b.bytes));
        FS_HIP(hipMemcpyAsync(b.copy.p, b.live, b.bytes, hipMemcpyDeviceToDevice, s->stream));
    }
    // candidates: the entry configuration first, then the other variants and bins
    std::vector<int> modes{s->mode};
    if (tp.variants) {
        for (int m : {fsi::MODE_RESIDENT, fsi::MODE_SUMMARY, fsi::MODE_STREAM}) {
            if (m == s->mode) continue;
            if (m == fsi::MODE_RESIDENT && units > fsi::RESIDENT_BITS) continue;
            if (m == fsi::MODE_STREAM && s->p.adaptive) continue;
            modes.push_back(m);
        }
    }
    const bool pushed = s->g->d_weights == nullptr && s->d_shed[0] == nullptr;
    std::vector<std::pair<int32_t, int32_t>> bins{{s->heavy_deg, s->seg_edges}};
    auto add_bins = [&](int32_t t, int32_t c) {
        if (std::find(bins.begin(), bins.end(), std::make_pair(t, c)) == bins.end()) bins.push_back({t, c});
    };
    // (thresholds at or above the largest degree bin nothing: the same run as
    // no bins, which is a candidate when the entry bins any row)
    if (s->nseg) add_bins(-1, 512);
    for (int32_t t : {8, 12, 16, 24, 32, 64, 128, 256}) {
        if (t >= s->g->max_degree) continue;
        if (pushed) add_bins(t, s->seg_edges); // pushed rows read no segments
        else
            for (int32_t c : {256, 1024}) add_bins(t, c);
    }
    hipEvent_t e0, e1;
    FS_HIP(hipEventCreate(&e0));
    FS_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    int best_mode = s->mode;
    std::pair<int32_t, int32_t> best = bins[0];
    fs_status st = FS_OK;
    int trials = 0;
    for (int m : modes) {
        if (st != FS_OK) break;
        if ((st = apply_variant(s, m)) != FS_OK) break;
        for (const auto& c : bins) {
            if ((st = apply_bins(s, c.first, c.second)) != FS_OK) break;
            // (the summary of the restored bitmap)
            if (refresh_summary(s) != hipSuccess) { st = fail(FS_ERR_DEVICE, "summary"); break; }
            // one untimed warm-up step, then the timed trial, then restore
            uint32_t done = 0;
            if ((st = launch_sequence(s, 1)) != FS_OK) break;
            if (hipEventRecord(e0, s->stream) != hipSuccess) { st = fail(FS_ERR_DEVICE, "event"); break; }
            while (done < (uint32_t)trial_steps && st == FS_OK) {
                const uint32_t r = std::min<uint32_t>(s->chunk, (uint32_t)trial_steps - done);
                st = launch_sequence(s, r);
                done += r;
            }
            if (st != FS_OK) break;
            float ms = 0.0f;
            if (hipEventRecord(e1, s->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = fail(FS_ERR_DEVICE, "event timing");
                break;
            }
            if (trials == 0) out->entry_us_per_step = 1e3 * ms / trial_steps;
            ++trials;
            if (ms < best_ms) {
                best_ms = ms;
                best_mode = m;
                best = c;
            }
            for (auto& b : bufs)
                if (b.live && hipMemcpyAsync(b.live, b.copy.p, b.bytes, hipMemcpyDeviceToDevice, s->stream) != hipSuccess) {
                    st = fail(FS_ERR_DEVICE, "restore");
                    break;
                }
            if (st != FS_OK) break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (auto& b : bufs)
        if (b.live) (void)hipMemcpyAsync(b.live, b.copy.p, b.bytes, hipMemcpyDeviceToDevice, s->stream);
    FS_HIP(hipStreamSynchronize(s->stream));
    if (st != FS_OK) return st;
    // the choice, on the restored state (bins recount pushed pressure, the
    // summary is rebuilt from the restored bitmap)
    if ((st = apply_variant(s, best_mode)) != FS_OK) return st;
    if ((st = apply_bins(s, best.first, best.second)) != FS_OK) return st;
    FS_HIP(refresh_summary(s));
    FS_HIP(hipStreamSynchronize(s->stream));
    out->variant = s->mode + 1;
    out->heavy_degree = s->heavy_deg;
    out->segment_edges = s->seg_edges;
    out->trials = trials;
    out->us_per_step = 1e3 * best_ms / trial_steps;
    if (tp.cache_path)
        return cache_store(tp.cache_path, out->signature, s->mode, s->heavy_deg, s->seg_edges, out->us_per_step);
    return FS_OK;
}

} // namespace fsr

using namespace fsr;

#define FS_GUARD_BEGIN try {
#define FS_GUARD_END                                                        \
    }                                                                       \
    catch (const std::bad_alloc&) { return fail(FS_ERR_OUT_OF_MEMORY, "host allocation failed"); } \
    catch (const std::exception& e) { return fail(FS_ERR_DEVICE, e.what()); }                   \
    catch (...) { return fail(FS_ERR_DEVICE, "unknown exception"); }

extern "C" {

const char* fs_version(void) { return "flashspread-hip 0.1 (gfx950)"; }

fs_status fs_set_allocator(fs_alloc_fn alloc, fs_free_fn free_fn, void* ctx)
{
    if ((alloc == nullptr) != (free_fn == nullptr))
        return fail(FS_ERR_INVALID_ARG, "give both alloc and free, or neither");
    std::lock_guard<std::mutex> lk(g_hook_mu);
    g_hook.alloc = alloc;
    g_hook.free = free_fn;
    g_hook.ctx = alloc ? ctx : nullptr;
    return FS_OK;
}

const char* fs_status_string(fs_status s)
{
    switch (s) {
    case FS_OK: return "FS_OK";
    case FS_ERR_INVALID_ARG: return "FS_ERR_INVALID_ARG";
    case FS_ERR_INVALID_CSR: return "FS_ERR_INVALID_CSR";
    case FS_ERR_OUT_OF_MEMORY: return "FS_ERR_OUT_OF_MEMORY";
    case FS_ERR_DEVICE: return "FS_ERR_DEVICE";
    case FS_ERR_BUSY: return "FS_ERR_BUSY";
    case FS_ERR_BUDGET: return "FS_ERR_BUDGET";
    default: return "FS_ERR_UNKNOWN";
    }
}

const char* fs_last_error(void) { return g_err.c_str(); }

fs_status fs_graph_create(int64_t n, const int32_t* row_ptr, const int32_t* col_ind, const float* weights,
                          fs_graph** out)
{
    FS_GUARD_BEGIN
    if (!out) return fail(FS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 1 || n >= (int64_t)1 << 31) return fail(FS_ERR_INVALID_ARG, "n must satisfy 1 <= n < 2^31");
    if (!row_ptr) return fail(FS_ERR_INVALID_ARG, "row_ptr is NULL");
    if (row_ptr[0] != 0) return fail(FS_ERR_INVALID_CSR, "row_ptr[0] must be 0");
    int32_t maxd = 0, mind = INT32_MAX;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t d = (int64_t)row_ptr[i + 1] - (int64_t)row_ptr[i];
        if (d < 0)
            return fail(FS_ERR_INVALID_CSR, "row_ptr decreases at row " + std::to_string(i));
        if (d > maxd) maxd = (int32_t)d;
        if (d < mind) mind = (int32_t)d;
    }
    const int64_t nnz = row_ptr[n];
    if (nnz > 0 && !col_ind) return fail(FS_ERR_INVALID_ARG, "col_ind is NULL");
    for (int64_t e = 0; e < nnz; ++e)
        if (col_ind[e] < 0 || (int64_t)col_ind[e] >= n)
            return fail(FS_ERR_INVALID_CSR, "col_ind[" + std::to_string(e) + "] out of range");
    int dev = 0;
    FS_HIP(hipGetDevice(&dev));
    fs_graph* g = new fs_graph();
    g->device = dev;
    g->n = n;
    g->nnz = nnz;
    g->max_degree = maxd;
    g->min_degree = mind;
    g->mean_degree = (double)nnz / (double)n;
    if (mind == maxd) {
        g->h_row_ptr.assign(row_ptr, row_ptr + n + 1);
        if (nnz) g->h_col_ind.assign(col_ind, col_ind + nnz);
        if (weights && nnz) g->h_weights.assign(weights, weights + nnz);
    } else {
        // degree-sorted internal order (counting sort, stable): rows keep
        // their edges in the caller's order, columns are relabelled
        std::vector<int64_t> cnt((size_t)maxd + 2, 0);
        for (int64_t i = 0; i < n; ++i) ++cnt[(size_t)(row_ptr[i + 1] - row_ptr[i]) + 1];
        for (size_t d = 1; d < cnt.size(); ++d) cnt[d] += cnt[d - 1];
        g->h_orig.resize((size_t)n);
        g->h_inv.resize((size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t pos = cnt[(size_t)(row_ptr[i + 1] - row_ptr[i])]++;
            g->h_orig[(size_t)pos] = (int32_t)i;
            g->h_inv[(size_t)i] = (int32_t)pos;
        }
        g->h_row_ptr.resize((size_t)n + 1);
        g->h_row_ptr[0] = 0;
        for (int64_t j = 0; j < n; ++j) {
            const int32_t i = g->h_orig[(size_t)j];
            g->h_row_ptr[(size_t)j + 1] = g->h_row_ptr[(size_t)j] + (row_ptr[i + 1] - row_ptr[i]);
        }
        g->h_col_ind.resize((size_t)nnz);
        if (weights) g->h_weights.resize((size_t)nnz);
        for (int64_t j = 0; j < n; ++j) {
            const int32_t i = g->h_orig[(size_t)j];
            int32_t o = g->h_row_ptr[(size_t)j];
            for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e, ++o) {
                g->h_col_ind[(size_t)o] = g->h_inv[(size_t)col_ind[e]];
                if (weights) g->h_weights[(size_t)o] = weights[e];
            }
        }
    }
    std::vector<int32_t> orig_dev((size_t)n);
    for (int64_t j = 0; j < n; ++j) orig_dev[(size_t)j] = g->h_orig.empty() ? (int32_t)j : g->h_orig[(size_t)j];
    auto cleanup = [&](fs_status st) {
        dev_free(g->d_row_ptr);
        dev_free(g->d_col_ind);
        dev_free(g->d_weights);
        dev_free(g->d_orig);
        delete g;
        return st;
    };
    hipError_t e;
    if ((e = dev_alloc((void**)&g->d_row_ptr, sizeof(int32_t) * (size_t)(n + 1))) != hipSuccess ||
        (e = dev_alloc((void**)&g->d_col_ind, sizeof(int32_t) * (size_t)nnz)) != hipSuccess ||
        (e = dev_alloc((void**)&g->d_orig, sizeof(int32_t) * (size_t)n)) != hipSuccess ||
        (weights && (e = dev_alloc((void**)&g->d_weights, sizeof(float) * (size_t)nnz)) != hipSuccess))
        return cleanup(fail(FS_ERR_OUT_OF_MEMORY, std::string("device allocation: ") + hipGetErrorString(e)));
    if ((e = hipMemcpy(g->d_row_ptr, g->h_row_ptr.data(), sizeof(int32_t) * (size_t)(n + 1), hipMemcpyHostToDevice)) !=
            hipSuccess ||
        (nnz && (e = hipMemcpy(g->d_col_ind, g->h_col_ind.data(), sizeof(int32_t) * (size_t)nnz,
                               hipMemcpyHostToDevice)) != hipSuccess) ||
        (e = hipMemcpy(g->d_orig, orig_dev.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice)) != hipSuccess ||
        (weights && nnz &&
         (e = hipMemcpy(g->d_weights, g->h_weights.data(), sizeof(float) * (size_t)nnz, hipMemcpyHostToDevice)) !=
             hipSuccess))
        return cleanup(fail(FS_ERR_DEVICE, std::string("upload: ") + hipGetErrorString(e)));
    *out = g;
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_graph_destroy(fs_graph* g)
{
    FS_GUARD_BEGIN
    if (!g) return fail(FS_ERR_INVALID_ARG, "graph is NULL");
    if (g->users.load() > 0) return fail(FS_ERR_BUSY, "graph is still used by a sim");
    DeviceGuard dg(g->device);
    dev_free(g->d_row_ptr);
    dev_free(g->d_col_ind);
    dev_free(g->d_weights);
    dev_free(g->d_orig);
    dev_free(g->d_out_ptr);
    dev_free(g->d_out_ind);
    delete g;
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_graph_get_info(const fs_graph* g, fs_graph_info* out)
{
    if (!g || !out) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    out->n = g->n;
    out->nnz = g->nnz;
    out->max_degree = g->max_degree;
    out->weighted = g->d_weights != nullptr;
    out->mean_degree = g->mean_degree;
    return FS_OK;
}

fs_status fs_sim_create(fs_graph* g, const fs_sim_params* p, fs_sim** out)
{
    FS_GUARD_BEGIN
    if (!out) return fail(FS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!g || !p) return fail(FS_ERR_INVALID_ARG, "NULL graph or params");
    if (p->storage != FS_STORAGE_FP32 && p->storage != FS_STORAGE_COMPACT)
        return fail(FS_ERR_INVALID_ARG, "unknown storage");
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(FS_ERR_INVALID_ARG, "dt must be finite and > 0");
    if (!(p->beta >= 0.0) || !std::isfinite(p->beta)) return fail(FS_ERR_INVALID_ARG, "beta must be finite and >= 0");
    const int R = p->n_replicas;
    if (R < 1 || R > 64 || (R & (R - 1))) return fail(FS_ERR_INVALID_ARG, "n_replicas must be a power of two in [1, 64]");
    if ((int64_t)g->n * R >= (int64_t)1 << 31) return fail(FS_ERR_INVALID_ARG, "n * n_replicas must be below 2^31");
    if (p->history_len < 0 || p->history_len == 1) return fail(FS_ERR_INVALID_ARG, "history_len must be 0 or >= 2");
    if (p->steps_per_graph < 0 || p->steps_per_graph > 100000)
        return fail(FS_ERR_INVALID_ARG, "steps_per_graph out of range");
    if (p->heavy_degree < -1) return fail(FS_ERR_INVALID_ARG, "heavy_degree must be -1, 0 or positive");
    if (p->columns != FS_COLUMNS_AUTO && p->columns != FS_COLUMNS_PLAIN)
        return fail(FS_ERR_INVALID_ARG, "columns must be FS_COLUMNS_AUTO or FS_COLUMNS_PLAIN");
    if (p->segment_edges != 0 && (p->segment_edges < 64 || p->segment_edges > (1 << 20)))
        return fail(FS_ERR_INVALID_ARG, "segment_edges must be 0 or in [64, 2^20]");
    if (p->adaptive) {
        if (p->storage != FS_STORAGE_FP32)
            return fail(FS_ERR_INVALID_ARG, "adaptive steps need FP32 storage (ages in days)");
        if (p->variant == 1) return fail(FS_ERR_INVALID_ARG, "adaptive steps need variant 0, 2 or 3");
        if (!(p->epsilon > 0.0) || !std::isfinite(p->epsilon))
            return fail(FS_ERR_INVALID_ARG, "epsilon must be finite and > 0");
        if (!(p->delta >= 0.0) || !std::isfinite(p->delta))
            return fail(FS_ERR_INVALID_ARG, "delta must be finite and >= 0");
    }
    HazardDev hz[2];
    fs_status st;
    if ((st = prep_hazard(p->ei, p->storage, p->dt, &hz[0], "ei")) != FS_OK) return st;
    if ((st = prep_hazard(p->ir, p->storage, p->dt, &hz[1], "ir")) != FS_OK) return st;
    fsi::ShedDev shed;
    if ((st = prep_shed(p->shedding, p->shed_law, p->shed_scale, p->storage, p->dt, &shed)) != FS_OK) return st;
    const bool shedding = p->shedding != FS_SHED_CONSTANT;
    if (shedding && (int64_t)g->n * R >= (int64_t)1 << 29)
        return fail(FS_ERR_INVALID_ARG, "age-dependent shedding needs n * n_replicas below 2^29");

    DeviceGuard dg(g->device);
    fs_sim* s = new fs_sim();
    s->g = g;
    g->users.fetch_add(1);
    s->p = *p;
    s->device = g->device;
    s->R = R;
    while ((1 << s->lgR) < R) ++s->lgR;
    s->storage = p->storage;
    s->H = p->history_len ? p->history_len : 1024;
    const size_t units = (size_t)g->n * (size_t)R;
    hipError_t e = hipSuccess;
    auto bad = [&](hipError_t err, const char* what) {
        release_sim(s);
        return fail(err == hipErrorOutOfMemory ? FS_ERR_OUT_OF_MEMORY : FS_ERR_DEVICE,
                    std::string(what) + ": " + hipGetErrorString(err));
    };
    if (p->stream) {
        s->stream = (hipStream_t)p->stream;
    } else {
        if ((e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) != hipSuccess)
            return bad(e, "stream");
        s->own_stream = true;
    }
    if (p->variant < 0 || p->variant > 3) {
        release_sim(s);
        return fail(FS_ERR_INVALID_ARG, "variant must be 0 (auto), 1 (stream), 2 (resident) or 3 (summary)");
    }
    const bool fits_lds = units <= fsi::RESIDENT_BITS;
    if (p->variant == 2 && !fits_lds) {
        release_sim(s);
        return fail(FS_ERR_INVALID_ARG, "the resident variant holds at most 2^20 units (n * n_replicas)");
    }
    // automatic choice (measured on MI355X): the LDS bitmap when it fits; else
    // the LDS summary for adaptive steps, for bitmaps beyond 8 MB (the
    // summary screens random reads that would miss the L2), and for
    // uniform-degree graphs with at most 4 replicas; else the streaming
    // variant, whose higher occupancy wins once replicas share bitmap words
    const bool uniform = g->min_degree == g->max_degree && g->max_degree <= fsi::UNIFORM_MAX_DEG;
    const bool summary_auto = p->adaptive || bitmap_words(units) * 8 > ((size_t)8 << 20) || (uniform && R <= 4);
    s->mode = p->variant == 1 ? fsi::MODE_STREAM
            : p->variant == 2 ? fsi::MODE_RESIDENT
            : p->variant == 3 ? fsi::MODE_SUMMARY
            : fits_lds ? fsi::MODE_RESIDENT
            : summary_auto ? fsi::MODE_SUMMARY : fsi::MODE_STREAM;
    // summary groups: the fewest 32-bit bitmap words per group, a power of
    // two, whose groups fit SUMMARY_BITS (one word per group up to 2^25 units)
    {
        const size_t words32 = (units + 31) / 32;
        s->sum_shift = 0;
        while (((words32 + ((size_t)1 << s->sum_shift) - 1) >> s->sum_shift) > fsi::SUMMARY_BITS) ++s->sum_shift;
        s->sum_bits = (uint32_t)((words32 + ((size_t)1 << s->sum_shift) - 1) >> s->sum_shift);
    }
    s->sum_words = (s->sum_bits + 63) / 64;
    s->tpb = s->mode == fsi::MODE_STREAM ? fsi::STREAM_TPB : fsi::RESIDENT_TPB;
    const size_t chunks = (units + 63) / 64;
    const size_t tiles = (chunks + s->tpb / 64 - 1) / (s->tpb / 64); // workgroups with work
    if (s->mode != fsi::MODE_STREAM) {
        int cus = 0;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, s->device)) != hipSuccess)
            return bad(e, "device attribute");
        s->G = (uint32_t)std::min<size_t>(tiles, (size_t)std::max(cus, 1));
        s->cus = (uint32_t)std::max(cus, 1);
    } else {
        s->G = (uint32_t)std::min<size_t>(tiles, fsi::max_step_grid(R));
    }
    s->bit_words = (uint32_t)bitmap_words(units);
    s->nchunks = (uint32_t)chunks;
    s->live_bytes = (chunks + fsi::LIVE_TILE - 1) / fsi::LIVE_TILE * fsi::LIVE_TILE;
    s->shed = shed;
    s->chunk = (uint32_t)std::max(p->steps_per_graph, 64);
    const size_t hist_words = (size_t)s->H * R * 4;
    const size_t part_words = (size_t)s->chunk * s->G * R * 4;
    keep_pool(s->device);
    if ((e = sim_alloc(s, &s->d_state, units * state_bytes(s->storage))) != hipSuccess ||
        (e = sim_alloc(s, &s->d_age, units * age_bytes(s->storage))) != hipSuccess ||
        (e = sim_alloc(s, &s->d_iota[0], (size_t)s->bit_words * 8)) != hipSuccess ||
        (e = sim_alloc(s, &s->d_iota[1], (size_t)s->bit_words * 8)) != hipSuccess ||
        (p->record_rates && (e = sim_alloc(s, (void**)&s->d_rates, units * sizeof(float))) != hipSuccess) ||
        (e = sim_alloc(s, (void**)&s->d_ctl, sizeof(fsi::Ctl))) != hipSuccess ||
        (e = sim_alloc(s, (void**)&s->d_hist, hist_words * sizeof(uint32_t))) != hipSuccess ||
        (e = sim_alloc(s, (void**)&s->d_part, part_words * sizeof(uint32_t))) != hipSuccess ||
        (e = sim_alloc(s, (void**)&s->d_rc_part, RC_GRID * 4 * sizeof(uint32_t))) != hipSuccess ||
        (e = sim_alloc(s, (void**)&s->d_cnt4, 4 * sizeof(uint32_t))) != hipSuccess ||
        (s->mode == fsi::MODE_SUMMARY &&
         (e = sim_alloc(s, (void**)&s->d_summary, ((size_t)s->sum_bits + 511) / 512 * 64)) != hipSuccess) ||
        (p->adaptive && ((e = sim_alloc(s, (void**)&s->d_lam_part, 2 * (size_t)s->G * sizeof(float))) != hipSuccess ||
                         (e = sim_alloc(s, (void**)&s->d_dt_hist, (size_t)s->H * sizeof(float))) != hipSuccess)) ||
        (shedding && ((e = sim_alloc(s, (void**)&s->d_shed[0], units * shed_bytes(s->storage))) != hipSuccess ||
                      (e = sim_alloc(s, (void**)&s->d_shed[1], units * shed_bytes(s->storage))) != hipSuccess)) ||
        (p->compaction && ((e = sim_alloc(s, (void**)&s->d_live, s->live_bytes)) != hipSuccess ||
                           (e = sim_alloc(s, (void**)&s->d_act, (2 + chunks) * sizeof(uint32_t))) != hipSuccess)))
        return bad(e, "device allocation");
    if ((e = hipMemsetAsync(s->d_state, 0, units * state_bytes(s->storage), s->stream)) != hipSuccess ||
        (e = hipMemsetAsync(s->d_age, 0, units * age_bytes(s->storage), s->stream)) != hipSuccess ||
        (e = hipMemsetAsync(s->d_iota[0], 0, (size_t)s->bit_words * 8, s->stream)) != hipSuccess ||
        (e = hipMemsetAsync(s->d_iota[1], 0, (size_t)s->bit_words * 8, s->stream)) != hipSuccess ||
        (s->d_rates && (e = hipMemsetAsync(s->d_rates, 0, units * sizeof(float), s->stream)) != hipSuccess) ||
        (e = hipMemsetAsync(s->d_ctl, 0, sizeof(fsi::Ctl), s->stream)) != hipSuccess ||
        (e = hipMemsetAsync(s->d_hist, 0, hist_words * sizeof(uint32_t), s->stream)) != hipSuccess ||
        (s->d_summary &&
         (e = hipMemsetAsync(s->d_summary, 0, ((size_t)s->sum_bits + 511) / 512 * 64, s->stream)) != hipSuccess) ||
        (s->d_shed[0] && (e = hipMemsetAsync(s->d_shed[0], 0, units * shed_bytes(s->storage), s->stream)) != hipSuccess) ||
        (s->d_shed[1] && (e = hipMemsetAsync(s->d_shed[1], 0, units * shed_bytes(s->storage), s->stream)) != hipSuccess) ||
        // every unit starts in S: every chunk is live; the padding never is
        (s->d_live && (e = hipMemsetAsync(s->d_live, 0, s->live_bytes, s->stream)) != hipSuccess) ||
        (s->d_live && (e = hipMemsetAsync(s->d_live, 1, chunks, s->stream)) != hipSuccess) ||
        (s->d_act && (e = hipMemsetAsync(s->d_act, 0, (2 + chunks) * sizeof(uint32_t), s->stream)) != hipSuccess) ||
        (e = hipStreamSynchronize(s->stream)) != hipSuccess)
        return bad(e, "initialisation");

    StepArgs& a = s->args;
    a.row_ptr = g->d_row_ptr;
    a.col_ind = g->d_col_ind;
    a.weights = g->d_weights;
    a.state = s->d_state;
    a.age = s->d_age;
    a.iota0 = s->d_iota[0];
    a.iota1 = s->d_iota[1];
    a.rates = s->d_rates;
    a.ctl = s->d_ctl;
    a.part = s->d_part;
    a.n = (int32_t)g->n;
    a.lgR = s->lgR;
    a.step_off = 0;
    a.sum_shift = s->sum_shift;
    a.adaptive = p->adaptive ? 1 : 0;
    a.lam_part = s->d_lam_part;
    a.dt_hist = s->d_dt_hist;
    a.eps = (float)p->epsilon;
    a.delta = (float)p->delta;
    a.hist_len = (uint32_t)s->H;
    a.summary = (const uint32_t*)s->d_summary;
    a.sum_bits = s->sum_bits;
    a.same_kind = hz[0].kind == hz[1].kind;
    a.hz[0] = hz[0];
    a.hz[1] = hz[1];
    fsi::LawsDev laws{};
    laws.hz[0] = hz[0];
    laws.hz[1] = hz[1];
    laws.shed = shed;
    if ((e = sim_alloc(s, (void**)&s->d_laws, sizeof(fsi::LawsDev))) != hipSuccess ||
        (e = hipMemcpyAsync(s->d_laws, &laws, sizeof(fsi::LawsDev), hipMemcpyHostToDevice, s->stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s->stream)) != hipSuccess)
        return bad(e, "hazard laws");
    // (the laws sit at the start of the block)
    a.hz_dev = (const fsi::HazardDev*)s->d_laws;
    a.shed_dev = (const fsi::ShedDev*)((const char*)s->d_laws + offsetof(fsi::LawsDev, shed));
    a.beta = (float)p->beta;
    a.dt = (float)p->dt;
    a.key0 = (uint32_t)p->seed;
    a.key1 = (uint32_t)(p->seed >> 32);
    a.shed0 = s->d_shed[0];
    a.shed1 = s->d_shed[1];
    a.act = s->d_act;
    a.live = s->d_live;
    if (!p->adaptive) {
        // the hazard table: the ages fixed steps reach from 0, then both
        // laws' hazards there (on the device, by the step's own code)
        std::vector<float4> tab(fsi::HTAB_LEN);
        float x = 0.0f;
        for (uint32_t m = 0; m < fsi::HTAB_LEN; ++m) {
            tab[m] = make_float4(s->storage == 0 ? x : (float)m, 0.0f, 0.0f, 0.0f);
            x = x + a.dt;
        }
        if ((e = sim_alloc(s, (void**)&s->d_htab, tab.size() * sizeof(float4))) != hipSuccess ||
            (e = hipMemcpyAsync(s->d_htab, tab.data(), tab.size() * sizeof(float4), hipMemcpyHostToDevice,
                                s->stream)) != hipSuccess ||
            (e = fsk::launch_hazard_table(a.hz_dev, a.same_kind, s->d_htab, fsi::HTAB_LEN, s->stream)) != hipSuccess ||
            (e = hipStreamSynchronize(s->stream)) != hipSuccess)
            return bad(e, "hazard table");
        a.htab = s->d_htab;
        a.htab_len = fsi::HTAB_LEN;
        a.htab_inv = s->storage == 0 ? 1.0f / a.dt : 1.0f;
    }
    s->kfn = fsk::step_kernel_fn(s->storage, g->d_weights != nullptr, s->mode, -1, shedding,
                                 s->d_rates != nullptr || s->d_act != nullptr, s->lgR, 0);
    s->hfn = fsk::heavy_kernel_fn(g->d_weights != nullptr, shedding, s->mode == fsi::MODE_RESIDENT);
    s->pack = packing_allowed(g, p);
    if (!s->kfn || !s->hfn) {
        release_sim(s);
        return fail(FS_ERR_DEVICE, "no step kernel for this configuration");
    }
    {
        const int32_t hd = p->heavy_degree == 0 ? 64 : p->heavy_degree;
        const int32_t se = p->segment_edges == 0 ? 512 : p->segment_edges;
        fs_status bst = apply_bins(s, hd, se);
        if (bst != FS_OK) {
            const std::string msg = g_err;
            release_sim(s);
            return fail(bst, msg);
        }
    }
    *out = s;
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_sim_destroy(fs_sim* s)
{
    FS_GUARD_BEGIN
    if (!s) return fail(FS_ERR_INVALID_ARG, "sim is NULL");
    if (s->batch) return fail(FS_ERR_BUSY, "sim belongs to a batch: remove it first");
    DeviceGuard dg(s->device);
    hipError_t e = hipStreamSynchronize(s->stream);
    release_sim(s);
    if (e != hipSuccess) return fail(FS_ERR_DEVICE, std::string("pending work failed: ") + hipGetErrorString(e));
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_sim_seed(fs_sim* s, int32_t replica, int64_t count, const int64_t* nodes, int32_t compartment)
{
    FS_GUARD_BEGIN
    fs_status st = check_seed(s, replica, count, nodes, compartment);
    if (st != FS_OK || count == 0) return st;
    DeviceGuard dg(s->device);
    // stream-ordered staging buffer: allocating and freeing it does not wait
    // for work queued on other streams
    std::vector<int64_t> internal;
    if (!s->g->h_inv.empty()) {
        internal.resize((size_t)count);
        for (int64_t j = 0; j < count; ++j) internal[(size_t)j] = s->g->h_inv[(size_t)nodes[j]];
        nodes = internal.data();
    }
    StreamBuf tmp(s->stream);
    FS_HIP(hipMallocAsync(&tmp.p, sizeof(int64_t) * (size_t)count, s->stream));
    FS_HIP(hipMemcpyAsync(tmp.p, nodes, sizeof(int64_t) * (size_t)count, hipMemcpyHostToDevice, s->stream));
    return seed_staged(s, replica, (const int64_t*)tmp.p, count, compartment);
    FS_GUARD_END
}

} // extern "C"

// Seed-list staging of fs_sim_seed_noalloc: a fixed device array (each GPU
// the library runs on holds its own copy until the process ends) instead of
// a stream-ordered allocation per call.  Host code never passes the array's
// name to a kernel or a copy: on the host it is only a stand-in symbol, and
// the device address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) int64_t scratch[FS_SEED_NOALLOC_MAX];

namespace fsr {

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_DEVICES] = {};

// The device address of `scratch` on the current device `dev`, looked up
// once per device.
fs_status scratch_address(int dev, int64_t** out)
{
    if (dev < 0 || dev >= SCRATCH_DEVICES) return fail(FS_ERR_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FS_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = (int64_t*)g_scratch_ptr[dev];
    return FS_OK;
}

} // namespace fsr

extern "C" {

fs_status fs_sim_seed_noalloc(fs_sim* s, int32_t replica, int64_t count, const int64_t* nodes, int32_t compartment)
{
    FS_GUARD_BEGIN
    fs_status st = check_seed(s, replica, count, nodes, compartment);
    if (st != FS_OK || count == 0) return st;
    if (count > FS_SEED_NOALLOC_MAX)
        return fail(FS_ERR_INVALID_ARG, "fs_sim_seed_noalloc takes at most " + std::to_string(FS_SEED_NOALLOC_MAX) +
                                            " nodes per call (got " + std::to_string(count) + ")");
    DeviceGuard dg(s->device);
    int64_t* stage = nullptr;
    st = scratch_address(s->device, &stage);
    if (st != FS_OK) return st;
    // Every id of [0, count) is written before the seed kernel reads it, so
    // nothing of an earlier call's contents is used.
    if (s->g->h_inv.empty()) {
        FS_HIP(hipMemcpyAsync(stage, nodes, sizeof(int64_t) * (size_t)count, hipMemcpyHostToDevice, s->stream));
    } else {
        // degree-sorted graph: the caller's ids go through the inverse
        // relabelling on the host, a bounded piece at a time through a stack
        // buffer; each piece's copy is complete before the buffer is refilled
        constexpr int64_t PIECE = 1024;
        int64_t buf[PIECE];
        for (int64_t j0 = 0; j0 < count; j0 += PIECE) {
            const int64_t m = std::min<int64_t>(PIECE, count - j0);
            for (int64_t j = 0; j < m; ++j) buf[j] = s->g->h_inv[(size_t)nodes[j0 + j]];
            FS_HIP(hipMemcpyAsync(stage + j0, buf, sizeof(int64_t) * (size_t)m, hipMemcpyHostToDevice, s->stream));
            FS_HIP(hipStreamSynchronize(s->stream));
        }
    }
    // (seed_staged ends with a synchronisation of the sim's stream, so the
    // staging is free again, and the caller's array no longer read, on return)
    return seed_staged(s, replica, stage, count, compartment);
    FS_GUARD_END
}

fs_status fs_step(fs_sim* s, int64_t n_steps)
{
    FS_GUARD_BEGIN
    if (!s) return fail(FS_ERR_INVALID_ARG, "sim is NULL");
    if (s->batch) return fail(FS_ERR_BUSY, "sim belongs to a batch: step it with fs_batch_step");
    if (n_steps < 0) return fail(FS_ERR_INVALID_ARG, "n_steps < 0");
    if (n_steps == 0) return FS_OK;
    DeviceGuard dg(s->device);
    const int b = s->p.steps_per_graph;
    int64_t rem = n_steps;
    if (b > 0 && n_steps >= b) {
        if (!s->exec) {
            fs_status st = build_graph_exec(s, b);
            if (st != FS_OK) return st;
        }
        for (int64_t r = 0; r < n_steps / b; ++r) FS_HIP(hipGraphLaunch(s->exec, s->stream));
        rem = n_steps % b;
    }
    while (rem > 0) {
        const uint32_t r = (uint32_t)std::min<int64_t>(rem, s->chunk);
        fs_status st = launch_sequence(s, r);
        if (st != FS_OK) return st;
        rem -= r;
    }
    s->step += n_steps;
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_sync(fs_sim* s)
{
    if (!s) return fail(FS_ERR_INVALID_ARG, "sim is NULL");
    DeviceGuard dg(s->device);
    FS_HIP(hipStreamSynchronize(s->stream));
    return FS_OK;
}

fs_status fs_step_index(fs_sim* s, int64_t* out)
{
    if (!s || !out) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    *out = s->step;
    return FS_OK;
}

fs_status fs_counts(fs_sim* s, int32_t replica, int64_t out[4])
{
    FS_GUARD_BEGIN
    if (!s || !out) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    fs_status st = check_replica(s, replica, false);
    if (st != FS_OK) return st;
    DeviceGuard dg(s->device);
    uint32_t h[4];
    FS_HIP(fsk::launch_recount(s->storage, s->d_state, (int32_t)s->g->n, s->lgR, replica, s->d_rc_part, RC_GRID,
                               s->d_cnt4, s->stream));
    FS_HIP(hipMemcpyAsync(h, s->d_cnt4, sizeof h, hipMemcpyDeviceToHost, s->stream));
    FS_HIP(hipStreamSynchronize(s->stream));
    for (int c = 0; c < 4; ++c) out[c] = h[c];
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_history(fs_sim* s, int32_t replica, int64_t first_step, int64_t n, int64_t* out)
{
    FS_GUARD_BEGIN
    if (!s || (n > 0 && !out)) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    fs_status st = check_replica(s, replica, false);
    if (st != FS_OK) return st;
    if (n < 0) return fail(FS_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return FS_OK;
    const int64_t lo = std::max(s->hist_from, s->step - (int64_t)s->H);
    if (first_step < lo || first_step + n > s->step)
        return fail(FS_ERR_INVALID_ARG, "requested steps are not in the kept history [" + std::to_string(lo) +
                                            ", " + std::to_string(s->step) + ")");
    DeviceGuard dg(s->device);
    const size_t row = (size_t)s->R * 4;
    std::vector<uint32_t> h((size_t)s->H * row);
    FS_HIP(hipMemcpyAsync(h.data(), s->d_hist, h.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, s->stream));
    FS_HIP(hipStreamSynchronize(s->stream));
    for (int64_t j = 0; j < n; ++j) {
        const size_t slot = (size_t)((first_step + j) % s->H);
        for (int c = 0; c < 4; ++c) out[4 * j + c] = (int64_t)h[slot * row + (size_t)replica * 4 + c];
    }
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_step_sizes(fs_sim* s, int64_t first_step, int64_t n, double* out)
{
    FS_GUARD_BEGIN
    if (!s || (n > 0 && !out)) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    if (n < 0) return fail(FS_ERR_INVALID_ARG, "n < 0");
    if (n == 0) return FS_OK;
    const int64_t lo = std::max(s->hist_from, s->step - (int64_t)s->H);
    if (first_step < lo || first_step + n > s->step)
        return fail(FS_ERR_INVALID_ARG, "requested steps are not in the kept history [" + std::to_string(lo) +
                                            ", " + std::to_string(s->step) + ")");
    if (!s->d_dt_hist) {
        for (int64_t j = 0; j < n; ++j) out[j] = (double)(float)s->p.dt;
        return FS_OK;
    }
    DeviceGuard dg(s->device);
    std::vector<float> h((size_t)s->H);
    FS_HIP(hipMemcpyAsync(h.data(), s->d_dt_hist, h.size() * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    FS_HIP(hipStreamSynchronize(s->stream));
    for (int64_t j = 0; j < n; ++j) out[j] = (double)h[(size_t)((first_step + j) % s->H)];
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_get_state(fs_sim* s, int32_t replica, int32_t* state, float* age_days, uint16_t* age_steps,
                       int64_t* step_index)
{
    FS_GUARD_BEGIN
    if (!s || !state) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    fs_status st = check_replica(s, replica, false);
    if (st != FS_OK) return st;
    void* age_out = s->storage == FS_STORAGE_FP32 ? (void*)age_days : (void*)age_steps;
    if (!age_out || (s->storage == FS_STORAGE_FP32 ? age_steps != nullptr : age_days != nullptr))
        return fail(FS_ERR_INVALID_ARG, "pass exactly the age array of the sim's storage");
    DeviceGuard dg(s->device);
    const size_t n = (size_t)s->g->n;
    StreamBuf ds(s->stream); StreamBuf da(s->stream);
    FS_HIP(hipMallocAsync(&ds.p, n * sizeof(int32_t), s->stream));
    FS_HIP(hipMallocAsync(&da.p, n * age_bytes(s->storage), s->stream));
    FS_HIP(fsk::launch_get_replica(s->storage, s->d_state, s->d_age, (int32_t*)ds.p, da.p, (int32_t)n, s->lgR,
                                   replica, s->stream));
    const bool reorder = !s->g->h_orig.empty();
    std::vector<int32_t> st_int(reorder ? n : 0);
    std::vector<uint8_t> age_int(reorder ? n * age_bytes(s->storage) : 0);
    FS_HIP(hipMemcpyAsync(reorder ? (void*)st_int.data() : (void*)state, ds.p, n * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s->stream));
    FS_HIP(hipMemcpyAsync(reorder ? (void*)age_int.data() : age_out, da.p, n * age_bytes(s->storage),
                          hipMemcpyDeviceToHost, s->stream));
    FS_HIP(hipStreamSynchronize(s->stream));
    if (reorder) {
        to_caller(s->g, st_int.data(), state);
        if (s->storage == FS_STORAGE_FP32) to_caller(s->g, (const float*)age_int.data(), age_days);
        else to_caller(s->g, (const uint16_t*)age_int.data(), age_steps);
    }
    if (step_index) *step_index = s->step;
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_set_state(fs_sim* s, int32_t replica, const int32_t* state, const float* age_days,
                       const uint16_t* age_steps, int64_t step_index)
{
    FS_GUARD_BEGIN
    if (!s || !state) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    fs_status st = check_replica(s, replica, false);
    if (st != FS_OK) return st;
    const void* age_in = s->storage == FS_STORAGE_FP32 ? (const void*)age_days : (const void*)age_steps;
    if (!age_in || (s->storage == FS_STORAGE_FP32 ? age_steps != nullptr : age_days != nullptr))
        return fail(FS_ERR_INVALID_ARG, "pass exactly the age array of the sim's storage");
    if (step_index < -1) return fail(FS_ERR_INVALID_ARG, "step_index must be >= -1");
    const size_t n = (size_t)s->g->n;
    for (size_t i = 0; i < n; ++i)
        if (state[i] < 0 || state[i] > 3) return fail(FS_ERR_INVALID_ARG, "state values must lie in [0, 3]");
    if (s->storage == FS_STORAGE_FP32)
        for (size_t i = 0; i < n; ++i)
            if (!(age_days[i] >= 0.0f) || !std::isfinite(age_days[i]))
                return fail(FS_ERR_INVALID_ARG, "ages must be finite and >= 0");
    DeviceGuard dg(s->device);
    const int64_t new_step = step_index >= 0 ? step_index : s->step;
    const size_t units = n * (size_t)s->R;
    std::vector<int32_t> st_tmp;
    std::vector<float> ad_tmp;
    std::vector<uint16_t> as_tmp;
    state = to_internal(s->g, state, st_tmp);
    age_in = s->storage == FS_STORAGE_FP32 ? (const void*)to_internal(s->g, age_days, ad_tmp)
                                           : (const void*)to_internal(s->g, age_steps, as_tmp);
    StreamBuf ds(s->stream); StreamBuf da(s->stream);
    FS_HIP(hipMallocAsync(&ds.p, n * sizeof(int32_t), s->stream));
    FS_HIP(hipMallocAsync(&da.p, n * age_bytes(s->storage), s->stream));
    FS_HIP(hipMemcpyAsync(ds.p, state, n * sizeof(int32_t), hipMemcpyHostToDevice, s->stream));
    FS_HIP(hipMemcpyAsync(da.p, age_in, n * age_bytes(s->storage), hipMemcpyHostToDevice, s->stream));
    FS_HIP(fsk::launch_put_replica(s->storage, s->d_state, s->d_age, (const int32_t*)ds.p, da.p, (int32_t)n, s->lgR,
                                   replica, s->stream));
    FS_HIP(fsk::launch_rebuild_bits(s->storage, s->d_state, (uint32_t)units,
                                    (unsigned long long*)s->d_iota[new_step & 1], s->bit_words, s->stream));
    FS_HIP(refresh_derived(s, new_step));
    // the step index, and (adaptive steps) a restart of the step-size rule at the cap
    FS_HIP(fsk::launch_set_ctl(s->d_ctl, (unsigned long long)new_step, s->stream));
    FS_HIP(refresh_summary(s));
    FS_HIP(hipStreamSynchronize(s->stream));
    if (step_index >= 0) {
        s->step = step_index;
        s->hist_from = step_index;
    }
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_get_rates(fs_sim* s, int32_t replica, float* out)
{
    FS_GUARD_BEGIN
    if (!s || !out) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    fs_status st = check_replica(s, replica, false);
    if (st != FS_OK) return st;
    if (!s->d_rates) return fail(FS_ERR_INVALID_ARG, "sim was created without record_rates");
    DeviceGuard dg(s->device);
    const size_t n = (size_t)s->g->n;
    StreamBuf d(s->stream);
    FS_HIP(hipMallocAsync(&d.p, n * sizeof(float), s->stream));
    FS_HIP(fsk::launch_get_rates(s->d_rates, (float*)d.p, (int32_t)n, s->lgR, replica, s->stream));
    const bool reorder = !s->g->h_orig.empty();
    std::vector<float> r_int(reorder ? n : 0);
    FS_HIP(hipMemcpyAsync(reorder ? r_int.data() : out, d.p, n * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    FS_HIP(hipStreamSynchronize(s->stream));
    if (reorder) to_caller(s->g, r_int.data(), out);
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_sim_set_bins(fs_sim* s, int32_t heavy_degree, int32_t segment_edges)
{
    FS_GUARD_BEGIN
    if (!s) return fail(FS_ERR_INVALID_ARG, "sim is NULL");
    if (s->batch) return fail(FS_ERR_BUSY, "sim belongs to a batch");
    if (heavy_degree < -1) return fail(FS_ERR_INVALID_ARG, "heavy_degree must be >= -1");
    DeviceGuard dg(s->device);
    FS_HIP(hipStreamSynchronize(s->stream));
    return apply_bins(s, heavy_degree == 0 ? 64 : heavy_degree, segment_edges == 0 ? 512 : segment_edges);
    FS_GUARD_END
}

fs_status fs_sim_get_bins(fs_sim* s, int32_t* heavy_degree, int32_t* segment_edges, int64_t* segments)
{
    if (!s) return fail(FS_ERR_INVALID_ARG, "sim is NULL");
    if (heavy_degree) *heavy_degree = s->heavy_deg;
    if (segment_edges) *segment_edges = s->seg_edges;
    if (segments) *segments = s->nseg;
    return FS_OK;
}

fs_status fs_sim_tune(fs_sim* s, int32_t trial_steps, int32_t* heavy_degree, int32_t* segment_edges)
{
    FS_GUARD_BEGIN
    fs_tune_params p{};
    p.trial_steps = trial_steps;
    fs_tune_result r{};
    fs_status st = autotune(s, p, &r);
    if (st != FS_OK) return st;
    if (heavy_degree) *heavy_degree = r.heavy_degree;
    if (segment_edges) *segment_edges = r.segment_edges;
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_sim_autotune(fs_sim* s, const fs_tune_params* p, fs_tune_result* out)
{
    FS_GUARD_BEGIN
    if (!p || !out) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    return autotune(s, *p, out);
    FS_GUARD_END
}

fs_status fs_sim_get_variant(fs_sim* s, int32_t* variant)
{
    if (!s || !variant) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    *variant = s->mode + 1;
    return FS_OK;
}

fs_status fs_sim_get_column_bits(fs_sim* s, int32_t* bits)
{
    if (!s || !bits) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    *bits = (s->layout && s->layout->pbits) ? s->layout->pbits : 32;
    return FS_OK;
}

fs_status fs_eval_hazard(const fs_dist* law, int32_t storage, double dt, int64_t n, const void* ages, float* out)
{
    FS_GUARD_BEGIN
    if (!law || (n > 0 && (!ages || !out))) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    if (storage != FS_STORAGE_FP32 && storage != FS_STORAGE_COMPACT) return fail(FS_ERR_INVALID_ARG, "unknown storage");
    if (!(dt > 0.0)) return fail(FS_ERR_INVALID_ARG, "dt must be > 0");
    if (n < 0) return fail(FS_ERR_INVALID_ARG, "n < 0");
    HazardDev h;
    fs_status st = prep_hazard(*law, storage, dt, &h, "law");
    if (st != FS_OK) return st;
    if (n == 0) return FS_OK;
    const size_t ab = storage == FS_STORAGE_FP32 ? 4 : 2;
    DevBuf da, dout;
    FS_HIP(dev_alloc(&da.p, (size_t)n * ab));
    FS_HIP(dev_alloc(&dout.p, (size_t)n * sizeof(float)));
    FS_HIP(hipMemcpy(da.p, ages, (size_t)n * ab, hipMemcpyHostToDevice));
    FS_HIP(fsk::launch_eval_hazard(h, storage, da.p, (float*)dout.p, n, nullptr));
    FS_HIP(hipMemcpy(out, dout.p, (size_t)n * sizeof(float), hipMemcpyDeviceToHost));
    FS_HIP(hipDeviceSynchronize());
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_eval_shedding(const fs_dist* law, int32_t form, double scale, int32_t storage, double dt, int64_t n,
                           const void* ages, float* out)
{
    FS_GUARD_BEGIN
    if (!law || (n > 0 && (!ages || !out))) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    if (storage != FS_STORAGE_FP32 && storage != FS_STORAGE_COMPACT) return fail(FS_ERR_INVALID_ARG, "unknown storage");
    if (!(dt > 0.0)) return fail(FS_ERR_INVALID_ARG, "dt must be > 0");
    if (n < 0) return fail(FS_ERR_INVALID_ARG, "n < 0");
    if (form != FS_SHED_DENSITY && form != FS_SHED_HAZARD)
        return fail(FS_ERR_INVALID_ARG, "form must be FS_SHED_DENSITY or FS_SHED_HAZARD");
    fsi::ShedDev sd;
    fs_status st = prep_shed(form, *law, scale, storage, dt, &sd);
    if (st != FS_OK) return st;
    if (n == 0) return FS_OK;
    const size_t ab = storage == FS_STORAGE_FP32 ? 4 : 2;
    DevBuf da, dout;
    FS_HIP(dev_alloc(&da.p, (size_t)n * ab));
    FS_HIP(dev_alloc(&dout.p, (size_t)n * sizeof(float)));
    FS_HIP(hipMemcpy(da.p, ages, (size_t)n * ab, hipMemcpyHostToDevice));
    FS_HIP(fsk::launch_eval_shed(sd, storage, da.p, (float*)dout.p, n, nullptr));
    FS_HIP(hipMemcpy(out, dout.p, (size_t)n * sizeof(float), hipMemcpyDeviceToHost));
    FS_HIP(hipDeviceSynchronize());
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_eval_philox(int64_t n, const uint32_t* ctr, uint64_t seed, uint32_t* out)
{
    FS_GUARD_BEGIN
    if (n < 0 || (n > 0 && (!ctr || !out))) return fail(FS_ERR_INVALID_ARG, "bad argument");
    if (n == 0) return FS_OK;
    DevBuf dc, dout;
    FS_HIP(dev_alloc(&dc.p, (size_t)n * 16));
    FS_HIP(dev_alloc(&dout.p, (size_t)n * 16));
    FS_HIP(hipMemcpy(dc.p, ctr, (size_t)n * 16, hipMemcpyHostToDevice));
    FS_HIP(fsk::launch_eval_philox((const uint4*)dc.p, (uint32_t)seed, (uint32_t)(seed >> 32), (uint4*)dout.p, n,
                                   nullptr));
    FS_HIP(hipMemcpy(out, dout.p, (size_t)n * 16, hipMemcpyDeviceToHost));
    FS_HIP(hipDeviceSynchronize());
    return FS_OK;
    FS_GUARD_END
}

} // extern "C"
