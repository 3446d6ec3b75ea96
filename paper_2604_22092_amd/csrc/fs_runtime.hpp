// Private runtime structures of the library: the graph and simulation
// handles behind the C ABI and the helpers shared by the runtime sources.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "fs.h"
#include "fs_internal.hpp"
#include "fs_kernels.hpp"

using fsi::HazardDev;
using fsi::StepArgs;
using fsi::WG;

struct fs_batch;

namespace fsr {
// The degree-binned, wavefront-transposed layout of a graph's rows for one
// replica count, one pair of bin thresholds (light-degree limit, heavy
// segment length) and whether the columns of a uniform layout may be packed.
// It depends on nothing else, so every sim of the graph with these
// parameters shares one copy (the graph caches it).
struct Layout {
    int32_t limit = 0;           // rows with more edges than this are heavy
    int32_t seg_edges = 0;
    uint32_t nseg = 0;           // heavy-row segments
    int32_t udeg = -1;           // the uniform light degree of every chunk, or -1
    int32_t pbits = 0;           // packed columns of a uniform layout: bits per column, or 0
    int32_t* d_heavy_first = nullptr;
    fsi::Segment* d_segs = nullptr;
    uint16_t* d_ldeg = nullptr;       // light degree per node, HEAVY_ROW for binned rows
    uint2* d_chunk_meta = nullptr;    // per chunk: (first slot in col_t, shared degree or 255)
    int32_t* d_col_t = nullptr;
    float* d_w_t = nullptr;
    // binned rows, which are the internal nodes [hub_base, n), for pushes
    // (unweighted graphs): per node j the hub indices of the binned rows
    // listing j, hub_out_idx[hub_out_ptr[j] .. hub_out_ptr[j + 1])
    int32_t hub_base = 0;
    uint32_t hubs = 0;                // 0: no pushes (weighted graph or no binned row)
    int32_t* d_hub_out_ptr = nullptr;
    int32_t* d_hub_out_idx = nullptr;
    size_t bytes = 0;
    ~Layout();
};
using LayoutKey = std::tuple<int32_t, int32_t, int32_t, int32_t>; // (replicas, limit, seg_edges, packing allowed)
} // namespace fsr

struct fs_graph {
    int device = 0;
    int64_t n = 0, nnz = 0;
    int32_t* d_row_ptr = nullptr;
    int32_t* d_col_ind = nullptr;
    float* d_weights = nullptr;
    int32_t max_degree = 0;
    int32_t min_degree = 0;
    double mean_degree = 0.0;
    // Graphs whose rows do not all have one degree are kept with their nodes
    // in a degree-sorted internal order, so the 64-unit chunks of the step
    // are (almost all) uniform in degree.  h_orig[internal] is the caller's
    // node id and h_inv its inverse (both empty for the identity order); the
    // CSR copies below and every per-node device array are in internal order,
    // and the C ABI converts node ids and per-node arrays at its boundary.
    std::vector<int32_t> h_orig, h_inv;
    int32_t* d_orig = nullptr;      // internal -> caller's id on the device (identity when not reordered)
    std::vector<int32_t> h_row_ptr; // host copies (internal order) for degree binning and layouts
    std::vector<int32_t> h_col_ind;
    std::vector<float> h_weights;
    // outgoing CSR of the internal order (the Markovian engine's sparse
    // pushes), built on first use
    int32_t* d_out_ptr = nullptr;
    int32_t* d_out_ind = nullptr;
    std::atomic<int> users{0};
    std::mutex layout_mu;        // guards layouts and the outgoing CSR (sims of one graph may live on several threads)
    std::map<fsr::LayoutKey, std::shared_ptr<fsr::Layout>> layouts;
};

struct fs_sim {
    fs_graph* g = nullptr;
    fs_sim_params p{};
    int device = 0;
    int lgR = 0, R = 1;
    int storage = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* d_state = nullptr;
    void* d_age = nullptr;
    void* d_iota[2] = {nullptr, nullptr};
    float* d_rates = nullptr;
    fsi::Ctl* d_ctl = nullptr;
    uint32_t* d_hist = nullptr;    // [H][R][4] counts after each step
    uint32_t* d_part = nullptr;    // [chunk][G][R][4] per-workgroup partials
    uint32_t* d_rc_part = nullptr; // recount partials [RC_GRID][4]
    uint32_t* d_cnt4 = nullptr;
    float* d_lam_part = nullptr;   // adaptive step: per-workgroup rate maxima [2][G]
    float* d_dt_hist = nullptr;    // adaptive step: step size of each step, ring of H
    void* d_shed[2] = {nullptr, nullptr}; // age-dependent shedding: s(tau) per unit (float32, or binary16
                                          // with compact storage), ping-pong
    uint8_t* d_live = nullptr;     // compaction: live flag per chunk, zero-padded to LIVE_TILE
    uint32_t* d_act = nullptr;     // compaction: [2 + nchunks] active-chunk list
    float4* d_htab = nullptr;      // fixed steps: hazard table (StepArgs::htab)
    fsi::LawsDev* d_laws = nullptr; // both laws and the shedding profile (StepArgs::hz_dev, shed_dev)
    uint32_t nchunks = 0;          // 64-unit chunks
    size_t live_bytes = 0;
    fsi::ShedDev shed{};
    int H = 1024;
    uint32_t G = 0;                // step workgroups
    uint32_t cus = 0;              // compute units of the device (LDS variants)
    uint32_t tpb = 0;              // threads (units) per step workgroup / tile
    int mode = fsi::MODE_STREAM;   // step kernel variant
    unsigned long long* d_summary = nullptr; // MODE_SUMMARY: summary of the current bitmap
    uint32_t sum_bits = 0, sum_words = 0;
    int32_t sum_shift = 0;   // summary groups of 32 * 2^sum_shift units
    uint32_t bit_words = 0;        // 64-bit words per infectivity bitmap
    uint32_t chunk = 0;            // steps per launch sequence (partial slots)
    int64_t step = 0;      // index of the next step (host mirror of ctl->step)
    int64_t hist_from = 0; // first step whose count row is recorded
    StepArgs args{};
    const void* kfn = nullptr;
    // degree bins
    int32_t heavy_deg = 0;         // rows with degree > heavy_deg are binned; < 0: none
    int32_t seg_edges = 512;
    uint32_t nseg = 0;
    std::shared_ptr<fsr::Layout> layout; // shared with the graph's other sims
    void* d_seg_part = nullptr;          // this sim's heavy-segment partials [segment][R]
    bool hub_push = false;               // binned rows take pushed pressure (StepArgs::hub_T)
    bool pack = false;                   // a uniform layout's columns may be packed (StepArgs::pbits)
    uint32_t* d_hub = nullptr;           // hub_T [2][hub units] then hub_D [3][hub units]
    fsi::Segment* d_segs = nullptr;      // = layout->d_segs
    const void* hfn = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    fs_batch* batch = nullptr;     // the batch the sim belongs to, if any
    hipStream_t saved_stream = nullptr; // the sim's own stream while it runs on a batch's
};

namespace fsr {

// Records the detail message of a failure (read by fs_last_error) and returns s.
fs_status fail(fs_status s, const std::string& msg);
extern thread_local std::string g_err;

#define FS_HIP(call)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fsr::fail(e_ == hipErrorOutOfMemory ? FS_ERR_OUT_OF_MEMORY : FS_ERR_DEVICE, \
                             std::string(#call) + ": " + hipGetErrorString(e_));               \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int d)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != d) (void)hipSetDevice(d);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Device allocations go through hipMalloc; a failed allocation reports
// FS_ERR_OUT_OF_MEMORY and the caller releases what it already holds.
hipError_t dev_alloc(void** p, size_t bytes);
void dev_free(void* p);

// RAII device buffer for call-local temporaries.
struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { dev_free(p); }
};

// RAII stream-ordered temporary (hipMallocAsync on `s`), freed in stream order.
struct StreamBuf {
    void* p = nullptr;
    hipStream_t s;
    explicit StreamBuf(hipStream_t st) : s(st) {}
    ~StreamBuf()
    {
        if (p) (void)hipFreeAsync(p, s);
    }
};

// Releases a sim without waiting for its stream: its buffers are freed in
// stream order (callers guarantee no later work on other streams uses them).
void release_sim(fs_sim* s);
size_t state_bytes(int storage);
size_t age_bytes(int storage);
size_t shed_bytes(int storage); // a stored shedding value: float32, or binary16 with compact storage
uint32_t heavy_grid(const fs_sim* s);       // WG-thread heavy workgroups (batches too)
uint32_t sim_heavy_grid(const fs_sim* s);   // the sim's own heavy launch
uint32_t sim_heavy_block(const fs_sim* s);
fsi::HeavyArgs heavy_args(const fs_sim* s);
// Device bytes a sim of this graph and these parameters holds (an estimate
// used for admission by memory budget).
size_t sim_footprint(fs_graph* g, const fs_sim_params* p);
// Seeding (fs_sim_seed and its variants): the argument rules, and the device
// part once the internal node ids of `count` seeds sit in device memory at
// d_nodes (synchronises the sim's stream, so d_nodes may be reused after).
fs_status check_seed(const fs_sim* s, int32_t replica, int64_t count, const int64_t* nodes, int32_t compartment);
fs_status seed_staged(fs_sim* s, int32_t replica, const int64_t* d_nodes, int64_t count, int32_t compartment);
// Puts a sim whose layout has packed columns on the graph's layout with
// 32-bit columns (the batch kernel reads only those); the sim's stream must
// be idle.  Results do not change.
fs_status use_plain_columns(fs_sim* s);

} // namespace fsr
