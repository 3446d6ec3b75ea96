// Batches and the scenario server of the C ABI declared in include/fs.h.
//
// A batch advances several simulations (each with its own graph, laws,
// replicas and step index) by one fused launch per step: a table of the
// members' step arguments and a block-range table let every workgroup find
// its member, and the per-step counts of all members are reduced by one
// launch per sequence.  Each member runs exactly the streaming step it would
// run alone, so its results are the same alone and in the batch.
//
// The server keeps a queue of scenario requests.  A worker thread runs
// rounds of steps on one stream: large requests step alone with the kernel
// variant that suits them, small ones share a batch.  While one round runs on
// the device the worker admits queued requests (creating and seeding their
// sims on a second stream) and retires the requests the previous round
// finished, so the device always has the next round queued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "fs_runtime.hpp"

using namespace fsr;

namespace {

// Pinned host staging for asynchronous uploads: two buffers used in turn,
// each reused only after the event of its last upload has completed.
struct Staging {
    void* host[2] = {nullptr, nullptr};
    size_t cap[2] = {0, 0};
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool used[2] = {false, false};
    int cur = 0;
    ~Staging()
    {
        for (int i = 0; i < 2; ++i) {
            if (ev[i]) {
                (void)hipEventSynchronize(ev[i]);
                (void)hipEventDestroy(ev[i]);
            }
            if (host[i]) (void)hipHostFree(host[i]);
        }
    }
    // A buffer of at least `bytes` whose previous upload has finished.
    fs_status take(size_t bytes, void** out, int* slot)
    {
        const int i = cur;
        cur ^= 1;
        if (!ev[i]) FS_HIP(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
        if (used[i]) FS_HIP(hipEventSynchronize(ev[i]));
        if (cap[i] < bytes) {
            if (host[i]) (void)hipHostFree(host[i]);
            host[i] = nullptr;
            cap[i] = 0;
            FS_HIP(hipHostMalloc(&host[i], std::max<size_t>(bytes, 4096), hipHostMallocDefault));
            cap[i] = std::max<size_t>(bytes, 4096);
        }
        *out = host[i];
        *slot = i;
        return FS_OK;
    }
    fs_status mark(int slot, hipStream_t s)
    {
        FS_HIP(hipEventRecord(ev[slot], s));
        used[slot] = true;
        return FS_OK;
    }
};

} // namespace

struct fs_batch {
    int device = 0;
    int storage = 0;
    int weighted = -1; // fixed by the first member
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<fs_sim*> members;
    bool dirty = true;
    // device tables (one stream-ordered block), rebuilt when the membership changes
    void* d_tables = nullptr;
    size_t d_cap = 0;
    StepArgs* d_table = nullptr;
    uint32_t* d_first = nullptr;
    fsi::HeavyArgs* d_htable = nullptr;
    uint32_t* d_hfirst = nullptr;
    fsi::RedArgs* d_red = nullptr;
    uint32_t blocks = 0, hblocks = 0, hmembers = 0;
    uint32_t chunk = 0; // longest launch sequence (partial slots of the members)
    Staging staging;
};

namespace {

#define FS_GUARD_BEGIN try {
#define FS_GUARD_END                                                                            \
    }                                                                                           \
    catch (const std::bad_alloc&) { return fail(FS_ERR_OUT_OF_MEMORY, "host allocation failed"); } \
    catch (const std::exception& e) { return fail(FS_ERR_DEVICE, e.what()); }                   \
    catch (...) { return fail(FS_ERR_DEVICE, "unknown exception"); }

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Rebuilds the device tables from the current members: one staging buffer
// holds every table and one asynchronous copy uploads it.  Work already
// queued on the batch stream reads the tables it was launched with: the copy
// is ordered after it, and a grown table block is a new allocation while the
// old one is freed in stream order.
fs_status rebuild_tables(fs_batch* b)
{
    const size_t M = b->members.size();
    std::vector<StepArgs> table;
    std::vector<uint32_t> first(1, 0u), hfirst(1, 0u);
    std::vector<fsi::HeavyArgs> htable;
    std::vector<fsi::RedArgs> red;
    b->chunk = 1u << 30;
    for (fs_sim* s : b->members) {
        table.push_back(s->args);
        first.push_back(first.back() + s->G);
        if (s->nseg && !s->hub_push) {
            htable.push_back(heavy_args(s));
            hfirst.push_back(hfirst.back() + heavy_grid(s));
        }
        fsi::RedArgs r{};
        r.ctl = s->d_ctl;
        r.part = s->d_part;
        r.hist = s->d_hist;
        r.G = s->G;
        r.C = 4u * (uint32_t)s->R;
        r.H = (uint32_t)s->H;
        red.push_back(r);
        b->chunk = std::min(b->chunk, s->chunk);
    }
    b->blocks = first.back();
    b->hblocks = hfirst.back();
    b->hmembers = (uint32_t)htable.size();
    b->dirty = false;
    if (M == 0) return FS_OK;
    const size_t o_table = 0;
    const size_t o_first = align_up(o_table + M * sizeof(StepArgs));
    const size_t o_htable = align_up(o_first + (M + 1) * sizeof(uint32_t));
    const size_t o_hfirst = align_up(o_htable + std::max<size_t>(htable.size(), 1) * sizeof(fsi::HeavyArgs));
    const size_t o_red = align_up(o_hfirst + hfirst.size() * sizeof(uint32_t));
    const size_t bytes = align_up(o_red + M * sizeof(fsi::RedArgs));
    void* host = nullptr;
    int slot = 0;
    fs_status st = b->staging.take(bytes, &host, &slot);
    if (st != FS_OK) return st;
    char* h = (char*)host;
    std::memcpy(h + o_table, table.data(), M * sizeof(StepArgs));
    std::memcpy(h + o_first, first.data(), first.size() * sizeof(uint32_t));
    if (!htable.empty()) std::memcpy(h + o_htable, htable.data(), htable.size() * sizeof(fsi::HeavyArgs));
    std::memcpy(h + o_hfirst, hfirst.data(), hfirst.size() * sizeof(uint32_t));
    std::memcpy(h + o_red, red.data(), M * sizeof(fsi::RedArgs));
    if (bytes > b->d_cap) {
        if (b->d_tables) (void)hipFreeAsync(b->d_tables, b->stream);
        b->d_tables = nullptr;
        b->d_cap = 0;
        FS_HIP(hipMallocAsync(&b->d_tables, bytes * 2, b->stream));
        b->d_cap = bytes * 2;
    }
    char* d = (char*)b->d_tables;
    FS_HIP(hipMemcpyAsync(d, host, bytes, hipMemcpyHostToDevice, b->stream));
    if ((st = b->staging.mark(slot, b->stream)) != FS_OK) return st;
    b->d_table = (StepArgs*)(d + o_table);
    b->d_first = (uint32_t*)(d + o_first);
    b->d_htable = (fsi::HeavyArgs*)(d + o_htable);
    b->d_hfirst = (uint32_t*)(d + o_hfirst);
    b->d_red = (fsi::RedArgs*)(d + o_red);
    return FS_OK;
}

// The member rules of a batch (include/fs.h): every member runs the
// streaming step of the batch's storage with fixed steps, constant shedding
// and no compaction, and the members agree on weights (the batch kernel is
// instantiated for one of the two).
fs_status member_check(const fs_batch* b, const fs_sim* s, bool allow_packed = false)
{
    if (s->batch) return fail(FS_ERR_BUSY, "sim already belongs to a batch");
    if (s->device != b->device) return fail(FS_ERR_INVALID_ARG, "sim and batch are on different devices");
    if (s->mode != fsi::MODE_STREAM)
        return fail(FS_ERR_INVALID_ARG, "batch members run the streaming step: create the sim with variant = 1");
    if (s->storage != b->storage) return fail(FS_ERR_INVALID_ARG, "sim storage differs from the batch's");
    if (s->p.adaptive) return fail(FS_ERR_INVALID_ARG, "adaptive-step sims cannot join a batch");
    if (s->p.shedding != FS_SHED_CONSTANT)
        return fail(FS_ERR_INVALID_ARG, "sims with age-dependent shedding cannot join a batch");
    if (s->p.compaction) return fail(FS_ERR_INVALID_ARG, "sims with compaction cannot join a batch");
    if (!allow_packed && s->layout && s->layout->pbits != 0)
        return fail(FS_ERR_INVALID_ARG, "batch members read 32-bit columns (the sim has packed ones)");
    const int w = s->g->d_weights != nullptr;
    if (!b->members.empty() && w != b->weighted)
        return fail(FS_ERR_INVALID_ARG, "batch members must agree on weights");
    return FS_OK;
}

// Membership changes without waiting: the caller guarantees that queued
// batch work never touches a sim after it leaves (the next launch uses
// rebuilt tables) and that an added sim's own queued work is finished.
// The member rules are checked here too, so no path can add a sim the
// batch kernel would run with the wrong instantiation.
fs_status attach(fs_batch* b, fs_sim* s)
{
    const fs_status st = member_check(b, s);
    if (st != FS_OK) return st;
    b->weighted = s->g->d_weights != nullptr;
    s->saved_stream = s->stream;
    s->stream = b->stream;
    s->batch = b;
    b->members.push_back(s);
    b->dirty = true;
    return FS_OK;
}

void detach(fs_batch* b, fs_sim* s)
{
    s->stream = s->saved_stream;
    s->saved_stream = nullptr;
    s->batch = nullptr;
    b->members.erase(std::remove(b->members.begin(), b->members.end(), s), b->members.end());
    b->dirty = true;
}

fs_status batch_sequence(fs_batch* b, uint32_t r)
{
    const uint32_t M = (uint32_t)b->members.size();
    // the instantiation with rate recording only when a member records them
    bool rates = false;
    for (const fs_sim* s : b->members) rates = rates || s->d_rates != nullptr;
    const void* kfn = fsk::step_batch_kernel_fn(b->storage, b->weighted == 1, rates);
    const void* hfn = fsk::heavy_batch_kernel_fn(b->weighted == 1);
    if (!kfn || !hfn) return fail(FS_ERR_DEVICE, "no batch kernel for this configuration");
    for (uint32_t j = 0; j < r; ++j) {
        uint32_t off = j;
        if (b->hmembers) {
            void* hargv[] = {&b->d_htable, &b->d_hfirst, &b->hmembers, &off};
            FS_HIP(hipLaunchKernel(hfn, dim3(b->hblocks), dim3(WG), hargv, 0, b->stream));
        }
        uint32_t members = M;
        void* argv[] = {&b->d_table, &b->d_first, &members, &off};
        FS_HIP(hipLaunchKernel(kfn, dim3(b->blocks), dim3(fsi::STREAM_TPB), argv, 0, b->stream));
    }
    void* rargv[] = {&b->d_red};
    FS_HIP(hipLaunchKernel(fsk::reduce_batch_kernel_fn(), dim3(r, M), dim3(fsi::RED_TPB), rargv, 0, b->stream));
    return FS_OK;
}

// Queues n_steps steps of every member (no host wait).
fs_status batch_step(fs_batch* b, int64_t n_steps)
{
    if (n_steps <= 0 || b->members.empty()) return FS_OK;
    if (b->dirty) {
        fs_status st = rebuild_tables(b);
        if (st != FS_OK) return st;
    }
    int64_t rem = n_steps;
    while (rem > 0) {
        const uint32_t r = (uint32_t)std::min<int64_t>(rem, b->chunk);
        fs_status st = batch_sequence(b, r);
        if (st != FS_OK) return st;
        rem -= r;
    }
    for (fs_sim* s : b->members) s->step += n_steps;
    return FS_OK;
}

} // namespace

extern "C" {

fs_status fs_batch_create(int32_t storage, void* stream, fs_batch** out)
{
    FS_GUARD_BEGIN
    if (!out) return fail(FS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (storage != FS_STORAGE_FP32 && storage != FS_STORAGE_COMPACT) return fail(FS_ERR_INVALID_ARG, "unknown storage");
    std::unique_ptr<fs_batch> b(new fs_batch());
    FS_HIP(hipGetDevice(&b->device));
    b->storage = storage;
    if (stream) {
        b->stream = (hipStream_t)stream;
    } else {
        FS_HIP(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
        b->own_stream = true;
    }
    *out = b.release();
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_batch_destroy(fs_batch* b)
{
    FS_GUARD_BEGIN
    if (!b) return fail(FS_ERR_INVALID_ARG, "batch is NULL");
    DeviceGuard dg(b->device);
    const hipError_t e = hipStreamSynchronize(b->stream);
    while (!b->members.empty()) detach(b, b->members.back());
    if (b->d_tables) (void)hipFreeAsync(b->d_tables, b->stream);
    (void)hipStreamSynchronize(b->stream);
    const bool own = b->own_stream;
    hipStream_t s = b->stream;
    delete b;
    if (own) (void)hipStreamDestroy(s);
    if (e != hipSuccess) return fail(FS_ERR_DEVICE, std::string("pending work failed: ") + hipGetErrorString(e));
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_batch_add(fs_batch* b, fs_sim* s)
{
    FS_GUARD_BEGIN
    if (!b || !s) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    fs_status st = member_check(b, s, true);
    if (st != FS_OK) return st;
    DeviceGuard dg(b->device);
    FS_HIP(hipStreamSynchronize(s->stream));
    // the batch kernel reads 32-bit columns: a sim with packed ones moves to
    // the graph's layout with plain columns first
    if ((st = use_plain_columns(s)) != FS_OK) return st;
    return attach(b, s);
    FS_GUARD_END
}

fs_status fs_batch_remove(fs_batch* b, fs_sim* s)
{
    FS_GUARD_BEGIN
    if (!b || !s) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    if (s->batch != b) return fail(FS_ERR_INVALID_ARG, "sim is not a member of this batch");
    DeviceGuard dg(b->device);
    FS_HIP(hipStreamSynchronize(b->stream));
    detach(b, s);
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_batch_size(fs_batch* b, int32_t* members)
{
    if (!b || !members) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    *members = (int32_t)b->members.size();
    return FS_OK;
}

fs_status fs_batch_step(fs_batch* b, int64_t n_steps)
{
    FS_GUARD_BEGIN
    if (!b) return fail(FS_ERR_INVALID_ARG, "batch is NULL");
    if (n_steps < 0) return fail(FS_ERR_INVALID_ARG, "n_steps < 0");
    DeviceGuard dg(b->device);
    return batch_step(b, n_steps);
    FS_GUARD_END
}

fs_status fs_batch_sync(fs_batch* b)
{
    if (!b) return fail(FS_ERR_INVALID_ARG, "batch is NULL");
    DeviceGuard dg(b->device);
    FS_HIP(hipStreamSynchronize(b->stream));
    return FS_OK;
}

} // extern "C"

// ------------------------------------------------------------------ server

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Pinned host buffers for count histories, reused across requests (worker
// thread only).
struct PinnedPool {
    std::vector<std::pair<void*, size_t>> free_list;
    std::map<void*, size_t> size_of;
    ~PinnedPool()
    {
        for (auto& f : size_of) (void)hipHostFree(f.first);
    }
    void* take(size_t bytes)
    {
        for (size_t i = 0; i < free_list.size(); ++i)
            if (free_list[i].second >= bytes) {
                void* p = free_list[i].first;
                free_list.erase(free_list.begin() + (long)i);
                return p;
            }
        void* p = nullptr;
        if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
        size_of[p] = bytes;
        return p;
    }
    void give(void* p)
    {
        if (p) free_list.push_back({p, size_of[p]});
    }
};

// Requests with at least this many units give every wavefront of the GPU a
// chunk by themselves: they run their own step kernels (the variant that
// suits their size), each on a stream of its own, so that the kernels of two
// such requests (and the batch's) overlap on the device.  Smaller ones share the batch's
// fused launches.  At most MAX_SOLO large requests step at once (sharing the
// GPU between more of them only lengthens each one's latency).  Measured on
// the serving mix: with every request in the batch instead, the server
// finished 42.7 scenarios/s at saturation against 71.4 with this threshold.
constexpr size_t SOLO_UNITS = (size_t)1 << 18;
#ifndef FS_MAX_SOLO
#define FS_MAX_SOLO 2
#endif
constexpr int MAX_SOLO = FS_MAX_SOLO;

struct Request {
    int64_t id = 0;
    fs_graph* g = nullptr;
    fs_sim_params p{};
    int64_t n_steps = 0;
    std::vector<int64_t> seeds;
    size_t bytes = 0;
    fs_sim* sim = nullptr;
    bool solo = false;               // runs its own step kernels instead of joining the batch
    int slot = -1;                   // solo: its stream slot (fs_server::solo_stream)
    int64_t done_steps = 0;          // steps queued so far
    uint32_t* pinned_hist = nullptr; // [n_steps][R][4] counts, copied after the last round
    fs_request_info info{};
    std::vector<int64_t> history;    // [n_steps][R][4]
    std::string error;
    bool finished = false;
};

} // namespace

struct fs_server {
    fs_server_params p{};
    int device = 0;
    hipStream_t stream = nullptr;       // rounds: every admitted request's steps
    hipStream_t admit_stream = nullptr; // creation and seeding of new requests
    hipStream_t solo_stream[MAX_SOLO] = {}; // one per solo slot
    hipEvent_t slot_ev[MAX_SOLO] = {};      // end of the slot's request (its steps and history copy)
    bool slot_used[MAX_SOLO] = {};
    bool own_stream = false;
    // small requests share one batch per weightedness ([0]: unit weights,
    // [1]: weighted graphs), since a batch launch runs one instantiation
    fs_batch* batch[2] = {nullptr, nullptr};
    size_t budget = 0, in_use = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;             // submitted, not admitted
    std::vector<std::shared_ptr<Request>> active;           // batch members stepping in the next round
    std::vector<std::shared_ptr<Request>> running;          // solo requests, every step queued
    std::map<int64_t, std::shared_ptr<Request>> requests;   // every request not yet collected
    int64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    std::string worker_error;
    uint64_t rounds = 0;
    PinnedPool pinned;
};

namespace {



// Creates and seeds the sim of an admitted request on the admission stream,
// while a round runs (worker thread, lock not held).
fs_status start_request(fs_server* sv, Request& q)
{
    fs_sim_params p = q.p;
    p.storage = sv->p.storage;
    p.variant = q.solo ? 0 : 1;
    // batched requests read 32-bit columns; solo ones may take packed ones
    p.columns = q.solo ? q.p.columns : FS_COLUMNS_PLAIN;
    p.steps_per_graph = 0;
    p.history_len = (int32_t)std::max<int64_t>(q.n_steps, 2);
    p.stream = sv->admit_stream;
    p.record_rates = 0;
    fs_status st = fs_sim_create(q.g, &p, &q.sim);
    if (st != FS_OK) return st;
    if (!q.seeds.empty() && (st = fs_sim_seed(q.sim, -1, (int64_t)q.seeds.size(), q.seeds.data(), FS_E)) != FS_OK)
        return st;
    q.pinned_hist = (uint32_t*)sv->pinned.take((size_t)q.n_steps * q.p.n_replicas * 4 * sizeof(uint32_t));
    if (!q.pinned_hist) return fail(FS_ERR_OUT_OF_MEMORY, "pinned host buffer");
    return FS_OK;
}

// Releases a request's sim in stream order (no wait) and its pinned buffer.
void drop_sim(fs_server* sv, Request& q)
{
    if (q.sim) {
        if (q.sim->batch) detach(q.sim->batch, q.sim);
        release_sim(q.sim);
        q.sim = nullptr;
    }
    if (q.pinned_hist) {
        sv->pinned.give(q.pinned_hist);
        q.pinned_hist = nullptr;
    }
}

// Ends request q with status st (the lock is held).
void end_request(Request& q, fs_status st, const std::string& err)
{
    q.info.status = st;
    if (st != FS_OK) q.error = err;
    if (q.info.t_done == 0.0) q.info.t_done = now_s();
    q.finished = true;
    q.g->users.fetch_sub(1);
}

struct Round {
    hipEvent_t ev = nullptr;
    bool pending = false;
    std::vector<std::shared_ptr<Request>> ending; // requests whose last steps it holds
};

// Retires the solo requests whose queued work has finished (lock not held;
// returns the retired ones).
fs_status retire_solos(fs_server* sv, std::vector<std::shared_ptr<Request>>& running,
                       std::vector<std::shared_ptr<Request>>& done)
{
    fs_status st = FS_OK;
    for (auto& q : running) {
        const hipError_t e = hipEventQuery(sv->slot_ev[q->slot]);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) {
            st = fail(FS_ERR_DEVICE, std::string("request failed: ") + hipGetErrorString(e));
            break;
        }
        const int R = q->p.n_replicas;
        q->history.assign((size_t)q->n_steps * R * 4, 0);
        for (size_t i = 0; i < q->history.size(); ++i) q->history[i] = q->pinned_hist[i];
        drop_sim(sv, *q);
        q->info.t_done = now_s();
        done.push_back(q);
    }
    return st;
}

// The worker.  Each iteration: (1) requests admitted last time join: small
// ones the batch, large ones a solo slot, where every step of theirs and the
// copy of their count history are queued at once on the slot's stream; (2)
// one round of steps is queued for the batch, and the count histories of the
// members it finishes are queued for copying right after it; (3) queued
// requests are admitted while that round runs; (4) the previous round is
// waited for and its finished members retired, and finished solo requests
// are retired.  The device thus has a round queued while the host works, and
// a large request's steps wait for no round.
void worker_loop(fs_server* sv)
{
    (void)hipSetDevice(sv->device);
    Round rounds[2];
    fs_status st = FS_OK;
    std::string err;
    for (auto& r : rounds)
        if (hipEventCreateWithFlags(&r.ev, hipEventDisableTiming) != hipSuccess) {
            r.ev = nullptr;
            st = FS_ERR_DEVICE;
            err = "event creation failed";
        }
    int cur = 0;
    std::vector<std::shared_ptr<Request>> joining;
    std::unique_lock<std::mutex> lk(sv->mu);
    while (st == FS_OK) {
        Round& prev = rounds[cur ^ 1];
        Round& now = rounds[cur];
        if (sv->active.empty() && joining.empty() && !prev.pending) {
            if (sv->stop && sv->queue.empty() && sv->running.empty()) break;
            if (sv->running.empty())
                sv->cv_work.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
            else // (solo requests to retire: look again shortly)
                sv->cv_work.wait_for(lk, std::chrono::microseconds(200), [&] { return !sv->queue.empty(); });
        }
        // 1. join: admitted sims (their setup stream is synchronised) move to
        //    the server stream and into the batch, or (large ones) to the
        //    stream of their solo slot with every step queued
        for (auto& q : joining) {
            q->sim->stream = sv->stream;
            fs_status jst = FS_OK;
            if (q->solo) {
                q->sim->stream = sv->solo_stream[q->slot];
                lk.unlock();
                jst = fs_step(q->sim, q->n_steps);
                const size_t bytes = (size_t)q->n_steps * q->p.n_replicas * 4 * sizeof(uint32_t);
                if (jst == FS_OK && (hipMemcpyAsync(q->pinned_hist, q->sim->d_hist, bytes, hipMemcpyDeviceToHost,
                                                    q->sim->stream) != hipSuccess ||
                                     hipEventRecord(sv->slot_ev[q->slot], q->sim->stream) != hipSuccess))
                    jst = fail(FS_ERR_DEVICE, "history copy");
                lk.lock();
            } else {
                jst = attach(sv->batch[q->g->d_weights ? 1 : 0], q->sim);
            }
            if (jst != FS_OK) {
                const std::string jerr = g_err;
                if (q->solo) (void)hipStreamSynchronize(q->sim->stream);
                drop_sim(sv, *q);
                if (q->solo) sv->slot_used[q->slot] = false;
                sv->in_use -= q->bytes;
                end_request(*q, jst, jerr);
                sv->cv_done.notify_all();
                continue;
            }
            (q->solo ? sv->running : sv->active).push_back(q);
        }
        joining.clear();
        // 2. queue one round of the batch
        now.ending.clear();
        now.pending = false;
        if (!sv->active.empty()) {
            int64_t r = sv->p.steps_per_round;
            for (auto& q : sv->active) r = std::min(r, q->n_steps - q->done_steps);
            std::vector<std::shared_ptr<Request>> act = sv->active;
            lk.unlock();
            for (fs_batch* b : sv->batch)
                if (st == FS_OK) st = batch_step(b, r);
            for (auto& q : act) {
                if (st != FS_OK) break;
                q->done_steps += r;
                if (q->done_steps < q->n_steps) continue;
                now.ending.push_back(q);
                const size_t bytes = (size_t)q->n_steps * q->p.n_replicas * 4 * sizeof(uint32_t);
                if (hipMemcpyAsync(q->pinned_hist, q->sim->d_hist, bytes, hipMemcpyDeviceToHost, q->sim->stream) !=
                    hipSuccess)
                    st = fail(FS_ERR_DEVICE, "history copy");
                if (q->sim->batch) detach(q->sim->batch, q->sim); // the next round's tables leave it out
            }
            if (st == FS_OK && hipEventRecord(now.ev, sv->stream) != hipSuccess) st = fail(FS_ERR_DEVICE, "event record");
            if (st != FS_OK) err = g_err;
            now.pending = st == FS_OK;
            lk.lock();
            for (auto& q : now.ending)
                sv->active.erase(std::remove(sv->active.begin(), sv->active.end(), q), sv->active.end());
            if (st != FS_OK) break;
        }
        // 3. admissions while the round runs: arrival order, except that a
        //    large request waiting for a solo slot does not hold back smaller
        //    ones; within the slot limit and the memory budget
        for (auto it = sv->queue.begin(); it != sv->queue.end();) {
            std::shared_ptr<Request> q = *it;
            q->solo = (size_t)q->g->n * (size_t)q->p.n_replicas >= SOLO_UNITS;
            const bool idle = sv->active.empty() && sv->running.empty() && joining.empty() && !now.pending &&
                              !prev.pending;
            if ((int)(sv->active.size() + sv->running.size() + joining.size()) >= sv->p.max_active) break;
            if (!idle && sv->in_use + q->bytes > sv->budget) break;
            int slot = -1;
            if (q->solo) {
                for (int i = 0; i < MAX_SOLO && slot < 0; ++i)
                    if (!sv->slot_used[i]) slot = i;
                if (slot < 0) {
                    ++it;
                    continue;
                }
                sv->slot_used[slot] = true;
                q->slot = slot;
            }
            sv->queue.erase(it);
            sv->in_use += q->bytes;
            lk.unlock();
            q->info.t_admit = now_s();
            const fs_status ast = start_request(sv, *q);
            const std::string aerr = ast == FS_OK ? std::string() : g_err;
            if (ast != FS_OK) drop_sim(sv, *q);
            lk.lock();
            if (ast != FS_OK) {
                sv->in_use -= q->bytes;
                if (q->solo) sv->slot_used[q->slot] = false;
                end_request(*q, ast, aerr);
                sv->cv_done.notify_all();
            } else {
                joining.push_back(q);
            }
            it = sv->queue.begin(); // the queue may have grown while unlocked
        }
        // 4. retire the previous round's finished requests
        if (prev.pending) {
            lk.unlock();
            if (hipEventSynchronize(prev.ev) != hipSuccess) {
                st = fail(FS_ERR_DEVICE, "round failed");
                err = g_err;
            }
            for (auto& q : prev.ending) {
                if (st == FS_OK) {
                    const int R = q->p.n_replicas;
                    q->history.assign((size_t)q->n_steps * R * 4, 0);
                    for (size_t i = 0; i < q->history.size(); ++i) q->history[i] = q->pinned_hist[i];
                }
                drop_sim(sv, *q);
                q->info.t_done = now_s();
            }
            lk.lock();
            ++sv->rounds;
            for (auto& q : prev.ending) {
                sv->in_use -= q->bytes;
                end_request(*q, st, err);
            }
            if (!prev.ending.empty()) sv->cv_done.notify_all();
            prev.ending.clear();
            prev.pending = false;
        }
        //    and the solo requests that have finished
        if (st == FS_OK && !sv->running.empty()) {
            std::vector<std::shared_ptr<Request>> running = sv->running, done;
            lk.unlock();
            st = retire_solos(sv, running, done);
            if (st != FS_OK) err = g_err;
            lk.lock();
            for (auto& q : done) {
                sv->running.erase(std::remove(sv->running.begin(), sv->running.end(), q), sv->running.end());
                sv->slot_used[q->slot] = false;
                sv->in_use -= q->bytes;
                end_request(*q, FS_OK, std::string());
            }
            if (!done.empty()) sv->cv_done.notify_all();
        }
        cur ^= 1;
    }
    if (st != FS_OK) {
        // a device failure ends every request and the server
        sv->worker_error = err;
        lk.unlock();
        (void)hipStreamSynchronize(sv->stream);
        for (hipStream_t ss : sv->solo_stream)
            if (ss) (void)hipStreamSynchronize(ss);
        lk.lock();
        for (auto& r : rounds) {
            for (auto& q : r.ending) {
                drop_sim(sv, *q);
                sv->in_use -= q->bytes;
                end_request(*q, st, err);
            }
            r.ending.clear();
        }
        for (auto* list : {&sv->active, &sv->running, &joining}) {
            for (auto& q : *list) {
                drop_sim(sv, *q);
                sv->in_use -= q->bytes;
                end_request(*q, st, err);
            }
            list->clear();
        }
        for (auto& q : sv->queue) end_request(*q, st, err);
        sv->queue.clear();
        sv->stop = true;
        sv->cv_done.notify_all();
    }
    lk.unlock();
    (void)hipStreamSynchronize(sv->stream);
    for (hipStream_t ss : sv->solo_stream)
        if (ss) (void)hipStreamSynchronize(ss);
    for (auto& r : rounds)
        if (r.ev) (void)hipEventDestroy(r.ev);
}

} // namespace

extern "C" {

fs_status fs_server_create(const fs_server_params* p, fs_server** out)
{
    FS_GUARD_BEGIN
    if (!out) return fail(FS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!p) return fail(FS_ERR_INVALID_ARG, "params is NULL");
    if (p->storage != FS_STORAGE_FP32 && p->storage != FS_STORAGE_COMPACT)
        return fail(FS_ERR_INVALID_ARG, "unknown storage");
    if (p->memory_budget < 0 || p->max_active < 0 || p->steps_per_round < 0)
        return fail(FS_ERR_INVALID_ARG, "negative limit");
    std::unique_ptr<fs_server> sv(new fs_server());
    sv->p = *p;
    if (sv->p.max_active == 0) sv->p.max_active = 64;
    if (sv->p.steps_per_round == 0) sv->p.steps_per_round = 25;
    FS_HIP(hipGetDevice(&sv->device));
    if (p->memory_budget > 0) {
        sv->budget = (size_t)p->memory_budget;
    } else {
        size_t free_b = 0, total_b = 0;
        FS_HIP(hipMemGetInfo(&free_b, &total_b));
        sv->budget = free_b / 10 * 8;
    }
    if (p->stream) {
        sv->stream = (hipStream_t)p->stream;
    } else {
        FS_HIP(hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking));
        sv->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&sv->admit_stream, hipStreamNonBlocking) != hipSuccess) {
        if (sv->own_stream) (void)hipStreamDestroy(sv->stream);
        return fail(FS_ERR_DEVICE, "admission stream");
    }
    for (int i = 0; i < MAX_SOLO; ++i)
        if (hipStreamCreateWithFlags(&sv->solo_stream[i], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sv->slot_ev[i], hipEventDisableTiming) != hipSuccess) {
            for (int j = 0; j <= i; ++j) {
                if (sv->solo_stream[j]) (void)hipStreamDestroy(sv->solo_stream[j]);
                if (sv->slot_ev[j]) (void)hipEventDestroy(sv->slot_ev[j]);
            }
            (void)hipStreamDestroy(sv->admit_stream);
            if (sv->own_stream) (void)hipStreamDestroy(sv->stream);
            return fail(FS_ERR_DEVICE, "solo stream");
        }
    fs_status st = FS_OK;
    for (fs_batch*& b : sv->batch)
        if (st == FS_OK) st = fs_batch_create(p->storage, sv->stream, &b);
    if (st != FS_OK) {
        const std::string err = g_err;
        for (fs_batch* b : sv->batch)
            if (b) (void)fs_batch_destroy(b);
        (void)hipStreamDestroy(sv->admit_stream);
        for (hipStream_t t : sv->solo_stream) (void)hipStreamDestroy(t);
        for (hipEvent_t e : sv->slot_ev) (void)hipEventDestroy(e);
        if (sv->own_stream) (void)hipStreamDestroy(sv->stream);
        return fail(st, err);
    }
    fs_server* raw = sv.release();
    raw->worker = std::thread(worker_loop, raw);
    *out = raw;
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_server_submit(fs_server* sv, const fs_request* rq, int64_t* id)
{
    FS_GUARD_BEGIN
    if (!sv || !rq || !id) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    *id = 0;
    if (!rq->graph) return fail(FS_ERR_INVALID_ARG, "request graph is NULL");
    if (rq->n_steps < 1 || rq->n_steps > (1 << 20)) return fail(FS_ERR_INVALID_ARG, "n_steps must be in [1, 2^20]");
    if (rq->n_seeds < 0 || (rq->n_seeds > 0 && !rq->seeds)) return fail(FS_ERR_INVALID_ARG, "bad seed list");
    if (rq->graph->device != sv->device) return fail(FS_ERR_INVALID_ARG, "graph is on another device");
    if (rq->params.n_replicas < 1 || rq->params.n_replicas > 64) return fail(FS_ERR_INVALID_ARG, "n_replicas out of range");
    if (rq->params.adaptive) return fail(FS_ERR_INVALID_ARG, "the server runs fixed-step requests only");
    if (rq->params.shedding != FS_SHED_CONSTANT || rq->params.compaction)
        return fail(FS_ERR_INVALID_ARG, "the server runs constant-shedding requests without compaction only");
    for (int64_t j = 0; j < rq->n_seeds; ++j)
        if (rq->seeds[j] < 0 || rq->seeds[j] >= rq->graph->n) return fail(FS_ERR_INVALID_ARG, "seed node out of range");
    auto q = std::make_shared<Request>();
    q->g = rq->graph;
    q->p = rq->params;
    q->p.storage = sv->p.storage;
    q->p.variant = 1;
    q->p.steps_per_graph = 0;
    q->p.history_len = (int32_t)std::max<int64_t>(rq->n_steps, 2);
    q->n_steps = rq->n_steps;
    q->seeds.assign(rq->seeds, rq->seeds + rq->n_seeds);
    q->bytes = sim_footprint(q->g, &q->p);
    q->info.n_steps = rq->n_steps;
    q->info.n_replicas = rq->params.n_replicas;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return fail(FS_ERR_DEVICE, "server stopped: " + sv->worker_error);
    if (q->bytes > sv->budget) return fail(FS_ERR_BUDGET, "request needs more device memory than the server budget");
    q->id = sv->next_id++;
    q->info.t_submit = now_s();
    q->g->users.fetch_add(1);
    sv->requests[q->id] = q;
    sv->queue.push_back(q);
    sv->cv_work.notify_one();
    *id = q->id;
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_server_wait(fs_server* sv, int64_t id, double timeout_s, int32_t* done)
{
    FS_GUARD_BEGIN
    if (!sv || !done) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    *done = 0;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->requests.find(id);
    if (it == sv->requests.end()) return fail(FS_ERR_INVALID_ARG, "unknown request id");
    std::shared_ptr<Request> q = it->second;
    auto ready = [&] { return q->finished; };
    if (timeout_s < 0) sv->cv_done.wait(lk, ready);
    else sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
    *done = q->finished ? 1 : 0;
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_server_result(fs_server* sv, int64_t id, int64_t* history, fs_request_info* info)
{
    FS_GUARD_BEGIN
    if (!sv) return fail(FS_ERR_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->requests.find(id);
    if (it == sv->requests.end()) return fail(FS_ERR_INVALID_ARG, "unknown request id");
    std::shared_ptr<Request> q = it->second;
    if (!q->finished) return fail(FS_ERR_BUSY, "request not finished");
    if (info) *info = q->info;
    sv->requests.erase(it);
    if (q->info.status != FS_OK) return fail(q->info.status, "request failed: " + q->error);
    if (history) std::copy(q->history.begin(), q->history.end(), history);
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_server_stats(fs_server* sv, fs_server_stats_t* out)
{
    if (!sv || !out) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    out->queued = (int64_t)sv->queue.size();
    out->active = (int64_t)(sv->active.size() + sv->running.size());
    out->memory_in_use = (int64_t)sv->in_use;
    out->memory_budget = (int64_t)sv->budget;
    out->rounds = (int64_t)sv->rounds;
    return FS_OK;
}

fs_status fs_server_destroy(fs_server* sv)
{
    FS_GUARD_BEGIN
    if (!sv) return fail(FS_ERR_INVALID_ARG, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        // queued requests are cancelled; admitted ones run to completion
        for (auto& q : sv->queue) {
            q->info.status = FS_ERR_BUSY;
            q->error = "cancelled: server destroyed";
            q->finished = true;
            q->g->users.fetch_sub(1);
        }
        sv->queue.clear();
        sv->stop = true;
        sv->cv_work.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    const std::string err = sv->worker_error;
    {
        DeviceGuard dg(sv->device);
        for (fs_batch* b : sv->batch) (void)fs_batch_destroy(b);
        (void)hipStreamSynchronize(sv->admit_stream);
        (void)hipStreamDestroy(sv->admit_stream);
        for (hipStream_t ss : sv->solo_stream) {
            (void)hipStreamSynchronize(ss);
            (void)hipStreamDestroy(ss);
        }
        for (hipEvent_t e : sv->slot_ev) (void)hipEventDestroy(e);
        if (sv->own_stream) (void)hipStreamDestroy(sv->stream);
    }
    delete sv;
    if (!err.empty()) return fail(FS_ERR_DEVICE, "server failed: " + err);
    return FS_OK;
    FS_GUARD_END
}

double fs_server_clock(void) { return now_s(); }

} // extern "C"
