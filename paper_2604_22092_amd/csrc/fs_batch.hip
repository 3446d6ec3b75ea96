// Batches and the scenario server of the C ABI declared in include/fs.h.
//
// A batch advances several simulations (each with its own graph, laws,
// replicas and step index) by one fused launch per step: a table of the
// members' step arguments and a block-range table let every workgroup find
// its member, and the per-step counts of all members are reduced by one
// launch per sequence.  Each member runs exactly the streaming step it would
// run alone, so its results are the same alone and in the batch.
//
// The server keeps a queue of scenario requests and one batch.  A worker
// thread admits queued requests while the memory budget and the slot limit
// allow, runs the batch a few steps at a time, and retires the requests that
// are done, so requests that arrive while others run join the next launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
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

struct fs_batch {
    int device = 0;
    int storage = 0;
    int weighted = -1; // fixed by the first member
    int rates = -1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<fs_sim*> members;
    bool dirty = true;
    // device tables, rebuilt when the membership changes
    StepArgs* d_table = nullptr;
    uint32_t* d_first = nullptr;
    fsi::HeavyArgs* d_htable = nullptr;
    uint32_t* d_hfirst = nullptr;
    fsi::RedArgs* d_red = nullptr;
    fsi::Ctl** d_ctls = nullptr;
    size_t cap = 0;
    uint32_t blocks = 0, hblocks = 0, hmembers = 0;
    uint32_t chunk = 0; // longest launch sequence (partial slots of the members)
    // host copies of the tables (kept alive for the asynchronous uploads)
    std::vector<StepArgs> h_table;
    std::vector<uint32_t> h_first, h_hfirst;
    std::vector<fsi::HeavyArgs> h_htable;
    std::vector<fsi::RedArgs> h_red;
    std::vector<fsi::Ctl*> h_ctls;
};

namespace {

#define FS_GUARD_BEGIN try {
#define FS_GUARD_END                                                                            \
    }                                                                                           \
    catch (const std::bad_alloc&) { return fail(FS_ERR_OUT_OF_MEMORY, "host allocation failed"); } \
    catch (const std::exception& e) { return fail(FS_ERR_DEVICE, e.what()); }                   \
    catch (...) { return fail(FS_ERR_DEVICE, "unknown exception"); }

void free_tables(fs_batch* b)
{
    dev_free(b->d_table);
    dev_free(b->d_first);
    dev_free(b->d_htable);
    dev_free(b->d_hfirst);
    dev_free(b->d_red);
    dev_free(b->d_ctls);
    b->d_table = nullptr;
    b->d_first = nullptr;
    b->d_htable = nullptr;
    b->d_hfirst = nullptr;
    b->d_red = nullptr;
    b->d_ctls = nullptr;
    b->cap = 0;
}

fs_status rebuild_tables(fs_batch* b)
{
    const size_t M = b->members.size();
    // the previous uploads read the host copies: let them finish first
    FS_HIP(hipStreamSynchronize(b->stream));
    if (M > b->cap) {
        free_tables(b);
        const size_t cap = std::max<size_t>(M, 16);
        FS_HIP(dev_alloc((void**)&b->d_table, cap * sizeof(StepArgs)));
        FS_HIP(dev_alloc((void**)&b->d_first, (cap + 1) * sizeof(uint32_t)));
        FS_HIP(dev_alloc((void**)&b->d_htable, cap * sizeof(fsi::HeavyArgs)));
        FS_HIP(dev_alloc((void**)&b->d_hfirst, (cap + 1) * sizeof(uint32_t)));
        FS_HIP(dev_alloc((void**)&b->d_red, cap * sizeof(fsi::RedArgs)));
        FS_HIP(dev_alloc((void**)&b->d_ctls, cap * sizeof(fsi::Ctl*)));
        b->cap = cap;
    }
    b->h_table.clear();
    b->h_first.assign(1, 0u);
    b->h_htable.clear();
    b->h_hfirst.assign(1, 0u);
    b->h_red.clear();
    b->h_ctls.clear();
    b->chunk = 1u << 30;
    for (fs_sim* s : b->members) {
        b->h_table.push_back(s->args);
        b->h_first.push_back(b->h_first.back() + s->G);
        if (s->nseg) {
            b->h_htable.push_back(heavy_args(s));
            b->h_hfirst.push_back(b->h_hfirst.back() + heavy_grid(s));
        }
        fsi::RedArgs r{};
        r.ctl = s->d_ctl;
        r.part = s->d_part;
        r.hist = s->d_hist;
        r.G = s->G;
        r.C = 4u * (uint32_t)s->R;
        r.H = (uint32_t)s->H;
        b->h_red.push_back(r);
        b->h_ctls.push_back(s->d_ctl);
        b->chunk = std::min(b->chunk, s->chunk);
    }
    b->blocks = b->h_first.back();
    b->hblocks = b->h_hfirst.back();
    b->hmembers = (uint32_t)b->h_htable.size();
    if (M) {
        FS_HIP(hipMemcpyAsync(b->d_table, b->h_table.data(), M * sizeof(StepArgs), hipMemcpyHostToDevice, b->stream));
        FS_HIP(hipMemcpyAsync(b->d_first, b->h_first.data(), (M + 1) * sizeof(uint32_t), hipMemcpyHostToDevice,
                              b->stream));
        FS_HIP(hipMemcpyAsync(b->d_red, b->h_red.data(), M * sizeof(fsi::RedArgs), hipMemcpyHostToDevice, b->stream));
        FS_HIP(hipMemcpyAsync(b->d_ctls, b->h_ctls.data(), M * sizeof(fsi::Ctl*), hipMemcpyHostToDevice, b->stream));
        if (b->hmembers) {
            FS_HIP(hipMemcpyAsync(b->d_htable, b->h_htable.data(), b->hmembers * sizeof(fsi::HeavyArgs),
                                  hipMemcpyHostToDevice, b->stream));
            FS_HIP(hipMemcpyAsync(b->d_hfirst, b->h_hfirst.data(), (b->hmembers + 1) * sizeof(uint32_t),
                                  hipMemcpyHostToDevice, b->stream));
        }
    }
    b->dirty = false;
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
    const void* kfn = fsk::step_batch_kernel_fn(b->storage, b->weighted == 1, b->rates == 1);
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
    FS_HIP(hipLaunchKernel(fsk::reduce_batch_kernel_fn(), dim3(r, M), dim3(WG), rargv, 0, b->stream));
    uint32_t members = M, rr = r;
    void* aargv[] = {&b->d_ctls, &members, &rr};
    FS_HIP(hipLaunchKernel(fsk::advance_batch_kernel_fn(), dim3((M + 63) / 64), dim3(64), aargv, 0, b->stream));
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
    free_tables(b);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    if (e != hipSuccess) return fail(FS_ERR_DEVICE, std::string("pending work failed: ") + hipGetErrorString(e));
    return FS_OK;
    FS_GUARD_END
}

fs_status fs_batch_add(fs_batch* b, fs_sim* s)
{
    FS_GUARD_BEGIN
    if (!b || !s) return fail(FS_ERR_INVALID_ARG, "NULL argument");
    if (s->batch) return fail(FS_ERR_BUSY, "sim already belongs to a batch");
    if (s->device != b->device) return fail(FS_ERR_INVALID_ARG, "sim and batch are on different devices");
    if (s->mode != fsi::MODE_STREAM)
        return fail(FS_ERR_INVALID_ARG, "batch members run the streaming step: create the sim with variant = 1");
    if (s->storage != b->storage) return fail(FS_ERR_INVALID_ARG, "sim storage differs from the batch's");
    const int w = s->g->d_weights != nullptr, rt = s->d_rates != nullptr;
    if (!b->members.empty() && (w != b->weighted || rt != b->rates))
        return fail(FS_ERR_INVALID_ARG, "batch members must agree on weights and record_rates");
    DeviceGuard dg(b->device);
    FS_HIP(hipStreamSynchronize(s->stream));
    b->weighted = w;
    b->rates = rt;
    s->saved_stream = s->stream;
    s->stream = b->stream;
    s->batch = b;
    b->members.push_back(s);
    b->dirty = true;
    return FS_OK;
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
    if (n_steps == 0 || b->members.empty()) return FS_OK;
    DeviceGuard dg(b->device);
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

struct Request {
    int64_t id = 0;
    fs_graph* g = nullptr;
    fs_sim_params p{};
    int64_t n_steps = 0;
    std::vector<int64_t> seeds;
    size_t bytes = 0;
    fs_sim* sim = nullptr;
    bool solo = false;             // runs its own step kernels instead of joining the batch
    int64_t done_steps = 0;
    fs_request_info info{};
    std::vector<int64_t> history; // [n_steps][R][4]
    std::string error;
    bool finished = false;
};

} // namespace

struct fs_server {
    fs_server_params p{};
    int device = 0;
    hipStream_t stream = nullptr;       // rounds: every admitted request's steps
    hipStream_t admit_stream = nullptr; // creation and seeding of new requests
    bool own_stream = false;
    fs_batch* batch = nullptr;
    size_t budget = 0, in_use = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;             // submitted, not admitted
    std::vector<std::shared_ptr<Request>> active;           // on the device
    std::map<int64_t, std::shared_ptr<Request>> requests;   // every request not yet collected
    int64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    std::string worker_error;
    uint64_t rounds = 0;
};

namespace {

// Requests with at least this many units give every wavefront of the GPU a
// chunk by themselves: they run their own step kernels (the variant that
// suits their size) on the server stream.  Smaller ones share the batch's
// fused launches.
constexpr size_t SOLO_UNITS = (size_t)1 << 18;

// Creates and seeds the sim of an admitted request on the admission stream,
// while the current round runs (worker thread).  The sim joins the rounds
// later (join_request).
fs_status start_request(fs_server* sv, Request& q)
{
    q.solo = (size_t)q.g->n * (size_t)q.p.n_replicas >= SOLO_UNITS;
    fs_sim_params p = q.p;
    p.storage = sv->p.storage;
    p.variant = q.solo ? 0 : 1;
    p.steps_per_graph = 0;
    p.history_len = (int32_t)std::max<int64_t>(q.n_steps, 2);
    p.stream = sv->admit_stream;
    p.record_rates = 0;
    fs_status st = fs_sim_create(q.g, &p, &q.sim);
    if (st != FS_OK) return st;
    if (!q.seeds.empty() && (st = fs_sim_seed(q.sim, -1, (int64_t)q.seeds.size(), q.seeds.data(), FS_E)) != FS_OK)
        return st;
    return FS_OK;
}

// Moves a created sim onto the server stream (its setup on the admission
// stream is complete: fs_sim_seed synchronised it) and, unless it runs solo,
// into the batch.  Called between rounds.
fs_status join_request(fs_server* sv, Request& q)
{
    q.sim->stream = sv->stream;
    return q.solo ? FS_OK : fs_batch_add(sv->batch, q.sim);
}

void drop_sim(fs_server* sv, Request& q)
{
    if (!q.sim) return;
    if (q.sim->batch) (void)fs_batch_remove(sv->batch, q.sim);
    (void)fs_sim_destroy(q.sim);
    q.sim = nullptr;
}

// Copies a finished request's counts and releases its sim (worker thread,
// between rounds).
fs_status finish_request(fs_server* sv, Request& q)
{
    const int R = q.p.n_replicas;
    fs_status st = q.sim->batch ? fs_batch_remove(sv->batch, q.sim) : FS_OK;
    if (st == FS_OK) {
        q.history.assign((size_t)q.n_steps * R * 4, 0);
        std::vector<int64_t> one((size_t)q.n_steps * 4);
        for (int r = 0; r < R && st == FS_OK; ++r) {
            st = fs_history(q.sim, r, 0, q.n_steps, one.data());
            for (int64_t k = 0; k < q.n_steps && st == FS_OK; ++k)
                for (int c = 0; c < 4; ++c) q.history[((size_t)k * R + r) * 4 + c] = one[(size_t)k * 4 + c];
        }
    }
    drop_sim(sv, q);
    return st;
}


// Ends request q with status st (the lock is held).
void end_request(fs_server* sv, Request& q, fs_status st, const std::string& err)
{
    q.info.status = st;
    if (st != FS_OK) q.error = err;
    if (q.info.t_done == 0.0) q.info.t_done = now_s();
    q.finished = true;
    q.g->users.fetch_sub(1);
}

// The worker: each iteration launches one round of steps for the active
// requests, admits queued requests while that round runs, waits for it,
// retires the requests that are done and lets the new ones join.
void worker_loop(fs_server* sv)
{
    (void)hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    std::vector<std::shared_ptr<Request>> joining;
    while (true) {
        if (sv->active.empty() && joining.empty()) {
            if (sv->stop && sv->queue.empty()) break;
            sv->cv_work.wait(lk, [&] { return sv->stop || !sv->queue.empty(); });
            if (sv->queue.empty()) continue;
        }
        // 1. launch one round: every active request advances by r steps,
        //    r bounded by the request closest to its end
        int64_t r = sv->p.steps_per_round;
        for (auto& q : sv->active) r = std::min(r, q->n_steps - q->done_steps);
        std::vector<std::shared_ptr<Request>> act = sv->active;
        lk.unlock();
        fs_status st = FS_OK;
        std::string err;
        if (!act.empty()) {
            st = fs_batch_step(sv->batch, r);
            for (auto& q : act)
                if (st == FS_OK && q->solo) st = fs_step(q->sim, r);
            if (st != FS_OK) err = g_err;
        }
        // 2. admissions (FIFO while the slot limit and the memory budget
        //    allow), overlapped with the round on the device
        lk.lock();
        while (st == FS_OK && !sv->queue.empty() &&
               (int)(sv->active.size() + joining.size()) < sv->p.max_active &&
               (sv->active.empty() && joining.empty() ? true : sv->in_use + sv->queue.front()->bytes <= sv->budget)) {
            std::shared_ptr<Request> q = sv->queue.front();
            sv->queue.pop_front();
            sv->in_use += q->bytes;
            lk.unlock();
            q->info.t_admit = now_s();
            const fs_status ast = start_request(sv, *q);
            const std::string aerr = ast == FS_OK ? std::string() : g_err;
            if (ast != FS_OK) drop_sim(sv, *q);
            lk.lock();
            if (ast != FS_OK) {
                sv->in_use -= q->bytes;
                end_request(sv, *q, ast, aerr);
                sv->cv_done.notify_all();
                continue;
            }
            joining.push_back(q);
        }
        lk.unlock();
        // 3. wait for the round
        if (!act.empty() && st == FS_OK) {
            st = fs_batch_sync(sv->batch);
            if (st != FS_OK) err = g_err;
        }
        // 4. retire the requests that are done; 5. the new ones join
        std::vector<std::shared_ptr<Request>> ended;
        for (auto& q : act) {
            q->done_steps += r;
            if (st != FS_OK || q->done_steps >= q->n_steps) ended.push_back(q);
        }
        std::vector<fs_status> fst(ended.size(), st);
        std::vector<std::string> ferr(ended.size(), err);
        for (size_t i = 0; i < ended.size(); ++i) {
            if (st == FS_OK) {
                fst[i] = finish_request(sv, *ended[i]);
                if (fst[i] != FS_OK) ferr[i] = g_err;
            } else {
                drop_sim(sv, *ended[i]);
            }
            ended[i]->info.t_done = now_s();
        }
        std::vector<std::shared_ptr<Request>> joined, failed;
        std::vector<std::string> jerr;
        for (auto& q : joining) {
            const fs_status jst = st == FS_OK ? join_request(sv, *q) : st;
            if (jst == FS_OK) {
                joined.push_back(q);
            } else {
                jerr.push_back(st == FS_OK ? g_err : err);
                drop_sim(sv, *q);
                failed.push_back(q);
            }
        }
        joining.clear();
        lk.lock();
        ++sv->rounds;
        for (size_t i = 0; i < ended.size(); ++i) {
            sv->active.erase(std::remove(sv->active.begin(), sv->active.end(), ended[i]), sv->active.end());
            sv->in_use -= ended[i]->bytes;
            end_request(sv, *ended[i], fst[i], ferr[i]);
        }
        for (size_t i = 0; i < failed.size(); ++i) {
            sv->in_use -= failed[i]->bytes;
            end_request(sv, *failed[i], st == FS_OK ? FS_ERR_DEVICE : st, jerr[i]);
        }
        for (auto& q : joined) sv->active.push_back(q);
        if (!ended.empty() || !failed.empty()) sv->cv_done.notify_all();
        if (st != FS_OK) {
            // a device failure ends every request and the server
            sv->worker_error = err;
            for (auto& q : sv->active) {
                drop_sim(sv, *q);
                sv->in_use -= q->bytes;
                end_request(sv, *q, st, err);
            }
            sv->active.clear();
            for (auto& q : sv->queue) end_request(sv, *q, st, err);
            sv->queue.clear();
            sv->stop = true;
            sv->cv_done.notify_all();
            break;
        }
    }
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
    fs_status st = fs_batch_create(p->storage, sv->stream, &sv->batch);
    if (st != FS_OK) {
        (void)hipStreamDestroy(sv->admit_stream);
        if (sv->own_stream) (void)hipStreamDestroy(sv->stream);
        return st;
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
    out->active = (int64_t)sv->active.size();
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
        // queued requests are cancelled; active ones run to completion
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
        (void)fs_batch_destroy(sv->batch);
        (void)hipStreamDestroy(sv->admit_stream);
        if (sv->own_stream) (void)hipStreamDestroy(sv->stream);
    }
    delete sv;
    if (!err.empty()) return fail(FS_ERR_DEVICE, "server failed: " + err);
    return FS_OK;
    FS_GUARD_END
}

double fs_server_clock(void) { return now_s(); }

} // extern "C"
