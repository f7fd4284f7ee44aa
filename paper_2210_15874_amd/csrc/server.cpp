// Job server: a native request loop that runs many trajectory-ensemble jobs
// (different circuits, sizes, noise rates and trajectory counts) on one
// device at once.
//
//   caller threads   stn_server_submit copies the job's inputs and returns.
//   planner threads  build (or take from the plan cache) the job's plan on
//                    the host and estimate its device memory; the device
//                    thread sees planned jobs in arrival order.
//   device thread    the only thread that calls HIP.  Admits planned jobs in
//                    arrival order while their estimated memory fits the
//                    budget, gives each admitted job a stream, and issues the
//                    jobs' work in chunks of trajectories (sample -> contract
//                    -> reduce), round-robin over the admitted jobs, so that
//                    chunks of jobs that arrived while others were running
//                    interleave with theirs on the device (continuous
//                    batching).  A job's draws depend only on (its seed, k,
//                    site), and its reduction is in trajectory order, so its
//                    result does not depend on what else ran beside it.
//
// Device memory: the whole byte budget is reserved once when the server
// starts and carved into blocks for plans, workspaces, batches and
// accumulators; blocks freed by finished jobs go to the next ones.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "stn_internal.h"

namespace stn {
namespace {

constexpr uint32_t kMaxStreams = 8;
constexpr uint32_t kMaxActive = 64;
constexpr uint32_t kChunksInFlight = 2;   // per job
constexpr int kPlanners = 4;              // host planning threads (a slow plan does not hold up the others)
constexpr double kSmallJobSeconds = 0.05;  // estimated device time of a job for the small-job stream
constexpr double kLongJobHold = 0.25;      // longest a long job waits for the small-job stream to drain
constexpr double kSmallChunkSeconds = 0.005;  // estimated device time of one chunk of a small job
constexpr uint32_t kTuneSample = 64;      // trajectories the autotuner times the launch shapes on
constexpr double kChunkTiles = 32768;     // statevector tiles per launch a chunk aims at

// ---------------------------------------------------------------- device pool
// One hipMalloc of the whole budget when the server starts; blocks are carved
// from it first-fit (256-byte aligned) and returned with their neighbours
// merged, so serving never calls hipMalloc / hipFree (which map and unmap
// memory and may wait for the device).
class DevicePool {
public:
    explicit DevicePool(uint64_t budget) : size_(budget / 256 * 256) {}
    ~DevicePool() {
        if (base_) (void)hipFree(base_);
    }

    // on the device thread, with the device current
    void init() {
        if (hipMalloc((void**)&base_, size_) != hipSuccess) {
            (void)hipGetLastError();
            base_ = nullptr;
            fail(STN_E_OOM, "could not reserve the server's device memory (" + std::to_string(size_) + " bytes)");
        }
        free_[0] = size_;
    }

    void* alloc(size_t bytes) {
        std::lock_guard<std::mutex> lk(m_);
        const uint64_t r = (std::max<uint64_t>(bytes, 1) + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < r) continue;
            const uint64_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > r) free_[off + r] = sz - r;
            used_[base_ + off] = r;
            in_use_ += r;
            peak_ = std::max(peak_, in_use_);
            return base_ + off;
        }
        return nullptr;
    }

    void release(void* p) {
        std::lock_guard<std::mutex> lk(m_);
        auto u = used_.find(static_cast<char*>(p));
        if (u == used_.end()) return;
        uint64_t off = (uint64_t)(u->first - base_), sz = u->second;
        used_.erase(u);
        in_use_ -= sz;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + sz) {
            sz += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += sz;
                return;
            }
        }
        free_[off] = sz;
    }

    uint64_t in_use() const { std::lock_guard<std::mutex> lk(m_); return in_use_; }
    uint64_t cached() const { std::lock_guard<std::mutex> lk(m_); return size_ - in_use_; }
    uint64_t peak() const { std::lock_guard<std::mutex> lk(m_); return peak_; }

private:
    mutable std::mutex m_;
    char* base_ = nullptr;
    uint64_t size_, in_use_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;           // offset -> size
    std::unordered_map<char*, uint64_t> used_;    // block -> size
};

void* pool_alloc(size_t bytes, void* ctx) { return static_cast<DevicePool*>(ctx)->alloc(bytes); }
void pool_free(void* p, void* ctx) { static_cast<DevicePool*>(ctx)->release(p); }

// ---------------------------------------------------------------- job inputs
// Deep copy of (circuit, noise model, observable); `key` is their byte image,
// which identifies a plan in the cache.
struct Inputs {
    uint32_t n = 0;
    std::vector<stn_gate> gates;
    std::vector<double> gate_mats;
    std::vector<size_t> gate_mat_off;
    std::vector<stn_channel> chans;
    std::vector<double> kraus;
    std::vector<size_t> kraus_off;
    std::vector<uint32_t> uv;
    std::vector<double> w;
    std::string key;

    template <class T> static void put(std::string& k, const T& v) { k.append(reinterpret_cast<const char*>(&v), sizeof(T)); }

    void copy(const stn_circuit* c, const stn_noise_model* nm, const stn_observable* ob, uint32_t precision) {
        if (!c || (c->n_gates && !c->gates)) fail(STN_E_INVALID, "circuit is NULL");
        n = c->n_qubits;
        put(key, n);
        put(key, precision);
        gates.assign(c->gates, c->gates + c->n_gates);
        for (auto& g : gates) {
            put(key, g.kind); put(key, g.q0); put(key, g.q1); put(key, g.theta);
            const size_t cnt = g.kind == STN_G_U1 ? 8 : g.kind == STN_G_U2 ? 32 : 0;
            gate_mat_off.push_back(gate_mats.size());
            if (cnt) {
                if (!g.mat) fail(STN_E_INVALID, "explicit gate without a matrix");
                gate_mats.insert(gate_mats.end(), g.mat, g.mat + cnt);
                for (size_t i = 0; i < cnt; ++i) put(key, g.mat[i]);
            }
        }
        if (nm && nm->n_channels) {
            if (!nm->channels) fail(STN_E_INVALID, "noise model channels are NULL");
            chans.assign(nm->channels, nm->channels + nm->n_channels);
        }
        for (auto& ch : chans) {
            put(key, ch.after_gate); put(key, ch.kind); put(key, ch.n_qubits); put(key, ch.q0); put(key, ch.q1);
            put(key, ch.param); put(key, ch.n_kraus);
            kraus_off.push_back(kraus.size());
            if (ch.kind == STN_CH_KRAUS) {
                const size_t d = ch.n_qubits == 2 ? 4 : 2, cnt = (size_t)ch.n_kraus * d * d * 2;
                if (!ch.kraus || cnt == 0) fail(STN_E_INVALID, "explicit channel without operators");
                kraus.insert(kraus.end(), ch.kraus, ch.kraus + cnt);
                for (size_t i = 0; i < cnt; ++i) put(key, ch.kraus[i]);
            }
        }
        if (ob && ob->n_terms) {
            if (!ob->uv || !ob->w) fail(STN_E_INVALID, "observable arrays are NULL");
            uv.assign(ob->uv, ob->uv + 2 * (size_t)ob->n_terms);
            w.assign(ob->w, ob->w + ob->n_terms);
            for (auto x : uv) put(key, x);
            for (auto x : w) put(key, x);
        }
        // pointers into the owned copies
        for (size_t i = 0; i < gates.size(); ++i)
            gates[i].mat = (gates[i].kind == STN_G_U1 || gates[i].kind == STN_G_U2) ? gate_mats.data() + gate_mat_off[i] : nullptr;
        for (size_t i = 0; i < chans.size(); ++i)
            chans[i].kraus = chans[i].kind == STN_CH_KRAUS ? kraus.data() + kraus_off[i] : nullptr;
    }
};

// ---------------------------------------------------------------- jobs
enum class JobState { Planning, Ready, Active, Finishing, Done };

struct Job {
    uint64_t id = 0, tag = 0, seed = 0, K = 0;
    Inputs in;
    stn_plan* plan = nullptr;
    stn_status status = STN_OK;
    std::string err;
    double t_submit = 0, t_admit = 0, t_done = 0;
    double t_ready = 0;                // planning finished
    double est_s = 0;                  // estimated device seconds of the whole job
    uint64_t est_bytes = 0;
    uint32_t B = 0;                    // trajectories per chunk
    // device-side state (device thread only)
    int stream = -1;
    stn_accum* acc = nullptr;
    stn_batch* batch[kChunksInFlight] = {};
    hipEvent_t ev[kChunksInFlight] = {};
    bool ev_live[kChunksInFlight] = {};
    hipEvent_t done_ev = nullptr;
    uint64_t k_issued = 0;
    uint32_t next = 0;
    uint32_t slot = 0;                 // pinned result slot
    uint64_t chunks = 0;
    bool finishing = false;
    bool tune = false;                 // autotune the launch shape on a sample of the first chunk
    uint64_t shape = 0;                // tuning cache key
};

}  // namespace
}  // namespace stn

struct stn_server {
    stn_server_opts opts{};
    std::chrono::steady_clock::time_point t0;
    std::unique_ptr<stn::DevicePool> pool;
    int device = 0;

    std::mutex m;                          // guards the queues, cache, results and stats below
    std::condition_variable cv_plan, cv_ready, cv_done;
    std::deque<std::shared_ptr<stn::Job>> to_plan, ready;
    uint32_t planning = 0;                 // jobs a planner thread is working on
    std::deque<stn_job_result> results;
    std::list<std::pair<std::string, stn_plan*>> cache;   // idle plans, most recent first
    uint64_t next_id = 1;
    uint64_t submitted = 0, completed = 0, planned = 0, inflight_jobs = 0;
    stn_server_stats st{};
    bool stop = false;
    bool started = false;                  // device thread initialised (memory reserved)
    std::string fatal;

    std::vector<std::thread> planners;
    std::thread worker;

    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace stn {
namespace {

// ---------------------------------------------------------------- planner
uint64_t estimate_bytes(const stn_plan* p, uint32_t B, uint64_t K) {
    const double S = (double)p->sites.size();
    const double words = std::max<double>(1.0, std::ceil(p->gates.size() / 32.0));
    double b = 0;
    const double N = std::ldexp(1.0, (int)p->n);
    const double elem = p->opts.precision == 128 ? 16.0 : 8.0;
    if (p->kind == STN_PLAN_SV_TILED) b += (double)B * N * elem + (double)B * std::ldexp(1.0, (int)p->n - (int)p->tile_bits) * 8.0;
    if (p->kind == STN_PLAN_LIGHTCONE) b += (double)B * p->obs_u.size() * 8.0 + p->lc_arena_bytes;
    if (p->kind == STN_PLAN_SV_GATES) b += (double)B * (N * elem + 64.0 * 8.0);
    b += kChunksInFlight * (double)B * (S + 4.0 * words + 16.0 + 8.0);     // batches
    b += std::ceil((double)K / kEnergyChunk) * kEnergyChunk * 8.0 + 2.0 * K * 8.0;  // accumulator
    b += 8.0 * (1 << 20);                                                  // tables and rounding
    return (uint64_t)b;
}

void plan_job(stn_server* sv, Job& j) {
    stn_plan* p = nullptr;
    {
        std::lock_guard<std::mutex> lk(sv->m);
        for (auto it = sv->cache.begin(); it != sv->cache.end(); ++it)
            if (it->first == j.in.key) {
                p = it->second;
                sv->cache.erase(it);
                sv->st.plan_cache_hits++;
                break;
            }
        if (!p) sv->st.plan_cache_misses++;
    }
    if (!p) {
        stn_plan_opts o;
        stn_plan_opts_default(&o);
        o.precision = sv->opts.precision;
        o.outputs = STN_OUT_ENERGY;
        o.plan_kind = STN_PLAN_AUTO;
        // large jobs may fill at most 15/16 of the budget (the rest is for small ones)
        o.hbm_budget = (uint64_t)(std::min(sv->opts.job_share, 15.0 / 16.0) * (double)sv->opts.hbm_budget);
        o.max_batch = sv->opts.chunk_max;
        o.dev_alloc = pool_alloc;
        o.dev_free = pool_free;
        o.alloc_ctx = sv->pool.get();
        const stn_circuit c{j.in.n, (uint32_t)j.in.gates.size(), j.in.gates.data()};
        const stn_noise_model nm{(uint32_t)j.in.chans.size(), j.in.chans.data()};
        const stn_observable ob{(uint32_t)j.in.w.size(), j.in.uv.data(), j.in.w.data()};
        const stn_status s = stn_plan_create(&c, &nm, ob.n_terms ? &ob : nullptr, &o, &p);
        if (s != STN_OK) {
            j.status = s;
            j.err = stn_last_error();
            return;
        }
        p->sync_on_destroy = false;
    }
    j.plan = p;
    j.B = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(p->max_batch, j.K));
    // statevector chunks only as large as it takes to fill the device
    // (~32k tiles per launch): the rest of the memory serves other jobs
    if (p->kind == STN_PLAN_SV_TILED) {
        const int tile_bits = (int)p->tile_bits;
        const int stored = (int)p->n - (p->sv_half ? 1 : 0);   // half-state plans keep 2^(n-1) amplitudes
        const double tiles = std::ldexp(1.0, std::max(0, stored - tile_bits));
        // the same amplitudes per launch for 15-qubit tiles (half the tiles)
        const double target = tile_bits == 15 ? kChunkTiles / 2 : kChunkTiles;
        j.B = (uint32_t)std::max(1.0, std::min((double)j.B, std::ceil(target / tiles)));
    }
    j.est_s = p->est_seconds_per_traj() * (double)j.K;
    // a job for the small-job stream runs in chunks of about kSmallChunkSeconds,
    // so that the other small jobs' chunks are issued between its chunks
    // instead of waiting behind all of it
    if (j.est_s > kSmallChunkSeconds && j.est_s <= kSmallJobSeconds) {
        const double chunks = std::ceil(j.est_s / kSmallChunkSeconds);
        j.B = (uint32_t)std::max(1.0, std::min((double)j.B, std::ceil((double)j.K / chunks)));
    }
    j.est_bytes = estimate_bytes(p, j.B, j.K);
    const uint64_t budget = sv->opts.hbm_budget;
    if (j.est_bytes > budget / 32 && j.est_bytes > budget - budget / 16) {
        j.status = STN_E_OOM;
        j.err = "job needs more device memory than the server budget";
    }
}

void planner_loop(stn_server* sv) {
    tl_plan_threads = 1;   // jobs are planned in parallel by the planner threads themselves
    for (;;) {
        std::shared_ptr<Job> j;
        {
            std::unique_lock<std::mutex> lk(sv->m);
            sv->cv_plan.wait(lk, [&] { return sv->stop || !sv->to_plan.empty(); });
            if (sv->to_plan.empty() || (sv->stop && !sv->opts.drain_on_destroy)) return;
            j = sv->to_plan.front();
            sv->to_plan.pop_front();
            sv->planning++;
        }
        try {
            plan_job(sv, *j);
        } catch (const Error& e) {
            j->status = e.status;
            j->err = e.msg;
        } catch (const std::exception& e) {
            j->status = STN_E_INVALID;
            j->err = e.what();
        }
        {
            // admission sees planned jobs in arrival order
            std::lock_guard<std::mutex> lk(sv->m);
            auto pos = std::upper_bound(sv->ready.begin(), sv->ready.end(), j,
                                        [](const std::shared_ptr<Job>& a, const std::shared_ptr<Job>& b) {
                                            return a->id < b->id;
                                        });
            j->t_ready = sv->now();
            sv->ready.insert(pos, j);
            sv->planning--;
            sv->planned++;
        }
        sv->cv_ready.notify_one();
    }
}

// ---------------------------------------------------------------- device thread
struct Device {
    stn_server* sv;
    hipStream_t streams[kMaxStreams] = {};
    hipStream_t upload = nullptr;
    uint32_t stream_jobs[kMaxStreams] = {};
    double* pinned = nullptr;              // kMaxActive x 2 doubles: mean, SE
    std::vector<uint32_t> free_slots;
    std::vector<std::shared_ptr<Job>> active;
    std::unordered_map<uint64_t, uint32_t> tuned;   // shape key -> launch-shape variant
    std::vector<hipEvent_t> ev_pool;
    uint64_t bytes_admitted = 0;
    size_t rr = 0;
    uint32_t cus = 0;

    hipEvent_t event() {
        if (!ev_pool.empty()) {
            hipEvent_t e = ev_pool.back();
            ev_pool.pop_back();
            return e;
        }
        hipEvent_t e;
        STN_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        return e;
    }

    void init() {
        STN_HIP(hipSetDevice(sv->device));
        warm_device_code();
        sv->pool->init();
        int c = 0;
        STN_HIP(hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, sv->device));
        cus = (uint32_t)c;
        for (uint32_t i = 0; i < sv->opts.n_streams; ++i) STN_HIP(hipStreamCreateWithFlags(&streams[i], hipStreamNonBlocking));
        // table uploads and tuning runs get a stream of their own: the device
        // thread waits for them, and must not wait behind the small jobs' chunks
        STN_HIP(hipStreamCreateWithFlags(&upload, hipStreamNonBlocking));
        STN_HIP(hipHostMalloc((void**)&pinned, kMaxActive * 2 * sizeof(double), hipHostMallocDefault));
        for (uint32_t i = 0; i < kMaxActive; ++i) free_slots.push_back(kMaxActive - 1 - i);
    }

    void shutdown() {
        for (auto& j : active) (void)hipStreamSynchronize(streams[j->stream]);
        for (auto& j : active) release(*j);
        active.clear();
        for (uint32_t i = 0; i < sv->opts.n_streams; ++i)
            if (streams[i]) (void)hipStreamDestroy(streams[i]);
        if (upload) {
            (void)hipStreamSynchronize(upload);
            (void)hipStreamDestroy(upload);
        }
        for (auto e : ev_pool) (void)hipEventDestroy(e);
        ev_pool.clear();
        if (pinned) (void)hipHostFree(pinned);
    }

    // frees the job's device state (its work has completed) and returns the
    // plan to the cache
    void release(Job& j) {
        for (uint32_t c = 0; c < kChunksInFlight; ++c) {
            delete j.batch[c];
            j.batch[c] = nullptr;
            if (j.ev[c]) ev_pool.push_back(j.ev[c]);
            j.ev[c] = nullptr;
            j.ev_live[c] = false;
        }
        if (j.done_ev) ev_pool.push_back(j.done_ev);
        j.done_ev = nullptr;
        delete j.acc;
        j.acc = nullptr;
        if (j.stream >= 0) stream_jobs[j.stream]--;
        free_slots.push_back(j.slot);
        bytes_admitted -= j.est_bytes;
        if (j.plan) {
            j.plan->d_work.reset();
            j.plan->d_partials.reset();
            stn_plan* drop = nullptr;
            {
                std::lock_guard<std::mutex> lk(sv->m);
                if (sv->opts.plan_cache) {
                    sv->cache.push_front({j.in.key, j.plan});
                    if (sv->cache.size() > sv->opts.plan_cache) {
                        drop = sv->cache.back().second;
                        sv->cache.pop_back();
                    }
                } else {
                    drop = j.plan;
                }
            }
            delete drop;
            j.plan = nullptr;
        }
    }

    stn_job_result record(const Job& j, stn_status s, const std::string& err) {
        stn_job_result r{};
        r.job_id = j.id;
        r.tag = j.tag;
        r.status = (uint32_t)s;
        r.plan_kind = j.plan ? j.plan->kind : 0;
        r.width = j.plan ? j.plan->width : 0;
        r.K = j.K;
        r.k_done = s == STN_OK ? j.K : 0;
        r.chunk = j.B;
        r.chunks = j.chunks;
        r.t_submit = j.t_submit;
        r.t_admit = j.t_admit;
        r.t_done = sv->now();
        if (s == STN_OK) {
            r.energy_mean = pinned[2 * j.slot];
            r.energy_se = pinned[2 * j.slot + 1];
        }
        std::snprintf(r.error, sizeof(r.error), "%s", err.c_str());
        return r;
    }

    // results are published after the job's resources (and its plan, to the
    // cache) have been released, so a caller that saw the result finds them free
    void publish(const stn_job_result& r) {
        {
            std::lock_guard<std::mutex> lk(sv->m);
            sv->results.push_back(r);
            sv->completed++;
            if (r.status == STN_OK) sv->st.trajectories += r.K;
            else sv->st.failed++;
        }
        sv->cv_done.notify_all();
    }

    // Arrival order; when the oldest waiting job does not fit, a later job of
    // at most 1/32 of the budget that fits may go ahead of it (small jobs
    // barely delay the large one and are not held behind it).  Jobs above
    // that size may fill only 15/16 of the budget, so small jobs always find
    // room.  A long job (estimated over kSmallJobSeconds of device time, so
    // bound for the large-job streams) is held back while the small-job
    // stream has work or other jobs are still being planned (they may be
    // short), for at most kLongJobHold seconds after its planning finished:
    // short jobs then get the whole device first rather than the CUs a long
    // job's persistent kernels leave free; the first job not held takes the
    // oldest job's place in the rule above.
    bool admit() {
        std::shared_ptr<Job> j;
        {
            std::lock_guard<std::mutex> lk(sv->m);
            if (sv->ready.empty()) return false;
            const bool room = active.size() < sv->opts.max_active && !free_slots.empty();
            const uint64_t budget = sv->opts.hbm_budget, small = budget / 32;
            const uint64_t left = budget - std::min(budget, bytes_admitted);
            const uint64_t left_big = (budget - budget / 16) - std::min(budget - budget / 16, bytes_admitted);
            const double now = sv->now();
            const bool small_busy = hipStreamQuery(streams[0]) == hipErrorNotReady || !sv->to_plan.empty() ||
                                    sv->planning > 0;
            size_t pick = SIZE_MAX;
            bool head = true;
            for (size_t i = 0; i < sv->ready.size(); ++i) {
                const auto& c = sv->ready[i];
                if (c->status != STN_OK) { pick = i; break; }       // failed planning: report now
                if (!room) continue;
                const bool held = sv->opts.n_streams > 1 && c->est_s > kSmallJobSeconds && small_busy &&
                                  now - c->t_ready < kLongJobHold;
                if (held) continue;
                const bool is_small = c->est_bytes <= small;
                if (head) {
                    head = false;
                    if (c->est_bytes <= (is_small ? left : left_big)) { pick = i; break; }
                    continue;
                }
                if (is_small && c->est_bytes <= left) { pick = i; break; }
            }
            if (pick == SIZE_MAX) return false;
            j = sv->ready[pick];
            sv->ready.erase(sv->ready.begin() + (ptrdiff_t)pick);
        }
        if (j->status != STN_OK) {   // planning failed: report at once
            const stn_job_result r = record(*j, j->status, j->err);
            delete j->plan;
            j->plan = nullptr;
            publish(r);
            return true;
        }
        j->t_admit = sv->now();
        j->slot = free_slots.back();
        free_slots.pop_back();
        bytes_admitted += j->est_bytes;
        // Streams that share a hardware queue run one after the other, so the
        // server keeps few (three job streams and the upload stream fill the
        // four queues a process gets by default): stream 0 carries the small
        // jobs (estimated under 50 ms of device time), so that they never wait
        // behind a large job's chunks; large jobs take the least-loaded of the
        // others.
        uint32_t best = 0;
        if (sv->opts.n_streams > 1 && j->est_s > kSmallJobSeconds) {
            best = 1;
            for (uint32_t i = 2; i < sv->opts.n_streams; ++i)
                if (stream_jobs[i] < stream_jobs[best]) best = i;
        }
        j->stream = (int)best;
        stream_jobs[best]++;
        try {
            ensure_uploaded(j->plan, upload);
            // persistent kernels leave reserve_cus CUs to the other jobs
            if (sv->opts.reserve_cus && cus > sv->opts.reserve_cus) j->plan->grid_cap = cus - sv->opts.reserve_cus;
            j->plan->graphs = sv->opts.graphs != 0;
            choose_shape(*j);
            j->acc = new stn_accum();
            j->acc->plan = j->plan;
            for (uint32_t c = 0; c < kChunksInFlight; ++c) {
                j->batch[c] = new stn_batch();
                j->ev[c] = event();
            }
            j->done_ev = event();
        } catch (const Error& e) {
            fail_job(*j, e);
            return true;
        }
        active.push_back(j);
        std::lock_guard<std::mutex> lk(sv->m);
        sv->st.max_active_jobs = std::max<uint64_t>(sv->st.max_active_jobs, active.size());
        return true;
    }

    // Launch shape of the job's contraction: a cached choice for its shape, or
    // autotuning on its first chunk when that chunk is cheap (the device thread
    // waits for it); otherwise the default.
    void choose_shape(Job& j) {
        stn_plan* p = j.plan;
        if (p->tuned) return;
        const uint32_t lg = 32 - __builtin_clz(std::max<uint32_t>(j.B, 1));
        j.shape = (uint64_t)p->kind | ((uint64_t)p->opts.precision << 8) | ((uint64_t)p->n << 16) |
                  ((uint64_t)p->width << 24) | ((uint64_t)lg << 32);
        auto it = tuned.find(j.shape);
        if (it != tuned.end()) {
            if (stn_plan_set_variant(p, it->second) != STN_OK) throw Error{STN_E_STATE, stn_last_error()};
            return;
        }
        // estimated seconds for the tuning sample (all shapes, warm and timed)
        const double per = p->est_seconds_per_traj();
        // networks in HBM run long per work item: their default shape is kept.
        // The device thread waits for the tuning runs, so they are done only
        // while no other job occupies the device.
        const bool hbm_tier = p->kind == STN_PLAN_LIGHTCONE && p->lc_arena_bytes > 0;
        j.tune = !hbm_tier && active.empty() && per * std::min<uint32_t>(j.B, kTuneSample) * 8.0 < 0.005;
    }

    void fail_job(Job& j, const Error& e) {
        if (j.stream >= 0) (void)hipStreamSynchronize(streams[j.stream]);
        const stn_job_result r = record(j, e.status, e.msg);
        release(j);
        publish(r);
    }

    // one chunk of j onto its stream; false when nothing could be issued
    bool issue(Job& j) {
        if (j.k_issued >= j.K) return false;
        const uint32_t c = j.next;
        if (j.ev_live[c]) {
            if (hipEventQuery(j.ev[c]) == hipErrorNotReady) return false;
            j.ev_live[c] = false;
        }
        hipStream_t s = streams[j.stream];
        const uint32_t K = (uint32_t)std::min<uint64_t>(j.B, j.K - j.k_issued);
        stn_batch* b = j.batch[c];
        batch_prepare(j.plan, b, j.k_issued, K);
        if (j.tune) {
            // on the private stream: sample the first trajectories, time every
            // launch shape on them, keep the fastest for the shape
            stn_batch probe;
            batch_prepare(j.plan, &probe, 0, std::min<uint32_t>(K, kTuneSample));
            launch_sample(j.plan, &probe, j.seed, upload);
            if (j.plan->kind != STN_PLAN_SV_LDS && j.plan->kind != STN_PLAN_SV_GATES) launch_frame(j.plan, &probe, upload);
            stn_tune_result tr{};
            const stn_status st0 = stn_plan_autotune(j.plan, &probe, 1, &tr, upload);
            if (st0 != STN_OK) throw Error{st0, stn_last_error()};
            tuned[j.shape] = tr.chosen;
            j.tune = false;
            std::lock_guard<std::mutex> lk(sv->m);
            sv->st.autotuned++;
        }
        launch_sample(j.plan, b, j.seed, s);
        if (j.plan->kind != STN_PLAN_SV_LDS && j.plan->kind != STN_PLAN_SV_GATES) launch_frame(j.plan, b, s);
        const stn_status st1 = stn_contract(j.plan, b, s);
        if (st1 != STN_OK) throw Error{st1, stn_last_error()};
        const stn_status st2 = stn_reduce(j.plan, b, j.acc, s);
        if (st2 != STN_OK) throw Error{st2, stn_last_error()};
        STN_HIP(hipEventRecord(j.ev[c], s));
        j.ev_live[c] = true;
        j.next = (c + 1) % kChunksInFlight;
        j.k_issued += K;
        j.chunks++;
        std::lock_guard<std::mutex> lk(sv->m);
        sv->st.chunks++;
        return true;
    }

    // the chunk slot of j is free (its previous use has finished)
    bool slot_free(Job& j) {
        const uint32_t c = j.next;
        if (!j.ev_live[c]) return true;
        if (hipEventQuery(j.ev[c]) == hipErrorNotReady) return false;
        j.ev_live[c] = false;
        return true;
    }

    // Whole-state-in-LDS jobs on the shared stream with a chunk ready: their
    // chunks go out together, one multi-batch launch draining a device-side
    // queue of all their trajectories (each job's results are those of its own
    // launches, bit for bit).  True when something was issued.
    bool gang() {
        if (!sv->opts.gang) return false;
        std::vector<Job*> g;
        for (auto& jp : active) {
            Job& j = *jp;
            if (j.stream != 0 || !j.plan || j.plan->kind != STN_PLAN_SV_LDS || j.tune || j.k_issued >= j.K)
                continue;
            if (slot_free(j)) g.push_back(&j);
        }
        if (g.size() < 2) return false;
        hipStream_t s = streams[0];
        std::vector<stn_plan*> plans;
        std::vector<stn_batch*> batches;
        std::vector<uint32_t> ks;
        for (Job* j : g) {
            const uint32_t K = (uint32_t)std::min<uint64_t>(j->B, j->K - j->k_issued);
            stn_batch* b = j->batch[j->next];
            batch_prepare(j->plan, b, j->k_issued, K);
            launch_sample(j->plan, b, j->seed, s);
            plans.push_back(j->plan);
            batches.push_back(b);
            ks.push_back(K);
        }
        const stn_status st = stn_contract_many(plans.data(), batches.data(), (uint32_t)g.size(), s);
        if (st != STN_OK) throw Error{st, stn_last_error()};
        for (size_t i = 0; i < g.size(); ++i) {
            Job& j = *g[i];
            const uint32_t c = j.next;
            const stn_status st2 = stn_reduce(j.plan, batches[i], j.acc, s);
            if (st2 != STN_OK) throw Error{st2, stn_last_error()};
            STN_HIP(hipEventRecord(j.ev[c], s));
            j.ev_live[c] = true;
            j.next = (c + 1) % kChunksInFlight;
            j.k_issued += ks[i];
            j.chunks++;
        }
        std::lock_guard<std::mutex> lk(sv->m);
        sv->st.chunks += g.size();
        sv->st.gang_launches++;
        sv->st.gang_chunks += g.size();
        return true;
    }

    // true when j made progress (chunk issued, finishing enqueued, or done)
    bool step(Job& j, bool& done) {
        done = false;
        if (j.k_issued < j.K) return issue(j);
        if (!j.finishing) {
            // all chunks enqueued: statistics in trajectory order, copied to the pinned slot
            hipStream_t s = streams[j.stream];
            accum_finish_energy(j.acc, s);
            STN_HIP(hipMemcpyAsync(pinned + 2 * j.slot, j.acc->d_stats.p, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
            STN_HIP(hipEventRecord(j.done_ev, s));
            j.finishing = true;
            return true;
        }
        const hipError_t q = hipEventQuery(j.done_ev);
        if (q == hipErrorNotReady) return false;
        if (q != hipSuccess) throw Error{STN_E_DEVICE, std::string("job stream: ") + hipGetErrorString(q)};
        const stn_job_result r = record(j, STN_OK, "");
        release(j);
        publish(r);
        done = true;
        return true;
    }

    void loop() {
        for (;;) {
            bool progress = false;
            while (admit()) progress = true;
            try {
                progress |= gang();
            } catch (const Error& e) {
                // a failed multi-batch launch fails every whole-state-in-LDS job on the shared stream
                for (size_t i = 0; i < active.size();) {
                    Job& j = *active[i];
                    if (j.stream == 0 && j.plan && j.plan->kind == STN_PLAN_SV_LDS) {
                        fail_job(j, e);
                        active.erase(active.begin() + i);
                        continue;
                    }
                    ++i;
                }
                progress = true;
            }
            // round-robin over the admitted jobs, one chunk each per round
            for (size_t i = 0; i < active.size();) {
                auto j = active[(rr + i) % active.size()];
                bool done = false;
                try {
                    progress |= step(*j, done);
                } catch (const Error& e) {
                    fail_job(*j, e);
                    done = true;
                    progress = true;
                }
                if (done) {
                    active.erase(std::find(active.begin(), active.end(), j));
                    continue;
                }
                ++i;
            }
            rr = active.empty() ? 0 : (rr + 1) % active.size();
            {
                std::unique_lock<std::mutex> lk(sv->m);
                sv->inflight_jobs = active.size();
                if (sv->stop && (!sv->opts.drain_on_destroy || (active.empty() && sv->completed == sv->submitted)))
                    return;
                if (!progress) {
                    if (active.empty()) sv->cv_ready.wait_for(lk, std::chrono::milliseconds(5));
                    else sv->cv_ready.wait_for(lk, std::chrono::microseconds(50));
                }
            }
        }
    }
};

void worker_main(stn_server* sv) {
    Device d;
    d.sv = sv;
    try {
        d.init();
        {
            std::lock_guard<std::mutex> lk(sv->m);
            sv->started = true;
        }
        sv->cv_done.notify_all();
        d.loop();
    } catch (const Error& e) {
        std::lock_guard<std::mutex> lk(sv->m);
        sv->fatal = e.msg;
        sv->started = true;
    }
    sv->cv_done.notify_all();
    d.shutdown();
}

thread_local std::string g_srv_err;
stn_status srv_error(stn_status s, const std::string& m) {
    g_srv_err = m;
    return s;
}

}  // namespace
}  // namespace stn

using namespace stn;

extern "C" {

void stn_server_opts_default(stn_server_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->hbm_budget = 64ull << 30;
    o->job_share = 0.5;
    o->n_streams = 3;
    o->max_active = 16;
    o->plan_cache = 64;
    o->precision = 64;
    o->drain_on_destroy = 1;
    o->reserve_cus = 32;
    o->graphs = 0;
    o->gang = 1;
}

stn_status stn_server_create(const stn_server_opts* opts, stn_server** out) {
    if (!out) return STN_E_INVALID;
    *out = nullptr;
    stn_server_opts o;
    if (opts) o = *opts;
    else stn_server_opts_default(&o);
    if (o.n_streams < 1 || o.n_streams > kMaxStreams || o.max_active < 1 || o.max_active > kMaxActive ||
        !(o.job_share > 0 && o.job_share <= 1) || o.hbm_budget < (64ull << 20) ||
        (o.precision != 64 && o.precision != 128) || o.graphs > 1 || o.gang > 1)
        return srv_error(STN_E_INVALID, "server options out of range");
    auto* sv = new stn_server();
    sv->opts = o;
    sv->t0 = std::chrono::steady_clock::now();
    sv->pool = std::make_unique<DevicePool>(o.hbm_budget);
    if (hipGetDevice(&sv->device) != hipSuccess) {
        (void)hipGetLastError();
        delete sv;
        return srv_error(STN_E_DEVICE, "no HIP device");
    }
    for (int i = 0; i < kPlanners; ++i) sv->planners.emplace_back(planner_loop, sv);
    sv->worker = std::thread(worker_main, sv);
    // the server's clock and memory are ready when create returns
    std::string fatal;
    {
        std::unique_lock<std::mutex> lk(sv->m);
        sv->cv_done.wait(lk, [&] { return sv->started; });
        fatal = sv->fatal;
        sv->t0 = std::chrono::steady_clock::now();
    }
    if (!fatal.empty()) {
        stn_server_destroy(sv);
        return srv_error(STN_E_OOM, fatal);
    }
    *out = sv;
    return STN_OK;
}

stn_status stn_server_submit(stn_server* sv, const stn_circuit* circuit, const stn_noise_model* noise,
                             const stn_observable* observable, uint64_t seed, uint64_t K, uint64_t tag,
                             uint64_t* job_id) {
    if (!sv || !circuit || !observable) return srv_error(STN_E_INVALID, "NULL argument");
    if (K == 0) return srv_error(STN_E_INVALID, "K must be positive");
    auto j = std::make_shared<Job>();
    try {
        j->in.copy(circuit, noise, observable, sv->opts.precision);
    } catch (const Error& e) {
        return srv_error(e.status, e.msg);
    } catch (const std::bad_alloc&) {
        return srv_error(STN_E_OOM, "host allocation failed");
    }
    j->seed = seed;
    j->K = K;
    j->tag = tag;
    {
        std::lock_guard<std::mutex> lk(sv->m);
        if (!sv->fatal.empty()) return srv_error(STN_E_DEVICE, "server stopped: " + sv->fatal);
        j->t_submit = sv->now();
        j->id = sv->next_id++;
        sv->submitted++;
        sv->to_plan.push_back(j);
    }
    sv->cv_plan.notify_one();
    if (job_id) *job_id = j->id;
    return STN_OK;
}

stn_status stn_server_poll(stn_server* sv, stn_job_result* out, uint32_t cap, uint32_t* n_out, double wait_s) {
    if (!sv || !n_out || (cap && !out)) return srv_error(STN_E_INVALID, "NULL argument");
    *n_out = 0;
    std::unique_lock<std::mutex> lk(sv->m);
    if (sv->results.empty() && wait_s > 0)
        sv->cv_done.wait_for(lk, std::chrono::duration<double>(wait_s), [&] { return !sv->results.empty() || !sv->fatal.empty(); });
    uint32_t n = 0;
    while (n < cap && !sv->results.empty()) {
        out[n++] = sv->results.front();
        sv->results.pop_front();
    }
    *n_out = n;
    if (!sv->fatal.empty() && n == 0) return srv_error(STN_E_DEVICE, "server stopped: " + sv->fatal);
    return STN_OK;
}

stn_status stn_server_drain(stn_server* sv, double timeout_s) {
    if (!sv) return srv_error(STN_E_INVALID, "NULL argument");
    std::unique_lock<std::mutex> lk(sv->m);
    const bool ok = sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                         [&] { return sv->completed == sv->submitted || !sv->fatal.empty(); });
    if (!sv->fatal.empty()) return srv_error(STN_E_DEVICE, "server stopped: " + sv->fatal);
    return ok ? STN_OK : srv_error(STN_E_STATE, "drain timed out");
}

stn_status stn_server_stats_read(stn_server* sv, stn_server_stats* out) {
    if (!sv || !out) return srv_error(STN_E_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->m);
    *out = sv->st;
    out->submitted = sv->submitted;
    out->completed = sv->completed;
    out->active = sv->inflight_jobs;
    out->waiting = sv->to_plan.size() + sv->ready.size();
    out->bytes_in_use = sv->pool->in_use();
    out->bytes_cached = sv->pool->cached();
    out->bytes_peak = sv->pool->peak();
    out->plans_cached = sv->cache.size();
    out->clock = sv->now();
    return STN_OK;
}

double stn_server_clock(const stn_server* sv) { return sv ? sv->now() : 0.0; }

const char* stn_server_last_error(void) { return g_srv_err.c_str(); }

void stn_server_destroy(stn_server* sv) {
    if (!sv) return;
    if (sv->opts.drain_on_destroy) (void)stn_server_drain(sv, 1e9);
    {
        std::lock_guard<std::mutex> lk(sv->m);
        sv->stop = true;
    }
    sv->cv_plan.notify_all();
    sv->cv_ready.notify_all();
    for (auto& t : sv->planners)
        if (t.joinable()) t.join();
    if (sv->worker.joinable()) sv->worker.join();
    // jobs planned but never admitted
    for (auto& j : sv->ready) delete j->plan;
    for (auto& e : sv->cache) delete e.second;
    sv->cache.clear();
    delete sv;
}

}  // extern "C"
