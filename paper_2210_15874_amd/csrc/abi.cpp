// extern "C" entry points of include/stn.h: argument checks, handle
// lifetimes, device memory, and dispatch to the kernel launchers.
#include <algorithm>
#include <unordered_map>
#include <cstring>
#include <new>

#include <mutex>

#include "stn_internal.h"

namespace stn {

namespace {
thread_local std::string g_last_error;

stn_status set_error(stn_status s, const std::string& m) {
    g_last_error = m;
    return s;
}
}  // namespace

void fail(stn_status s, const std::string& msg) { throw Error{s, msg}; }

void hip_check(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        if (e == hipErrorOutOfMemory) fail(STN_E_OOM, std::string(what) + ": out of device memory");
        fail(STN_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
    }
}

void* Allocator::alloc(size_t bytes) const {
    void* p = nullptr;
    ++gen;
    if (fn) {
        p = fn(bytes, ctx);
        if (!p) fail(STN_E_OOM, "device allocator returned NULL for " + std::to_string(bytes) + " bytes");
        return p;
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(e == hipErrorOutOfMemory ? STN_E_OOM : STN_E_DEVICE,
             "hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
    }
    return p;
}

void Allocator::release(void* p) const {
    if (!p) return;
    if (ffn) ffn(p, ctx);
    else (void)hipFree(p);
}

namespace {
// released pinned buffers (pointer, bytes); never destroyed, so that no
// hipHostFree runs after the runtime has shut down at process exit
struct PinnedPool {
    std::mutex m;
    std::vector<std::pair<void*, size_t>> bufs;
    size_t total = 0;
};
PinnedPool& pinned_pool() {
    static PinnedPool* pool = new PinnedPool();
    return *pool;
}
constexpr size_t kPinnedPoolBytes = size_t(2) << 30;
}  // namespace

void HostBuf::reset() {
    if (!p) return;
    PinnedPool& pool = pinned_pool();
    {
        std::lock_guard<std::mutex> lk(pool.m);
        if (pool.total + bytes <= kPinnedPoolBytes) {
            pool.bufs.emplace_back(p, bytes);
            pool.total += bytes;
            p = nullptr;
            bytes = 0;
            return;
        }
    }
    (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
}

void HostBuf::ensure(size_t nbytes) {
    if (p && bytes >= nbytes) return;
    reset();
    const size_t want = nbytes ? nbytes : 1;
    {
        // the smallest pooled buffer that is large enough
        PinnedPool& pool = pinned_pool();
        std::lock_guard<std::mutex> lk(pool.m);
        size_t best = pool.bufs.size();
        for (size_t i = 0; i < pool.bufs.size(); ++i)
            if (pool.bufs[i].second >= want && (best == pool.bufs.size() || pool.bufs[i].second < pool.bufs[best].second))
                best = i;
        if (best < pool.bufs.size()) {
            p = pool.bufs[best].first;
            bytes = pool.bufs[best].second;
            pool.total -= bytes;
            pool.bufs.erase(pool.bufs.begin() + (ptrdiff_t)best);
            return;
        }
    }
    void* q = nullptr;
    if (hipHostMalloc(&q, want) != hipSuccess || !q) {
        (void)hipGetLastError();
        fail(STN_E_OOM, "pinned host allocation of " + std::to_string(nbytes) + " bytes failed");
    }
    p = q;
    bytes = want;
}

void upload(DevBuf& d, const Allocator* a, const void* host, size_t bytes, hipStream_t s) {
    d.ensure(a, bytes);
    if (bytes) STN_HIP(hipMemcpyAsync(d.p, host, bytes, hipMemcpyHostToDevice, s));
}

template <class F>
stn_status guarded(F&& f) {
    try {
        f();
        return STN_OK;
    } catch (const Error& e) {
        return set_error(e.status, e.msg);
    } catch (const std::bad_alloc&) {
        return set_error(STN_E_OOM, "host allocation failed");
    } catch (const std::exception& e) {
        return set_error(STN_E_INVALID, e.what());
    }
}

void upload_plan_tables(stn_plan* p, hipStream_t s);

// Device tables are uploaded on the first call that needs the device, so a
// plan can be built and inspected on a host without a GPU.
void ensure_uploaded(stn_plan* p, hipStream_t s) {
    if (p->uploaded) return;
    upload_plan_tables(p, s);
    STN_HIP(hipStreamSynchronize(s));
    p->uploaded = true;
}

}  // namespace stn

using namespace stn;

namespace stn {

static hipEvent_t take_event(stn_plan* p) {
    if (!p->ev_pool.empty()) {
        hipEvent_t e = p->ev_pool.back();
        p->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    STN_HIP(hipEventCreate(&e));
    return e;
}

void prof_begin(stn_plan* p, int cls, hipStream_t s) {
    if (!p->prof) return;
    hipEvent_t a = take_event(p), b = take_event(p);
    STN_HIP(hipEventRecord(a, s));
    p->prof_cls[cls].ev.push_back({a, b});
}

void prof_end(stn_plan* p, int cls, hipStream_t s, double bytes, double flops) {
    if (!p->prof) return;
    STN_HIP(hipEventRecord(p->prof_cls[cls].ev.back().second, s));
    p->prof_cls[cls].bytes.push_back(bytes);
    p->prof_cls[cls].flops.push_back(flops);
}

void prof_clear(stn_plan* p) {
    for (auto& c : p->prof_cls) {
        for (auto& e : c.ev) {
            p->ev_pool.push_back(e.first);
            p->ev_pool.push_back(e.second);
        }
        c.ev.clear();
        c.bytes.clear();
        c.flops.clear();
    }
}

}  // namespace stn

stn_plan::~stn_plan() {
    // device buffers may still be read by enqueued kernels unless the owner
    // has already waited for them (the job server does)
    if (sync_on_destroy) (void)hipDeviceSynchronize();
    if (lc && lc_free) lc_free(lc);
    if (tiled && tiled_free) tiled_free(tiled);
    stn::prof_clear(this);
    for (auto e : ev_pool) (void)hipEventDestroy(e);
}

namespace stn {

// Stream-ordered end of a job's energy reduction: the per-trajectory
// energies gathered in trajectory order, then the fixed-order mean and
// standard error into d_stats[0..1].  Enqueues only.
void accum_finish_energy(stn_accum* a, hipStream_t s) {
    stn_plan* p = a->plan;
    a->d_stats.ensure(&p->alloc, 4 * 8);
    STN_HIP(hipMemsetAsync(a->d_stats.p, 0, 4 * 8, s));
    if (!(p->opts.outputs & STN_OUT_ENERGY) || !a->k_done) return;
    a->d_egather.ensure(&p->alloc, a->k_done * 8);
    std::sort(a->ranges.begin(), a->ranges.end());
    uint64_t pos = 0;
    for (auto& r : a->ranges) {
        uint64_t k = r.first;
        while (k < r.second) {
            const uint64_t c = k / kEnergyChunk, stop = std::min<uint64_t>(r.second, (c + 1) * kEnergyChunk);
            STN_HIP(hipMemcpyAsync(a->d_egather.as<double>() + pos, a->e_chunks[c].as<double>() + (k % kEnergyChunk),
                                   (stop - k) * 8, hipMemcpyDeviceToDevice, s));
            pos += stop - k;
            k = stop;
        }
    }
    launch_energy_stats(a, a->k_done, s);
}

// (Re)shapes a batch for trajectories k0 .. k0+K-1 of plan p; buffers only grow.
void batch_prepare(stn_plan* p, stn_batch* b, uint64_t k0, uint32_t K) {
    const size_t S = p->sites.size();
    b->plan = p;
    b->k0 = k0;
    b->K = K;
    b->contracted = false;
    b->words = (uint32_t)((p->gates.size() + 31) / 32);
    b->d_idx.ensure(&p->alloc, (size_t)K * S);
    if (p->kind != STN_PLAN_SV_LDS && p->kind != STN_PLAN_SV_GATES) {
        b->d_signs.ensure(&p->alloc, (size_t)K * std::max<uint32_t>(b->words, 1) * 4);
        b->d_frame.ensure(&p->alloc, (size_t)K * 16);
    }
    b->d_energy.ensure(&p->alloc, (size_t)K * 8);
}

}  // namespace stn

extern "C" {

const char* stn_version(void) { return "stn 0.1 (gfx950)"; }

const char* stn_last_error(void) { return g_last_error.c_str(); }

void stn_plan_opts_default(stn_plan_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = 64;
    o->outputs = STN_OUT_ENERGY;
    o->plan_kind = STN_PLAN_AUTO;
}

stn_status stn_plan_create(const stn_circuit* circuit, const stn_noise_model* noise,
                           const stn_observable* observable, const stn_plan_opts* opts, stn_plan** out) {
    if (!out) return set_error(STN_E_INVALID, "out is NULL");
    *out = nullptr;
    stn_plan* p = nullptr;
    stn_status st = guarded([&] {
        p = new stn_plan();
        if (opts) p->opts = *opts;
        else stn_plan_opts_default(&p->opts);
        if (p->opts.precision != 64 && p->opts.precision != 128) fail(STN_E_INVALID, "precision must be 64 or 128");
        if (p->opts.sv_tile_bits && (p->opts.precision != 64 || (p->opts.sv_tile_bits != 14 && p->opts.sv_tile_bits != 15)))
            fail(STN_E_INVALID, "sv_tile_bits must be 0, 14 or 15 (complex64 plans only)");
        if ((p->opts.dev_alloc == nullptr) != (p->opts.dev_free == nullptr))
            fail(STN_E_INVALID, "dev_alloc and dev_free must be given together");
        if (p->opts.lc_order_fn && p->opts.lc_slice_bits)
            fail(STN_E_INVALID, "a caller-supplied contraction order excludes slicing (lc_slice_bits must be 0)");
        p->alloc.fn = p->opts.dev_alloc;
        p->alloc.ffn = p->opts.dev_free;
        p->alloc.ctx = p->opts.alloc_ctx;
        build_plan(p, circuit, noise, observable);
    });
    if (st != STN_OK) {
        delete p;
        return st;
    }
    *out = p;
    return STN_OK;
}

stn_status stn_plan_info(const stn_plan* p, stn_plan_stats* o) {
    if (!p || !o) return set_error(STN_E_INVALID, "NULL argument");
    std::memset(o, 0, sizeof(*o));
    o->plan_kind = p->kind;
    o->n_qubits = p->n;
    o->n_gates = (uint32_t)p->gates.size();
    o->n_sites = (uint32_t)p->sites.size();
    o->max_batch = p->max_batch;
    o->width = p->width;
    o->n_passes = p->n_passes;
    o->n_steps = p->n_steps;
    o->bytes_per_traj = p->bytes_per_traj;
    o->flops_per_traj = p->flops_per_traj;
    o->peak_bytes = p->peak_bytes;
    o->lc_width = p->lc_width;
    o->lc_flops_per_traj = p->lc_flops_per_traj;
    o->variant = p->variant;
    o->tuned = p->tuned ? 1 : 0;
    o->graphs = p->graphs ? 1 : 0;
    o->graph_captures = p->graph_captures;
    o->graph_replays = p->graph_replays;
    o->lc_slices = p->lc_slices;
    o->lc_slice_bits = p->lc_slice_bits;
    o->est_s_per_traj = p->est_seconds_per_traj();
    o->lc_group = p->lc_group;
    o->lc_width_lower_bound = p->lc_width_lb;
    o->half_state = p->sv_half ? 1u : 0u;
    o->tile_bits = p->kind == STN_PLAN_SV_TILED ? p->tile_bits : 0u;
    return STN_OK;
}

namespace {
void plan_ref(stn_plan* p) { p->refs.fetch_add(1, std::memory_order_relaxed); }
void plan_unref(stn_plan* p) {
    if (p && p->refs.fetch_sub(1, std::memory_order_acq_rel) == 1) delete p;
}
}  // namespace

void stn_plan_destroy(stn_plan* p) { plan_unref(p); }

stn_status stn_profile(stn_plan* p, int enable) {
    if (!p) return set_error(STN_E_INVALID, "NULL argument");
    return guarded([&] {
        STN_HIP(hipDeviceSynchronize());
        prof_clear(p);
        p->prof = enable != 0;
    });
}

stn_status stn_profile_read(stn_plan* p, stn_kernel_stats* out) {
    if (!p || !out) return set_error(STN_E_INVALID, "NULL argument");
    return guarded([&] {
        STN_HIP(hipDeviceSynchronize());
        for (int c = 0; c < STN_K_COUNT; ++c) {
            stn_kernel_stats& o = out[c];
            o = stn_kernel_stats{};
            const ProfClass& pc = p->prof_cls[c];
            for (size_t i = 0; i < pc.ev.size(); ++i) {
                float ms = 0;
                STN_HIP(hipEventElapsedTime(&ms, pc.ev[i].first, pc.ev[i].second));
                o.ms += ms;
                o.bytes += pc.bytes[i];
                o.flops += pc.flops[i];
                ++o.launches;
            }
        }
    });
}

stn_status stn_plan_site(const stn_plan* p, uint32_t site, uint32_t* n_ops, uint64_t* thresholds, uint32_t cap) {
    if (!p || !n_ops) return set_error(STN_E_INVALID, "NULL argument");
    if (site >= p->sites.size()) return set_error(STN_E_INVALID, "site out of range");
    const SiteRec& r = p->sites[site];
    *n_ops = r.J;
    if (thresholds)
        for (uint32_t j = 0; j < r.J && j < cap; ++j) thresholds[j] = r.T[j];
    return STN_OK;
}

stn_status stn_sample(stn_plan* p, uint64_t seed, uint64_t k0, uint32_t K, stn_batch** out, void* stream) {
    if (!p || !out) return set_error(STN_E_INVALID, "NULL argument");
    *out = nullptr;
    if (K == 0) return set_error(STN_E_INVALID, "K must be positive");
    stn_batch* b = nullptr;
    stn_status st = guarded([&] {
        b = new stn_batch();
        batch_prepare(p, b, k0, K);
        hipStream_t s = (hipStream_t)stream;
        ensure_uploaded(p, s);
        launch_sample(p, b, seed, s);
        if (p->kind != STN_PLAN_SV_LDS && p->kind != STN_PLAN_SV_GATES) launch_frame(p, b, s);
    });
    if (st != STN_OK) {
        delete b;
        return st;
    }
    plan_ref(p);
    *out = b;
    return STN_OK;
}

stn_status stn_resample(stn_batch* b, uint64_t seed, uint64_t k0, uint32_t K, void* stream) {
    if (!b || !b->plan) return set_error(STN_E_INVALID, "NULL argument");
    if (K == 0) return set_error(STN_E_INVALID, "K must be positive");
    stn_plan* p = b->plan;
    return guarded([&] {
        batch_prepare(p, b, k0, K);
        b->has_states = false;
        hipStream_t s = (hipStream_t)stream;
        ensure_uploaded(p, s);
        launch_sample(p, b, seed, s);
        if (p->kind != STN_PLAN_SV_LDS && p->kind != STN_PLAN_SV_GATES) launch_frame(p, b, s);
    });
}

stn_status stn_batch_from_indices(stn_plan* p, const uint8_t* idx, uint64_t k0, uint32_t K, stn_batch** out,
                                  void* stream) {
    if (!p || !out || (!idx && K && !p->sites.empty())) return set_error(STN_E_INVALID, "NULL argument");
    *out = nullptr;
    if (K == 0) return set_error(STN_E_INVALID, "K must be positive");
    stn_batch* b = nullptr;
    stn_status st = guarded([&] {
        const size_t S = p->sites.size();
        for (size_t k = 0; k < K; ++k)
            for (size_t s = 0; s < S; ++s)
                if (idx[k * S + s] >= p->sites[s].J)
                    fail(STN_E_INVALID, "index out of range at trajectory " + std::to_string(k) + ", site " +
                                            std::to_string(s));
        hipStream_t s = (hipStream_t)stream;
        ensure_uploaded(p, s);
        b = new stn_batch();
        batch_prepare(p, b, k0, K);
        if (S) STN_HIP(hipMemcpyAsync(b->d_idx.p, idx, (size_t)K * S, hipMemcpyHostToDevice, s));
        if (p->kind != STN_PLAN_SV_LDS && p->kind != STN_PLAN_SV_GATES) launch_frame(p, b, s);
        STN_HIP(hipStreamSynchronize(s));
    });
    if (st != STN_OK) {
        delete b;
        return st;
    }
    plan_ref(p);
    *out = b;
    return STN_OK;
}

stn_status stn_batch_indices(const stn_batch* b, uint8_t* host_out) {
    if (!b || !host_out) return set_error(STN_E_INVALID, "NULL argument");
    return guarded([&] {
        const size_t bytes = (size_t)b->K * b->plan->sites.size();
        STN_HIP(hipDeviceSynchronize());
        if (bytes) STN_HIP(hipMemcpy(host_out, b->d_idx.p, bytes, hipMemcpyDeviceToHost));
    });
}

static uint32_t plan_variants(const stn_plan* p) {
    switch (p->kind) {
        case STN_PLAN_SV_LDS: return lds_variants();
        case STN_PLAN_SV_TILED: return tiled_variants(p);
        case STN_PLAN_LIGHTCONE: return tn_variants();
        default: return 1;
    }
}

static void contract_launch(stn_plan* p, stn_batch* b, hipStream_t s) {
    switch (p->kind) {
        case STN_PLAN_SV_LDS: launch_sv_lds(p, b, s); break;
        case STN_PLAN_SV_TILED:
            if (p->opts.precision == 128) launch_sv_tiled128(p, b, s);
            else launch_sv_tiled(p, b, s);
            break;
        case STN_PLAN_LIGHTCONE: launch_lightcone(p, b, s); break;
        case STN_PLAN_SV_GATES: launch_sv_gates(p, b, s); break;
        default: fail(STN_E_STATE, "plan has no lowering");
    }
}

// Contraction through a HIP graph per (batch, K, launch shape, CU cap,
// workspace): eager the first time, captured the second, replayed after.
static void contract_graph(stn_plan* p, stn_batch* b, hipStream_t s) {
    const uint64_t key[4] = {b->K, p->variant, p->grid_cap, p->alloc.gen};
    const bool same = std::equal(key, key + 4, b->gkey);
    if (b->gstate == 2 && same) {
        STN_HIP(hipGraphLaunch(b->gexec, s));
        p->graph_replays++;
        return;
    }
    if (b->gstate == 1 && same) {
        hipGraph_t g = nullptr;
        STN_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
            contract_launch(p, b, s);
        } catch (...) {
            (void)hipStreamEndCapture(s, &g);
            if (g) (void)hipGraphDestroy(g);
            b->gstate = 0;
            throw;
        }
        STN_HIP(hipStreamEndCapture(s, &g));
        if (p->alloc.gen != key[3]) {   // the eager run allocated everything; nothing may move now
            (void)hipGraphDestroy(g);
            b->gstate = 0;
            fail(STN_E_STATE, "device memory allocated during graph capture");
        }
        if (b->gexec) {
            (void)hipGraphExecDestroy(b->gexec);
            b->gexec = nullptr;
        }
        const hipError_t e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            b->gexec = nullptr;
            b->gstate = 0;
            STN_HIP(e);
        }
        b->gstate = 2;
        p->graph_captures++;
        STN_HIP(hipGraphLaunch(b->gexec, s));
        return;
    }
    contract_launch(p, b, s);
    b->gkey[0] = b->K;
    b->gkey[1] = p->variant;
    b->gkey[2] = p->grid_cap;
    b->gkey[3] = p->alloc.gen;
    b->gstate = 1;
}

stn_status stn_contract(stn_plan* p, stn_batch* b, void* stream) {
    if (!p || !b) return set_error(STN_E_INVALID, "NULL argument");
    if (b->plan != p) return set_error(STN_E_INVALID, "batch belongs to another plan");
    return guarded([&] {
        hipStream_t s = (hipStream_t)stream;
        ensure_uploaded(p, s);
        bool use_graph = p->graphs && !p->prof && s != nullptr;
        if (use_graph) {
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            STN_HIP(hipStreamIsCapturing(s, &cs));
            use_graph = cs == hipStreamCaptureStatusNone;
        }
        if (use_graph) contract_graph(p, b, s);
        else contract_launch(p, b, s);
        b->contracted = true;
    });
}

stn_status stn_contract_many(stn_plan* const* plans, stn_batch* const* batches, uint32_t count, void* stream) {
    if (count == 0) return STN_OK;
    if (!plans || !batches) return set_error(STN_E_INVALID, "NULL argument");
    for (uint32_t i = 0; i < count; ++i) {
        if (!plans[i] || !batches[i]) return set_error(STN_E_INVALID, "NULL plan or batch");
        if (batches[i]->plan != plans[i]) return set_error(STN_E_INVALID, "batch belongs to another plan");
        if (plans[i]->kind != STN_PLAN_SV_LDS)
            return set_error(STN_E_UNSUPPORTED, "multi-batch launches take whole-state-in-LDS plans only");
        if (plans[i]->opts.precision != plans[0]->opts.precision)
            return set_error(STN_E_INVALID, "all plans of a multi-batch launch need the same precision");
        for (uint32_t j = 0; j < i; ++j)
            if (batches[j] == batches[i]) return set_error(STN_E_INVALID, "a batch appears twice");
    }
    return guarded([&] {
        hipStream_t s = (hipStream_t)stream;
        for (uint32_t i = 0; i < count; ++i) ensure_uploaded(plans[i], s);
        launch_sv_lds_many(plans, batches, count, s);
        for (uint32_t i = 0; i < count; ++i) batches[i]->contracted = true;
    });
}

stn_status stn_contract_dedup(stn_plan* p, stn_batch* b, uint32_t* n_unique, void* stream) {
    if (!p || !b) return set_error(STN_E_INVALID, "NULL argument");
    if (b->plan != p) return set_error(STN_E_INVALID, "batch belongs to another plan");
    if (p->opts.outputs & (STN_OUT_RHO | STN_OUT_DIAG | STN_OUT_STATES))
        return set_error(STN_E_UNSUPPORTED, "de-duplicated contraction produces energies only");
    return guarded([&] {
        hipStream_t s = (hipStream_t)stream;
        ensure_uploaded(p, s);
        const uint32_t K = b->K;
        const bool by_index = p->kind == STN_PLAN_SV_LDS || p->kind == STN_PLAN_SV_GATES;   // else: gate signs and final frame X
        const size_t S = p->sites.size(), W = b->words;
        // the trajectories' keys, read back once the sampling has finished
        std::vector<uint8_t> idx;
        std::vector<uint32_t> sg;
        std::vector<uint64_t> fr;
        STN_HIP(hipStreamSynchronize(s));
        if (by_index) {
            idx.resize((size_t)K * S);
            if (!idx.empty()) STN_HIP(hipMemcpy(idx.data(), b->d_idx.p, idx.size(), hipMemcpyDeviceToHost));
        } else {
            sg.resize((size_t)K * W);
            fr.resize((size_t)K * 2);
            if (!sg.empty()) STN_HIP(hipMemcpy(sg.data(), b->d_signs.p, sg.size() * 4, hipMemcpyDeviceToHost));
            STN_HIP(hipMemcpy(fr.data(), b->d_frame.p, fr.size() * 8, hipMemcpyDeviceToHost));
        }
        auto key = [&](uint32_t k) {
            if (by_index) return std::string(reinterpret_cast<const char*>(idx.data() + (size_t)k * S), S);
            std::string kk(reinterpret_cast<const char*>(sg.data() + (size_t)k * W), W * 4);
            kk.append(reinterpret_cast<const char*>(&fr[2 * (size_t)k]), 8);   // the frame's X part signs the energy
            return kk;
        };
        std::unordered_map<std::string, uint32_t> first;
        std::vector<uint32_t> rep, map(K);
        for (uint32_t k = 0; k < K; ++k) {
            auto it = first.emplace(key(k), (uint32_t)rep.size());
            if (it.second) rep.push_back(k);
            map[k] = it.first->second;
        }
        if (n_unique) *n_unique = (uint32_t)rep.size();
        if (rep.size() == K) {   // nothing to share
            contract_launch(p, b, s);
            b->contracted = true;
            return;
        }
        // one representative per distinct key, in trajectory order
        const uint32_t U = (uint32_t)rep.size();
        if (!b->unique) b->unique = new stn_batch();
        stn_batch* u = b->unique;
        batch_prepare(p, u, b->k0, U);
        // host sources of the copies below: they live until the synchronisation after them
        std::vector<uint8_t> ui;
        std::vector<uint32_t> us;
        std::vector<uint64_t> uf;
        if (by_index) {
            ui.resize((size_t)U * S);
            for (uint32_t r = 0; r < U; ++r)
                std::copy_n(idx.data() + (size_t)rep[r] * S, S, ui.data() + (size_t)r * S);
            if (!ui.empty()) STN_HIP(hipMemcpyAsync(u->d_idx.p, ui.data(), ui.size(), hipMemcpyHostToDevice, s));
        } else {
            us.resize((size_t)U * W);
            uf.resize((size_t)U * 2);
            for (uint32_t r = 0; r < U; ++r) {
                std::copy_n(sg.data() + (size_t)rep[r] * W, W, us.data() + (size_t)r * W);
                uf[2 * r] = fr[2 * (size_t)rep[r]];
                uf[2 * r + 1] = fr[2 * (size_t)rep[r] + 1];
            }
            if (!us.empty()) STN_HIP(hipMemcpyAsync(u->d_signs.p, us.data(), us.size() * 4, hipMemcpyHostToDevice, s));
            STN_HIP(hipMemcpyAsync(u->d_frame.p, uf.data(), uf.size() * 8, hipMemcpyHostToDevice, s));
        }
        b->d_map.ensure(&p->alloc, (size_t)K * 4);
        STN_HIP(hipMemcpyAsync(b->d_map.p, map.data(), (size_t)K * 4, hipMemcpyHostToDevice, s));
        STN_HIP(hipStreamSynchronize(s));   // the host copies above are pageable
        contract_launch(p, u, s);
        launch_scatter_energy(u->d_energy.as<double>(), b->d_map.as<uint32_t>(), K, b->d_energy.as<double>(), s);
        b->contracted = true;
    });
}

stn_status stn_plan_set_graphs(stn_plan* p, uint32_t on) {
    if (!p) return set_error(STN_E_INVALID, "NULL argument");
    p->graphs = on != 0;
    return STN_OK;
}

stn_status stn_plan_autotune(stn_plan* p, stn_batch* b, uint32_t reps, stn_tune_result* out, void* stream) {
    if (!p || !b) return set_error(STN_E_INVALID, "NULL argument");
    if (b->plan != p) return set_error(STN_E_INVALID, "batch belongs to another plan");
    if (reps == 0) reps = 1;
    return guarded([&] {
        hipStream_t s = (hipStream_t)stream;
        ensure_uploaded(p, s);
        const uint32_t nv = std::min<uint32_t>(plan_variants(p), 8);
        hipEvent_t e0, e1;
        STN_HIP(hipEventCreate(&e0));
        STN_HIP(hipEventCreate(&e1));
        double ms[8] = {0};
        uint32_t best = 0;
        try {
            for (uint32_t v = 0; v < nv; ++v) {
                p->variant = v;
                contract_launch(p, b, s);   // warm (code object, attributes)
                STN_HIP(hipEventRecord(e0, s));
                for (uint32_t r = 0; r < reps; ++r) contract_launch(p, b, s);
                STN_HIP(hipEventRecord(e1, s));
                STN_HIP(hipEventSynchronize(e1));
                float t = 0;
                STN_HIP(hipEventElapsedTime(&t, e0, e1));
                ms[v] = t / reps;
                if (ms[v] < ms[best]) best = v;
            }
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            p->variant = 0;
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        p->variant = best;
        p->tuned = true;
        b->contracted = true;
        if (out) {
            std::memset(out, 0, sizeof(*out));
            out->n_variants = nv;
            out->chosen = best;
            for (uint32_t v = 0; v < nv; ++v) out->ms[v] = ms[v];
        }
    });
}

stn_status stn_plan_set_variant(stn_plan* p, uint32_t variant) {
    if (!p) return set_error(STN_E_INVALID, "NULL argument");
    if (variant >= plan_variants(p)) return set_error(STN_E_INVALID, "launch-shape variant out of range");
    p->variant = variant;
    p->tuned = true;
    return STN_OK;
}

stn_status stn_batch_results(const stn_batch* b, double* energies, double* states) {
    if (!b) return set_error(STN_E_INVALID, "NULL argument");
    if (!b->contracted) return set_error(STN_E_STATE, "batch not contracted");
    if (states && !b->has_states) return set_error(STN_E_STATE, "batch keeps no states (request STN_OUT_STATES)");
    return guarded([&] {
        STN_HIP(hipDeviceSynchronize());
        if (energies) STN_HIP(hipMemcpy(energies, b->d_energy.p, (size_t)b->K * 8, hipMemcpyDeviceToHost));
        if (states) {
            const size_t N = (size_t)1 << b->plan->n;
            const size_t cnt = N * b->K;
            if (b->plan->opts.precision == 128) {
                STN_HIP(hipMemcpy(states, b->d_states.p, cnt * 16, hipMemcpyDeviceToHost));
            } else {
                std::vector<float> tmp(cnt * 2);
                STN_HIP(hipMemcpy(tmp.data(), b->d_states.p, cnt * 8, hipMemcpyDeviceToHost));
                for (size_t i = 0; i < cnt * 2; ++i) states[i] = tmp[i];
            }
        }
    });
}

uint32_t stn_batch_size(const stn_batch* b) { return b ? b->K : 0; }

void stn_batch_destroy(stn_batch* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    stn_plan* p = b->plan;
    delete b;
    plan_unref(p);
}

stn_status stn_accum_create(stn_plan* p, stn_accum** out) {
    if (!p || !out) return set_error(STN_E_INVALID, "NULL argument");
    *out = nullptr;
    stn_accum* a = nullptr;
    stn_status st = guarded([&] {
        a = new stn_accum();
        a->plan = p;
        const size_t N = (size_t)1 << p->n;
        if (p->opts.outputs & STN_OUT_RHO) {
            a->d_rho.ensure(&p->alloc, N * N * 16);
            STN_HIP(hipMemset(a->d_rho.p, 0, N * N * 16));
        }
        if (p->opts.outputs & (STN_OUT_DIAG | STN_OUT_RHO)) {
            a->d_diag.ensure(&p->alloc, N * 8);
            STN_HIP(hipMemset(a->d_diag.p, 0, N * 8));
        }
    });
    if (st != STN_OK) {
        delete a;
        return st;
    }
    plan_ref(p);
    *out = a;
    return STN_OK;
}

stn_status stn_reduce(stn_plan* p, stn_batch* b, stn_accum* a, void* stream) {
    if (!p || !b || !a) return set_error(STN_E_INVALID, "NULL argument");
    if (b->plan != p || a->plan != p) return set_error(STN_E_INVALID, "batch / accumulator belong to another plan");
    if (!b->contracted) return set_error(STN_E_STATE, "batch not contracted");
    const uint64_t lo = b->k0, hi = b->k0 + b->K;
    for (auto& r : a->ranges)
        if (lo < r.second && r.first < hi) return set_error(STN_E_INVALID, "trajectory range already reduced");
    stn_status st = guarded([&] {
        // make sure the energy chunks covering [lo, hi) exist
        if (p->opts.outputs & STN_OUT_ENERGY) {
            const uint64_t last = (hi - 1) / kEnergyChunk;
            if (last > (1ull << 24)) fail(STN_E_INVALID, "trajectory index too large");
            if (a->e_chunks.size() <= last) a->e_chunks.resize(last + 1);
            for (uint64_t c = lo / kEnergyChunk; c <= last; ++c) a->e_chunks[c].ensure(&p->alloc, kEnergyChunk * 8);
        }
        launch_reduce(p, b, a, (hipStream_t)stream);
    });
    if (st == STN_OK) {
        a->ranges.push_back({lo, hi});
        a->k_done += b->K;
    }
    return st;
}

stn_status stn_accum_read(stn_accum* a, stn_result* out, void* stream) {
    if (!a || !out) return set_error(STN_E_INVALID, "NULL argument");
    std::memset(out, 0, sizeof(*out));
    return guarded([&] {
        stn_plan* p = a->plan;
        hipStream_t s = (hipStream_t)stream;
        const size_t N = (size_t)1 << p->n;
        out->k_done = a->k_done;
        double st[4] = {0, 0, 0, 0};
        accum_finish_energy(a, s);
        if ((p->opts.outputs & STN_OUT_ENERGY) && a->k_done) {
            a->h_energies.ensure(a->k_done * 8);
            STN_HIP(hipMemcpyAsync(a->h_energies.p, a->d_egather.p, a->k_done * 8, hipMemcpyDeviceToHost, s));
            out->energies = a->h_energies.as<double>();
        }
        if (p->opts.outputs & (STN_OUT_DIAG | STN_OUT_RHO)) {
            if (p->opts.outputs & STN_OUT_RHO) a->d_rho_out.ensure(&p->alloc, N * N * 16);
            a->d_diag_out.ensure(&p->alloc, N * 8);
            launch_finish_dense(a, s);
            a->h_diag.ensure(N * 8);
            STN_HIP(hipMemcpyAsync(a->h_diag.p, a->d_diag_out.p, N * 8, hipMemcpyDeviceToHost, s));
            out->diag = a->h_diag.as<double>();
            if (p->opts.outputs & STN_OUT_RHO) {
                a->h_rho.ensure(N * N * 16);
                STN_HIP(hipMemcpyAsync(a->h_rho.p, a->d_rho_out.p, N * N * 16, hipMemcpyDeviceToHost, s));
                out->rho = a->h_rho.as<double>();
            }
        }
        STN_HIP(hipMemcpyAsync(st, a->d_stats.p, 4 * 8, hipMemcpyDeviceToHost, s));
        STN_HIP(hipStreamSynchronize(s));
        out->energy_mean = st[0];
        out->energy_se = st[1];
        out->trace_mean = st[2];
    });
}

void stn_accum_destroy(stn_accum* a) {
    if (!a) return;
    (void)hipDeviceSynchronize();
    stn_plan* p = a->plan;
    delete a;
    plan_unref(p);
}

stn_status stn_accum_sample(stn_accum* a, const double* u, uint32_t m, uint32_t* out, void* stream) {
    if (!a) return set_error(STN_E_INVALID, "NULL argument");
    if (m && (!u || !out)) return set_error(STN_E_INVALID, "NULL uniforms or output");
    stn_plan* p = a->plan;
    if (!(p->opts.outputs & (STN_OUT_DIAG | STN_OUT_RHO)))
        return set_error(STN_E_STATE, "accumulator keeps no diagonal (request STN_OUT_DIAG)");
    if (!a->k_done) return set_error(STN_E_STATE, "no trajectories reduced");
    if (!m) return STN_OK;
    return guarded([&] {
        a->d_cdf.ensure(&p->alloc, sample_bits_scratch(p->n));
        launch_sample_bits(a, u, m, out, a->d_cdf.as<double>(), (hipStream_t)stream);
    });
}

stn_status stn_accum_sample_noalloc(stn_accum* a, const double* u, uint32_t m, uint32_t* out, void* stream) {
    if (!a) return set_error(STN_E_INVALID, "NULL argument");
    if (m && (!u || !out)) return set_error(STN_E_INVALID, "NULL uniforms or output");
    stn_plan* p = a->plan;
    if (!(p->opts.outputs & (STN_OUT_DIAG | STN_OUT_RHO)))
        return set_error(STN_E_STATE, "accumulator keeps no diagonal (request STN_OUT_DIAG)");
    if (p->n > kStaticSampleQubits)
        return set_error(STN_E_UNSUPPORTED, "stn_accum_sample_noalloc holds running sums of at most 2^" +
                                                std::to_string(kStaticSampleQubits) + " states; this plan has n = " +
                                                std::to_string(p->n) + " (use stn_accum_sample)");
    if (!a->k_done) return set_error(STN_E_STATE, "no trajectories reduced");
    if (!m) return STN_OK;
    return guarded([&] {
        hipError_t e = hipSuccess;
        double* scratch = static_sample_scratch(&e);
        if (!scratch) fail(STN_E_DEVICE, std::string("address of the sampler's static buffer: ") + hipGetErrorString(e));
        launch_sample_bits(a, u, m, out, scratch, (hipStream_t)stream);
    });
}

}  // extern "C"
