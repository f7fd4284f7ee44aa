// Internal declarations shared by the host planner, the ABI layer and the
// kernel launchers of the trajectory-ensemble library.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/stn.h"

namespace stn {

using cd = std::complex<double>;

// ---------------------------------------------------------------- errors
struct Error {
    stn_status status;
    std::string msg;
};
[[noreturn]] void fail(stn_status s, const std::string& msg);
void hip_check(hipError_t e, const char* what);
#define STN_HIP(x) ::stn::hip_check((x), #x)

// ---------------------------------------------------------------- device memory
struct Allocator {
    stn_alloc_fn fn = nullptr;
    stn_free_fn ffn = nullptr;
    void* ctx = nullptr;
    mutable uint64_t gen = 0;    // allocations made so far (a captured graph is valid while unchanged)
    void* alloc(size_t bytes) const;
    void release(void* p) const;
};

// Owning device buffer; memory comes from the plan's allocator.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    const Allocator* a = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) { reset(); p = o.p; bytes = o.bytes; a = o.a; o.p = nullptr; o.bytes = 0; }
        return *this;
    }
    ~DevBuf() { reset(); }
    void reset() { if (p && a) a->release(p); p = nullptr; bytes = 0; }
    void ensure(const Allocator* al, size_t nbytes) {
        if (p && bytes >= nbytes) return;
        reset();
        a = al;
        bytes = nbytes ? nbytes : 1;
        p = al->alloc(bytes);
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// Pinned host memory, grown as needed: device-to-host copies into it run at
// the link's rate instead of through a pageable staging copy.  Pinning
// hundreds of MiB costs tens of milliseconds, so released buffers go to a
// process-wide pool (at most 2 GiB) from which the next ensure() takes one;
// a buffer belongs to one owner at a time.
struct HostBuf {
    void* p = nullptr;
    size_t bytes = 0;
    HostBuf() = default;
    HostBuf(const HostBuf&) = delete;
    HostBuf& operator=(const HostBuf&) = delete;
    ~HostBuf() { reset(); }
    void reset();                 // back to the pool (or freed when the pool is full)
    void ensure(size_t nbytes);   // throws STN_E_OOM when the allocation fails
    template <class T> T* as() const { return static_cast<T*>(p); }
};

void upload(DevBuf& d, const Allocator* a, const void* host, size_t bytes, hipStream_t s);

// ---------------------------------------------------------------- plan data
enum OpKind : uint32_t {
    OP_DENSE1 = 0,   // 2x2 dense on q0
    OP_DENSE2 = 1,   // 4x4 dense on (q0, q1)
    OP_DIAG1 = 2,    // diag(d0, d1) on q0
    OP_DIAG2 = 3,    // diag(d0..d3) on (q0, q1)
    OP_PAULI = 4,    // Pauli string: x mask / z mask (global phase dropped)
    OP_SITE = 5,     // noise site: operator picked by the trajectory's index
    OP_IDENT = 6
};

// One instruction of the whole-state-in-LDS interpreter.  mat indexes the
// complex value table (2, 4 or 16 entries).
struct LdsOp {
    uint32_t kind;
    uint32_t q0, q1;
    uint32_t mat;       // offset into value table (dense / diag)
    uint64_t xmask, zmask;
    uint32_t site;      // OP_SITE: site index; operator table at site_op[site_op_off[site] + j]
    uint32_t pad;
};

// Gate-by-gate lowering: consecutive operator-list entries whose qubits fit
// one tile of storage bits run as one pass over the tiles.
constexpr uint32_t kGroupMaxOps = 128;
struct GateGroup {
    uint32_t op0, n_ops;     // entries gate_group_ops[op0 .. op0 + n_ops)
    uint32_t nbits;          // tile bits
    uint8_t tb[16];          // storage bit of each tile-local bit, ascending
    uint8_t local[32];       // tile-local bit of each qubit, 0xFF outside the tile
};

struct SiteRec {
    uint32_t gate = 0, nq = 1, q0 = 0, q1 = 0, J = 0;
    std::vector<double> q;           // selection probabilities
    std::vector<uint64_t> T;         // thresholds, T[J-1] = 2^32
    std::vector<cd> ops;             // J * d*d inserted operators K_j/sqrt(q_j)
    bool pauli = false;              // every inserted operator is a Pauli string (up to phase)
    std::vector<uint64_t> px, pz;    // per operator: global x / z masks when pauli
};

struct GateRec {
    uint32_t kind = 0, nq = 1, q0 = 0, q1 = 0;
    double theta = 0;
    std::vector<cd> m;               // 2x2 or 4x4 matrix
    bool rotation = false;           // exp(-i theta/2 * P) with P a Pauli string
    uint64_t gx = 0, gz = 0;         // generator P's x / z masks (rotations)
    // Tiled lowering: rx(theta) = -i X rx(theta - pi); when |sin(theta/2)| >
    // |cos(theta/2)| the gate is applied as rx(theta_eff = theta - pi) and the
    // X (det_x mask) joins the trajectory's Pauli frame right after the gate.
    double theta_eff = 0;
    uint64_t det_x = 0;
};

// Tiled statevector lowering (QAOA structure: H prefix, then layers of
// diagonal zz blocks and rx mixer blocks, Pauli noise).
struct TiledLayer {
    std::vector<uint32_t> zz_gates;  // gate indices of the diagonal block
    std::vector<int32_t> zz_mult;    // angle = mult * base_angle
    double base_angle = 0;
    int32_t mult_sum = 0;            // sum |mult|: phase index range [-mult_sum, mult_sum]
    std::vector<int32_t> rx_gate;    // per qubit: rx gate index in the mixer block, -1 = none
};

// One pass over the state: load a tile, [diagonal of layer diag_a], rotate the
// tile's qubits of layer mix1, [diagonal of layer diag_b, rotate the tile's
// qubits of layer mix2], store (or reduce to the energy).  The two segments
// let the last tile of one layer and the first tile of the next share a pass.
struct TiledPass {
    uint32_t tile_mask = 0;          // storage bits inside the tile (= qubits, identity layout)
    int32_t diag_a = -1;             // layer whose diagonal is applied after the load (-1 none)
    int32_t mix1 = -1;               // layer rotated in the first segment
    uint32_t mix1_mask = 0;          // its qubits rotated here
    int32_t diag_b = -1;             // layer whose diagonal is applied between the segments
    int32_t mix2 = -1;               // layer rotated in the second segment (-1: no second segment)
    uint32_t mix2_mask = 0;
    bool init = false;               // generate |+>^n instead of loading
    bool last = false;               // accumulate the energy instead of storing
};

// Event-timed launches of one kernel class (profiling on).
struct ProfClass {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    std::vector<double> bytes, flops;
};

}  // namespace stn

struct stn_plan {
    // the caller's handle plus one per batch and accumulator made through the
    // C ABI (they free their buffers through alloc): the last release deletes
    std::atomic<uint32_t> refs{1};
    stn::Allocator alloc;
    stn_plan_opts opts{};
    uint32_t n = 0;
    uint32_t kind = STN_PLAN_SV_LDS;
    uint32_t max_batch = 0;
    std::vector<stn::GateRec> gates;
    std::vector<stn::SiteRec> sites;
    std::vector<uint32_t> obs_u, obs_v;
    std::vector<double> obs_w;
    bool frame_ok = false;           // Pauli-frame rewrite valid for this circuit
    bool uploaded = false;           // device tables present (uploaded on first device use)
    // cost model
    double bytes_per_traj = 0, flops_per_traj = 0, peak_bytes = 0;
    uint32_t width = 0, n_passes = 0, n_steps = 0;
    uint32_t lc_width = 0;                  // lightcone networks: width and flops, when they were built
    double lc_flops_per_traj = 0;
    double lc_est_s = 0;                    // their estimated seconds per trajectory
    double lc_arena_bytes = 0;              // HBM tier: global-memory arenas of the persistent workgroups
    // estimated device seconds per trajectory of the chosen lowering (admission and
    // scheduling in the job server; a cost-model figure, not a measurement)
    double est_seconds_per_traj() const {
        return kind == STN_PLAN_LIGHTCONE ? lc_est_s : bytes_per_traj / 3e12 + flops_per_traj / 5e13;
    }

    // device tables shared by every lowering
    stn::DevBuf d_site_T;            // uint64 thresholds, flattened
    stn::DevBuf d_site_off;          // uint32 offset of each site's thresholds, S+1 entries
    stn::DevBuf d_site_gate;         // uint32 gate index of each site
    stn::DevBuf d_site_px, d_site_pz;// uint64 Pauli masks per (site, op), flattened like T
    stn::DevBuf d_gate_gx, d_gate_gz;// uint64 generator masks per gate (0,0 = not a rotation)
    stn::DevBuf d_gate_dx;           // uint64 deterministic X mask applied after each gate (tiled lowering)
    stn::DevBuf d_obs;               // observable: u, v (uint32 pairs)
    stn::DevBuf d_obs_w;             // weights (double)
    stn::DevBuf d_obs_adj;           // observable terms per qubit: offsets [n + 1], then term indices

    // SV_LDS lowering
    std::vector<stn::LdsOp> lds_ops;
    std::vector<stn::GateGroup> gate_groups;   // gate-by-gate lowering: fused passes over tiles
    std::vector<stn::LdsOp> gate_group_ops;    // their operators, on tile-local qubits
    stn::DevBuf d_gate_group_ops;
    std::vector<stn::cd> lds_vals;          // dense / diag values of gates
    std::vector<uint32_t> site_op_off;      // per site: first entry in site_ops
    std::vector<stn::LdsOp> site_ops;       // per (site, j) operator descriptors
    stn::DevBuf d_lds_ops, d_lds_vals32, d_lds_vals64, d_site_ops, d_site_op_off;

    // SV_TILED lowering
    std::vector<stn::TiledLayer> layers;
    std::vector<stn::TiledPass> passes;
    void* tiled = nullptr;                  // pass tables of the tiled kernels (kernels_sv_tiled.hip)
    void (*tiled_free)(void*) = nullptr;
    stn::DevBuf d_work;                     // psi workspace [max_batch x 2^n]
    stn::DevBuf d_partials;                 // per (trajectory, tile) energy partials

    // per-kernel timing (stn_profile)
    bool prof = false;
    stn::ProfClass prof_cls[STN_K_COUNT];
    std::vector<hipEvent_t> ev_pool;

    // lightcone lowering (see lightcone.cpp)
    void* lc = nullptr;
    void (*lc_free)(void*) = nullptr;

    bool sync_on_destroy = true;            // false: the owner has waited for every enqueued use
    uint32_t variant = 0;                   // launch shape of the contraction kernels (autotuner)
    uint32_t grid_cap = 0;                  // persistent kernels use at most this many workgroups (0: all CUs)
    uint32_t lc_slices = 0, lc_slice_bits = 0;   // lightcone: networks per trajectory, most sliced variables
    uint32_t lc_group = 0;                       // lightcone: trajectories per workgroup work item
    uint32_t lc_width_lb = 0;                    // lightcone: lc_width is a lower bound (search stopped at the cap)
    bool sv_half = false;                        // tiled complex64: psi(~z) = psi(z), only qubit n-1 = 0 stored
    uint32_t tile_bits = 0;                      // tiled: qubits per tile (complex64: 14 or 15)
    bool graphs = false;                    // stn_contract replays HIP graphs (stn_plan_set_graphs)
    uint64_t graph_captures = 0, graph_replays = 0;
    bool tuned = false;
    ~stn_plan();
};

struct stn_batch {
    stn_plan* plan = nullptr;
    uint64_t k0 = 0;
    uint32_t K = 0;
    uint32_t words = 0;              // sign words per trajectory
    stn::DevBuf d_idx;               // uint8 [K x S]
    stn::DevBuf d_signs;             // uint32 [K x words]: bit g = rotation gate g flipped
    stn::DevBuf d_frame;             // uint64 [K x 2]: final frame x mask, z mask
    stn::DevBuf d_energy;            // double [K]
    stn::DevBuf d_states;            // complex [K x 2^n] (float2 or double2)
    stn::DevBuf d_gates_part;        // double [K x 64]: gate-by-gate lowering's energy slice sums
    stn::DevBuf d_queue;             // multi-batch launches led by this batch: their item counter
    stn::DevBuf d_map;               // stn_contract_dedup: representative of each trajectory
    stn_batch* unique = nullptr;     // stn_contract_dedup: the distinct trajectories
    bool contracted = false;
    bool has_states = false;
    // contraction graph of this batch: 0 none, 1 eager run done with gkey,
    // 2 captured with gkey (K, launch shape, CU cap, allocator generation)
    int gstate = 0;
    uint64_t gkey[4] = {0, 0, 0, 0};
    hipGraphExec_t gexec = nullptr;
    stn_batch() = default;
    stn_batch(const stn_batch&) = delete;
    stn_batch& operator=(const stn_batch&) = delete;
    ~stn_batch() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        delete unique;
    }
};

struct stn_accum {
    stn_plan* plan = nullptr;
    uint64_t k_done = 0;
    std::vector<std::pair<uint64_t, uint64_t>> ranges;  // reduced k ranges [a, b)
    std::vector<stn::DevBuf> e_chunks;                  // per-k energies, 65536 per chunk
    stn::DevBuf d_rho;               // double2 [2^n x 2^n] (upper triangle accumulated)
    stn::DevBuf d_diag;              // double [2^n]
    stn::DevBuf d_rho_out;           // double2 [2^n x 2^n]: mirrored, scaled by 1/K
    stn::DevBuf d_diag_out;          // double [2^n]: scaled by 1/K
    stn::DevBuf d_stats;             // double [4]: energy mean, SE, trace
    stn::DevBuf d_egather;           // double [k_done]: energies in trajectory order
    stn::DevBuf d_cdf;               // double [2^n]: running sums of d_diag (bitstring sampling)
    stn::DevBuf d_parts;             // double [2^n / 2048]: chunk sums of sigma (its trace)
    stn::HostBuf h_rho, h_diag, h_energies;   // pinned copies returned by stn_accum_read
};

namespace stn {
constexpr uint32_t kEnergyChunk = 65536;

// profiling hooks around a kernel launch on stream s (no-ops when off)
void prof_begin(stn_plan* p, int cls, hipStream_t s);
void prof_end(stn_plan* p, int cls, hipStream_t s, double bytes, double flops);
void prof_clear(stn_plan* p);

// device tables of a plan, uploaded on first device use (synchronises s)
void ensure_uploaded(stn_plan* p, hipStream_t s);
// (re)shapes a batch for trajectories k0 .. k0+K-1; buffers only grow
void batch_prepare(stn_plan* p, stn_batch* b, uint64_t k0, uint32_t K);
// enqueues the gather of per-trajectory energies and their statistics into d_stats
void accum_finish_energy(stn_accum* a, hipStream_t s);

// launch-shape variants of each lowering's contraction (results do not depend on them)
uint32_t lds_variants();
// one batch of a whole-state-in-LDS plan, as seen by the multi-batch kernel
struct LdsJob {
    const LdsOp* ops;
    const void* vals;
    const LdsOp* site_ops;
    const uint32_t* site_off;
    const uint8_t* idx;
    const uint32_t* obs_uv;
    const double* obs_w;
    double* energy;
    void* states;
    uint64_t item0;
    uint32_t n, n_ops, S, n_terms;
};
// batches per multi-batch launch (the descriptors are kernel arguments)
constexpr uint32_t kLdsQueueJobs = 32;
struct LdsQueue {
    LdsJob job[kLdsQueueJobs];
    uint64_t total;     // items of all batches
    uint32_t n_jobs;
};
void launch_sv_lds_many(stn_plan* const* plans, stn_batch* const* batches, uint32_t count, hipStream_t s);
uint32_t tn_variants();
uint32_t tiled_variants(const stn_plan* p);

// planner (plan.cpp)
void build_plan(stn_plan* p, const stn_circuit* c, const stn_noise_model* nm, const stn_observable* ob);

// Host threads a plan built on this thread may use for its lightcone
// networks (0: up to 8).  The job server's planner threads set 1: they
// already plan several jobs at once, and the device thread must not wait for
// a CPU.
extern thread_local uint32_t tl_plan_threads;

// load every kernel source file's device code on the current device, so that
// a job server's first jobs do not pay for it
void warm_code_sample();
void warm_code_sv_lds();
void warm_code_sv_gates();
void warm_code_sv_tiled();
void warm_code_sv_tiled128();
void warm_code_reduce();
void warm_code_tn();
inline void warm_device_code() {
    warm_code_sample();
    warm_code_sv_lds();
    warm_code_sv_gates();
    warm_code_sv_tiled();
    warm_code_sv_tiled128();
    warm_code_reduce();
    warm_code_tn();
}

// launchers (kernels_*.hip)
void launch_sample(stn_plan* p, stn_batch* b, uint64_t seed, hipStream_t s);
void launch_frame(stn_plan* p, stn_batch* b, hipStream_t s);
void launch_sv_lds(stn_plan* p, stn_batch* b, hipStream_t s);
void launch_sv_tiled(stn_plan* p, stn_batch* b, hipStream_t s);
// gate-by-gate HBM statevector lowering (any circuit and channel)
constexpr uint32_t kGatesMaxQubits = 30;
void launch_sv_gates(stn_plan* p, stn_batch* b, hipStream_t s);
// gate-by-gate lowering: fuses the operator list into tile passes (plan time)
// and uploads them
void build_gate_groups(stn_plan* p);
void upload_gate_groups(stn_plan* p, hipStream_t s);
void launch_reduce(stn_plan* p, stn_batch* b, stn_accum* a, hipStream_t s);
// fixed-order energy statistics over the gathered per-trajectory energies
void launch_energy_stats(stn_accum* a, uint64_t K, hipStream_t s);
// dst[k] = src[map[k]] for k < K
void launch_scatter_energy(const double* src, const uint32_t* map, uint32_t K, double* dst, hipStream_t s);
// rho_out = mirror(rho)/K, diag_out = diag/K, stats[2] = trace
void launch_finish_dense(stn_accum* a, hipStream_t s);
// m bitstrings drawn from the accumulated diagonal with the uniforms u (device arrays)
// bitstring sampling: running sums of acc's diagonal into work (device, at
// least sample_bits_scratch(n) bytes), then one draw per uniform
size_t sample_bits_scratch(uint32_t n);
void launch_sample_bits(stn_accum* a, const double* u, uint32_t m, uint32_t* out, double* work, hipStream_t s);
// the sampler's fixed device buffer on the current device (running sums of up
// to 2^kStaticSampleQubits states); NULL with the HIP error in *err when its
// address is unavailable
constexpr uint32_t kStaticSampleQubits = 20;
double* static_sample_scratch(hipError_t* err);
void launch_lightcone(stn_plan* p, stn_batch* b, hipStream_t s);
// lightcone lowering (kernels_tn.hip): networks of every observable term
void build_lightcone(stn_plan* p);
void upload_lightcone(stn_plan* p, hipStream_t s);
// tiled lowering (kernels_sv_tiled.hip): pass tables
void upload_tiled(stn_plan* p, hipStream_t s);
// complex128 tiled lowering (kernels_sv_tiled128.hip)
uint32_t tiled128_tile_bits();
void upload_tiled128(stn_plan* p, hipStream_t s);
void launch_sv_tiled128(stn_plan* p, stn_batch* b, hipStream_t s);
}  // namespace stn
