/*
 * stn.h - C ABI of the stochastic-noise trajectory-ensemble library (gfx950).
 *
 * Method (arXiv 2210.15874, Sec. III-G "Stochastic Noise Implementation"):
 * a noisy circuit is simulated as an ensemble of K noiseless-structure
 * circuits; after every gate that carries noise channels, one uniform draw
 * per channel picks a Kraus operator of the channel (Eq.(1), Sec. III-F) and
 * the operator it names is inserted.  Each member (trajectory) is contracted
 * to a statevector psi_k and the ensemble is reduced to
 *     rho_hat = (1/K) sum_k |psi_k><psi_k|,   sigma_approx = diag(rho_hat),
 * or to the QAOA MaxCut energy <C> = (1/K) sum_k <psi_k|C|psi_k>.
 *
 * The call sequence is plan -> sample -> contract -> reduce -> read:
 *   stn_plan_create   host: validates the circuit and noise model, builds the
 *                     noise-site table and the lowering (see stn_plan_kind),
 *                     uploads gate tables.  Once per job.
 *   stn_sample        device: Kraus index of every (trajectory, site) from
 *                     Philox4x32-10, plus the per-trajectory gate signs and
 *                     final Pauli frame.
 *   stn_contract      device: contracts every trajectory of a batch; the
 *                     trajectory index is the batch dimension of every kernel.
 *   stn_reduce        device: FP64 ensemble reduction into an accumulator.
 *   stn_accum_read    device -> host: K, rho_hat / sigma / <C> +- SE.
 *
 * Conventions
 *   - Qubit q is bit q of a basis index (little-endian).  A k-qubit matrix
 *     acting on (q0, q1) has local index bit(q0) + 2*bit(q1).
 *   - Complex matrices are row-major, interleaved (re, im) doubles.
 *   - rx/ry/rz(theta) = exp(-i theta P/2); zz(theta) = diag(1, e^{-i theta},
 *     e^{-i theta}, 1); cx has control q0, target q1.
 *   - Draw of site s in trajectory k: Philox4x32-10 with key (seed low, seed
 *     high) and counter (k low, k high, s, 0); word 0 is r.  With the
 *     selection probabilities q_j of the channel and binary64 prefix sums
 *     c_j, thresholds T_j = min(2^32, floor(c_j * 2^32)), T_{J-1} = 2^32, and
 *     the picked index is j = min{ j : r < T_j }.  The inserted operator is
 *     K_j / sqrt(q_j) with q_j = Tr(K_j^dagger K_j)/d.
 *
 * Ownership: every input is copied by the call that receives it; handles are
 * owned by the library until the matching *_destroy.  Device memory is taken
 * from opts->dev_alloc / dev_free when given, else from hipMalloc / hipFree.
 *
 * Streams: calls taking `stream` (a hipStream_t, NULL = legacy default stream)
 * only enqueue work; stn_accum_read and stn_batch_* readers synchronise it.
 *
 * Errors: every call returns a stn_status; no exception or abort crosses the
 * ABI.  A failing call leaves its output handles NULL and the accumulator
 * unchanged.  stn_last_error() returns a message for the last failure on the
 * calling thread.
 */
#ifndef STN_H
#define STN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    STN_OK = 0,
    STN_E_INVALID = 1,      /* malformed input (qubit out of range, non-CPTP channel, ...) */
    STN_E_UNSUPPORTED = 2,  /* valid input outside what the chosen lowering handles */
    STN_E_OOM = 3,          /* device allocation failed or budget exceeded */
    STN_E_DEVICE = 4,       /* HIP runtime error */
    STN_E_STATE = 5         /* call out of order (e.g. reduce before contract) */
} stn_status;

typedef enum {
    STN_G_H = 0, STN_G_X = 1, STN_G_Y = 2, STN_G_Z = 3,
    STN_G_RX = 4, STN_G_RY = 5, STN_G_RZ = 6, STN_G_ZZ = 7, STN_G_CX = 8,
    STN_G_U1 = 9,   /* explicit 2x2: mat = 8 doubles */
    STN_G_U2 = 10   /* explicit 4x4: mat = 32 doubles */
} stn_gate_kind;

typedef struct {
    uint32_t kind;          /* stn_gate_kind */
    uint32_t q0, q1;        /* q1 ignored for one-qubit gates */
    double theta;           /* rotation angle (rx, ry, rz, zz) */
    const double* mat;      /* U1 / U2 only, else NULL */
} stn_gate;

typedef struct {
    uint32_t n_qubits;
    uint32_t n_gates;
    const stn_gate* gates;
} stn_circuit;

typedef enum {
    STN_CH_BITFLIP = 0,     /* [sqrt(p) X, sqrt(1-p) I]                      (Sec. III-F) */
    STN_CH_DEPOL1 = 1,      /* [sqrt(1-3l/4) I, sqrt(l/4) X, Y, Z]           (Sec. III-F) */
    STN_CH_DEPOL2 = 2,      /* 16 Pauli products P_a(x)P_b, index 4a+b, P_a on q0,
                               weights 1-15l/16 (I(x)I) and l/16                        */
    STN_CH_AMPDAMP = 3,     /* [[1,0],[0,sqrt(1-g)]], [[0,sqrt(g)],[0,0]]                */
    STN_CH_KRAUS = 4        /* explicit: n_kraus matrices of 2x2 or 4x4 (by qubit count) */
} stn_channel_kind;

typedef struct {
    uint32_t after_gate;    /* index of the gate it follows; non-decreasing along the list */
    uint32_t kind;          /* stn_channel_kind */
    uint32_t n_qubits;      /* 1 or 2 */
    uint32_t q0, q1;
    double param;           /* p, lambda or gamma */
    uint32_t n_kraus;       /* STN_CH_KRAUS only */
    const double* kraus;    /* STN_CH_KRAUS only: n_kraus row-major interleaved matrices */
} stn_channel;

typedef struct {
    uint32_t n_channels;
    const stn_channel* channels;   /* site s = position in this array */
} stn_noise_model;

/* MaxCut-type observable C = sum_t w_t (1 - Z_{u_t} Z_{v_t}) / 2. */
typedef struct {
    uint32_t n_terms;
    const uint32_t* uv;     /* 2 * n_terms qubit indices */
    const double* w;        /* n_terms weights */
} stn_observable;

enum {
    STN_OUT_RHO = 1,        /* rho_hat (n <= 13) */
    STN_OUT_DIAG = 2,       /* sigma_approx = diag(rho_hat) (n <= 13; up to 30 in the gate-by-gate lowering) */
    STN_OUT_ENERGY = 4,     /* <C> and its standard error (needs an observable) */
    STN_OUT_STATES = 8      /* keep per-trajectory statevectors in the batch (n <= 13) */
};

typedef enum {
    STN_PLAN_AUTO = 0,
    STN_PLAN_SV_LDS = 1,    /* whole trajectory state in LDS, any circuit, n <= 13 (c64) / 12 (c128) */
    STN_PLAN_SV_TILED = 2,  /* HBM statevector, LDS/register-tiled passes, QAOA-structured
                               circuits with Pauli noise, energy only */
    STN_PLAN_LIGHTCONE = 3, /* per-term lightcone tensor networks, energy only */
    STN_PLAN_SV_GATES = 4   /* HBM statevector, one pass per gate or noise site: any circuit and any
                               channel (non-unitary ones included), 2 <= n <= 30, energy and sigma */
} stn_plan_kind;

typedef void* (*stn_alloc_fn)(size_t bytes, void* ctx);
typedef void (*stn_free_fn)(void* ptr, void* ctx);

/* The doubled network <0|U^dagger Z_u Z_v U|0> of one observable term, as a
 * lightcone plan builds it (Sec. III-A: tensors over binary variables).  The
 * arrays belong to the library and are valid during the callback only. */
typedef struct {
    uint32_t term;                  /* observable term index */
    uint32_t u, v;                  /* its qubits */
    uint32_t n_vars;                /* variables 0 .. n_vars-1 */
    uint32_t n_tensors;
    const uint32_t* tensor_offsets; /* n_tensors + 1 entries */
    const uint32_t* tensor_vars;    /* variables of tensor t: [tensor_offsets[t], tensor_offsets[t+1]) */
} stn_term_network;

/* Caller-supplied contraction order (Sec. III-A/B: bucket elimination sums the
 * variables out in a given order, whose quality sets the width).  Fills
 * order[0 .. n_vars) with a permutation of the network's variables, first
 * eliminated first, and returns 0; a nonzero return rejects the plan. */
typedef int (*stn_order_fn)(const stn_term_network* net, uint32_t* order, void* ctx);

typedef struct {
    uint32_t precision;     /* 64: complex64 contraction (FP32 arithmetic); 128: complex128 */
    uint32_t outputs;       /* STN_OUT_* bits */
    uint32_t plan_kind;     /* stn_plan_kind */
    uint32_t max_batch;     /* trajectories contracted per launch; 0 = derive from hbm_budget */
    uint64_t hbm_budget;    /* bytes of device working memory allowed; 0 = 64 GiB */
    uint32_t order_restarts;/* lightcone plans: randomized min-fill restarts (0 = 1 pass) */
    uint64_t order_seed;
    stn_alloc_fn dev_alloc; /* optional device allocator (e.g. a caching allocator) */
    stn_free_fn dev_free;
    void* alloc_ctx;
    uint32_t lc_max_rank;   /* lightcone plans: largest step rank (summed variable included: rank + 1
                               index bits); 0 = 23, the most the kernels take */
    uint32_t lc_slice_bits; /* lightcone plans: a network needing larger steps is sliced (Sec. III-C:
                               up to this many variables fixed to each value, the 2^bits results
                               summed); 0 = no slicing, at most 16 */
    stn_order_fn lc_order_fn; /* lightcone plans: NULL = min-fill (order_restarts, order_seed); else
                               called once per term, in term order, on the thread that calls
                               stn_plan_create, whenever lightcone networks are built (an AUTO plan
                               builds them to compare costs).  Not a permutation, or a nonzero
                               return: STN_E_INVALID.  Steps above lc_max_rank: STN_E_UNSUPPORTED
                               (an AUTO plan then takes another lowering).  Needs lc_slice_bits = 0 */
    void* lc_order_ctx;     /* passed to lc_order_fn */
    uint32_t sv_full_state; /* tiled plans: 1 = keep all 2^n amplitudes per trajectory.  0 (default):
                               keep the 2^(n-1) with qubit n-1 = 0.  Every trajectory circuit of the tiled
                               lowering (H on every qubit, then zz and rx gates whose signs the Pauli frame
                               sets) commutes with X on all qubits and starts from a state it fixes, so
                               psi(~z) = psi(z) exactly, and the ZZ observable takes equal values at z and ~z;
                               needs n >= 15 (complex64) / 13 (complex128) */
    uint32_t sv_tile_bits;  /* complex64 tiled plans: qubits per tile, 14 (512-thread workgroups, two resident per CU)
                               or 15 (1024 threads, one per CU; the strided tile of n <= 26 then reads 128-byte
                               runs); 0 (default) = 15 for n >= 25, else 14.  15 needs n >= 15.  Other values, or
                               nonzero on a complex128 plan: STN_E_INVALID */
} stn_plan_opts;

typedef struct {
    uint32_t plan_kind;     /* the lowering chosen */
    uint32_t n_qubits, n_gates, n_sites;
    uint32_t max_batch;
    uint32_t width;         /* contraction width: n for statevector plans, max rank for lightcone */
    uint32_t n_passes;      /* statevector HBM passes per trajectory (tiled plan; gate-by-gate plan: its fused
                               groups of operator-list entries, one launch each) */
    uint32_t n_steps;       /* contraction steps (lightcone plan) */
    double bytes_per_traj;  /* algorithmic HBM bytes per trajectory (cost model; gate-by-gate plan: an upper
                               bound, every fused group counted as moving the whole state) */
    double flops_per_traj;  /* algorithmic flops per trajectory (cost model) */
    double peak_bytes;      /* device working memory at max_batch */
    uint32_t lc_width;      /* lightcone networks' width when the planner built them (0: not built); a lower bound when
                               above the rank the lightcone lowering runs (its flops are then infinite) */
    double lc_flops_per_traj; /* their flops per trajectory */
    uint32_t variant;       /* launch shape of the contraction kernels (stn_plan_autotune) */
    uint32_t tuned;         /* 1 after stn_plan_autotune or stn_plan_set_variant */
    uint32_t graphs;        /* 1 while stn_contract uses HIP graphs (stn_plan_set_graphs) */
    uint64_t graph_captures;/* contraction graphs captured so far */
    uint64_t graph_replays; /* contractions run by replaying a captured graph */
    uint32_t lc_slices;     /* lightcone plans: networks contracted per trajectory (terms x slices) */
    uint32_t lc_slice_bits; /* largest number of sliced variables of one term */
    double est_s_per_traj;  /* cost model's device seconds per trajectory of the chosen lowering (the job
                               server's admission and scheduling estimate; not a measurement) */
    uint32_t lc_group;      /* lightcone plans: trajectories one workgroup contracts in lockstep */
    uint32_t lc_width_lower_bound; /* 1 when lc_width is only a lower bound: the elimination-order search
                               stopped at the first step above the rank cap, before finishing the order */
    uint32_t half_state;    /* tiled plan keeps half the amplitudes (see stn_plan_opts.sv_full_state); bytes_per_traj
                               and peak_bytes count those */
    uint32_t tile_bits;     /* tiled plan: qubits per tile (see stn_plan_opts.sv_tile_bits); 0 for other lowerings */
} stn_plan_stats;

typedef struct {
    uint32_t n_variants;    /* launch shapes of this plan's lowering */
    uint32_t chosen;        /* the fastest, now the plan's */
    double ms[8];           /* per variant: mean event time of one contraction of the batch */
} stn_tune_result;

typedef struct {
    uint64_t k_done;        /* trajectories reduced so far */
    double energy_mean;     /* <C>_hat (ENERGY) */
    double energy_se;       /* std(<C>_k, ddof=1)/sqrt(K) */
    double trace_mean;      /* Tr rho_hat (RHO / DIAG); 1 up to rounding for Pauli noise */
    const double* rho;      /* 2^n x 2^n interleaved complex128, row-major, /K applied (RHO) */
    const double* diag;     /* 2^n doubles, /K applied (DIAG) */
    const double* energies; /* k_done per-trajectory <C>_k in trajectory order (ENERGY) */
} stn_result;

typedef struct stn_plan stn_plan;
typedef struct stn_batch stn_batch;
typedef struct stn_accum stn_accum;

/* Version string of the library. */
const char* stn_version(void);

/* Message for the last non-OK status returned on this thread. */
const char* stn_last_error(void);

/* Fills *opts with defaults: precision 64, outputs ENERGY, plan AUTO. */
void stn_plan_opts_default(stn_plan_opts* opts);

/* Plan one job (Sec. III-G: the ideal circuit, the noise model; III-A:
 * bucket elimination order for lightcone plans).  observable may be NULL when
 * ENERGY is not requested.  On success *out owns copies of all inputs and the
 * device tables; STN_E_INVALID / STN_E_UNSUPPORTED describe the offending
 * gate / channel in stn_last_error(). */
stn_status stn_plan_create(const stn_circuit* circuit, const stn_noise_model* noise,
                           const stn_observable* observable, const stn_plan_opts* opts,
                           stn_plan** out);
stn_status stn_plan_info(const stn_plan* plan, stn_plan_stats* out);
/* Releases the caller's handle (NULL: no-op).  Batches and accumulators made
 * from the plan keep it alive: its memory goes with the last of them, so the
 * handles may be destroyed in any order.  The plan must not be used through
 * this handle afterwards. */
void stn_plan_destroy(stn_plan* plan);

/* Noise-site table of a plan (Sec. III-G selection rule): *n_ops receives
 * the site's operator count J and thresholds[0 .. min(J, cap)) its integer
 * thresholds T_j (T_{J-1} = 2^32).  Host-only; needs no device.  Planning
 * itself touches no device either: device tables are uploaded by the first
 * stn_sample / stn_batch_from_indices / stn_contract on the plan. */
stn_status stn_plan_site(const stn_plan* plan, uint32_t site, uint32_t* n_ops, uint64_t* thresholds,
                         uint32_t cap);

/* Draw trajectories k0 .. k0+K-1 of job `seed` (Sec. III-G: one uniform
 * number per channel picks its Kraus operator).  The draws depend only on
 * (seed, k, site).  K may exceed max_batch: contract splits it. */
stn_status stn_sample(stn_plan* plan, uint64_t seed, uint64_t k0, uint32_t K,
                      stn_batch** out, void* stream);

/* Draws trajectories k0 .. k0+K-1 of job `seed` into an existing batch of
 * its plan, replacing its contents (Sec. III-G selection rule: the same
 * draws as stn_sample).  Device
 * buffers are kept when large enough, so a caller running many chunks
 * allocates once; work already enqueued on the batch must be ordered before
 * this call (same stream). */
stn_status stn_resample(stn_batch* batch, uint64_t seed, uint64_t k0, uint32_t K, void* stream);

/* Batch from caller-chosen Kraus indices: idx is a host array [K x n_sites]
 * of uint8 (index j of each site's operator, < the channel's operator count).
 * Used to enumerate outcomes exactly. k0 only labels the trajectories. */
stn_status stn_batch_from_indices(stn_plan* plan, const uint8_t* idx, uint64_t k0, uint32_t K,
                                  stn_batch** out, void* stream);

/* Copies the batch's Kraus index table [K x n_sites] to host memory. Syncs. */
stn_status stn_batch_indices(const stn_batch* batch, uint8_t* host_out);

/* Contract every trajectory of the batch (Sec. III-G: simulate each noisy
 * circuit to its statevector).  Produces per-trajectory energies and, for
 * RHO / DIAG / STATES outputs, the statevectors. */
stn_status stn_contract(stn_plan* plan, stn_batch* batch, void* stream);

/* Copies per-trajectory results to host memory (syncs): energies[K] (FP64)
 * and, when the batch keeps states, states[K x 2^n] complex (interleaved
 * doubles; complex64 batches are widened).  Either pointer may be NULL. */
stn_status stn_batch_results(const stn_batch* batch, double* energies, double* states);
uint32_t stn_batch_size(const stn_batch* batch);
/* Syncs the device, frees the batch and releases its hold on the plan. */
void stn_batch_destroy(stn_batch* batch);

/* Per-kernel timing of a plan's launches, taken with HIP events recorded on
 * the stream each kernel is launched on.  bytes / flops are the algorithmic
 * HBM traffic and arithmetic of the launches (the cost model's counts, not
 * hardware counters). */
enum {
    STN_K_SAMPLE = 0,       /* Philox selection of every (trajectory, site) */
    STN_K_FRAME = 1,        /* Pauli-frame scan */
    STN_K_SV_LDS = 2,       /* whole-state-in-LDS contraction */
    STN_K_SV_PASS = 3,      /* HBM statevector passes (tiled, or gate by gate) */
    STN_K_TILE_SUM = 4,     /* per-trajectory energy from tile partials */
    STN_K_HERK = 5,         /* FP64 rho_hat accumulation */
    STN_K_DIAG = 6,         /* FP64 sigma accumulation */
    STN_K_TN_STEP = 7,      /* lightcone tensor-network step */
    STN_K_COUNT = 8
};
typedef struct {
    uint64_t launches;
    double ms;              /* summed event time */
    double bytes;           /* summed algorithmic bytes */
    double flops;           /* summed algorithmic flops */
} stn_kernel_stats;

/* Enables (1) or disables (0) per-kernel timing on the plan and clears it. */
stn_status stn_profile(stn_plan* plan, int enable);
/* Fills out[0 .. STN_K_COUNT) with the timings since enabling. Syncs. */
stn_status stn_profile_read(stn_plan* plan, stn_kernel_stats* out);

/* Contracts each distinct trajectory of the batch once (Sec. III-G: many
 * sampled circuits coincide, e.g. all error-free ones) and copies its energy
 * to the trajectories that equal it.  Trajectories are equal when their
 * Kraus indices are (whole-state-in-LDS plans) or when their gate signs and
 * final-frame X part are (Pauli-frame plans: tiled, lightcone).  Energies are
 * those of stn_contract, bit for bit; *n_unique (may be NULL) receives the
 * number of distinct trajectories.  Energy outputs only (RHO / DIAG /
 * STATES: STN_E_UNSUPPORTED).  Synchronises the stream (the keys are read on
 * the host). */
stn_status stn_contract_dedup(stn_plan* plan, stn_batch* batch, uint32_t* n_unique, void* stream);

/* Contracts the batches of several whole-state-in-LDS plans (n <= 13 in
 * complex64, n <= 12 in complex128; all of one precision) in one launch
 * (Sec. III-D, sample parallelism: many small circuits share one GPU):
 * persistent workgroups take (batch, trajectory) items from a device-side
 * queue (an atomic counter over the items of all batches, batch after batch)
 * until it is empty, so many small jobs fill the device together.  Results
 * equal stn_contract of each batch, bit for bit.  The launch shape is that of
 * plans[0]; the queue's item counter lives with batches[0], so a batch must
 * not lead two multi-batch launches that may overlap (on two streams).  Up to
 * 32 batches go into one launch (more: several launches).  The call copies
 * nothing from the host and never waits for the stream.  Other lowerings:
 * STN_E_UNSUPPORTED; mixed precision or a repeated batch: STN_E_INVALID. */
stn_status stn_contract_many(stn_plan* const* plans, stn_batch* const* batches, uint32_t count, void* stream);

/* Launch-shape autotuning: contracts `batch` (a sampled batch of this plan)
 * `reps` times with every launch shape of the plan's lowering (threads per
 * workgroup of the LDS and lightcone kernels, persistent grid of the tiled
 * one), timed with HIP events on `stream`, and keeps the fastest.  Results do
 * not depend on the shape (each output has one writer in a fixed order), so
 * the batch is left contracted.  Synchronises the stream. */
stn_status stn_plan_autotune(stn_plan* plan, stn_batch* batch, uint32_t reps, stn_tune_result* out, void* stream);
/* Sets the launch shape directly (a cached tuning result); out of range:
 * STN_E_INVALID. */
stn_status stn_plan_set_variant(stn_plan* plan, uint32_t variant);

/* HIP graphs for the contraction (on: 1, off: 0; off by default).  With
 * graphs on, stn_contract runs a batch's launches eagerly the first time it
 * sees that batch with a given K, launch shape, CU cap and device workspace,
 * captures them into a HIP graph the second time and replays the graph on
 * later calls (a caller that refills one batch with stn_resample for every
 * chunk pays the launch sequence once).  A change of any of these (for
 * example a reallocation by the plan's allocator) starts over.  Results are
 * those of eager launches, bit for bit.  Graphs are not used while profiling
 * is on, on the NULL stream, or when the caller is already capturing the
 * stream.  The graph belongs to the batch and is freed with it. */
stn_status stn_plan_set_graphs(stn_plan* plan, uint32_t on);

/* Accumulator of one job's ensemble sums (FP64, device-resident). */
stn_status stn_accum_create(stn_plan* plan, stn_accum** out);

/* FP64 reduction of a contracted batch (Sec. III-G: sigma_approx = sum phi_k/K,
 * generalised to rho_hat and <C>). */
stn_status stn_reduce(stn_plan* plan, stn_batch* batch, stn_accum* acc, void* stream);

/* Finishes the fixed-order reductions and copies the result to host memory
 * owned by the accumulator (valid until the next read or destroy). Syncs. */
stn_status stn_accum_read(stn_accum* acc, stn_result* out, void* stream);
/* Syncs the device, frees the accumulator and releases its hold on the plan. */
void stn_accum_destroy(stn_accum* acc);

/* Bitstring samples from the ensemble's probability vector (Sec. III-G:
 * sigma_approx, the average of the trajectories' probability vectors, is a
 * distribution over the 2^n basis states).  For each j < m, out[j] = the basis
 * index x (qubit q in bit q) drawn by inverse transform with the uniform u[j]:
 * with the running sums F(x) = sigma(0) + ... + sigma(x) of the trajectories
 * reduced into acc so far, the smallest x with F(x) > u[j] F(2^n - 1); when
 * rounding leaves none, the smallest x with F(x) >= u[j] F(2^n - 1).  Indices
 * of zero mass are never drawn unless all mass is zero (then x = 0).
 *   u    device, m doubles in [0, 1), caller-owned (other values still give
 *        indices in [0, 2^n))
 *   out  device, m uint32, caller-owned
 * Needs a plan with STN_OUT_DIAG or STN_OUT_RHO and at least one reduced
 * batch (STN_E_STATE otherwise); m = 0 does nothing.  Up to 2^13 states the
 * running sums are searched in LDS, above that in device memory.  Enqueued on stream,
 * after the stn_reduce calls enqueued there before it; does not sync. */
stn_status stn_accum_sample(stn_accum* acc, const double* u, uint32_t m, uint32_t* out, void* stream);

/* stn_accum_sample for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, hosts that forbid hipMalloc): the
 * same draws, bit for bit, with the running sums kept in a fixed device
 * buffer of the library (2^20 + 512 doubles, 8 MiB + 4 KiB per device, held
 * until the process ends) instead of memory the accumulator allocates.  It
 * calls no allocator.  Arguments, ownership and stream order as for
 * stn_accum_sample; plans with n > 20 get STN_E_UNSUPPORTED.  The buffer is
 * shared by every call on a device and overwritten by each one: calls that
 * overlap on one device (different streams or threads without ordering
 * between them) race and may return wrong indices. */
stn_status stn_accum_sample_noalloc(stn_accum* acc, const double* u, uint32_t m, uint32_t* out, void* stream);

/* ---------------------------------------------------------------- job server
 * Many ensemble jobs (Sec. III-G, each one circuit + noise model + K) of
 * different sizes on one device at once.  Planner threads plan submitted
 * jobs on the host (reusing cached plans of identical inputs); a device
 * thread admits planned jobs in arrival order while their estimated device
 * memory fits hbm_budget (a job of at most 1/32 of the budget may go ahead of
 * a larger one that does not fit yet; larger jobs fill at most 15/16 of the
 * budget, so small ones always find room), gives each a stream, and issues their
 * trajectories in chunks (sample -> contract -> reduce), round-robin over the
 * admitted jobs, so that jobs arriving while others run share the device
 * with them.  A job's result depends only on its inputs, seed and K: it is
 * the same (bit for bit) alone and in any mix.
 *
 * Device memory: hbm_budget bytes are reserved with one hipMalloc when the
 * server starts (stn_server_create returns once they are) and handed out
 * first-fit; plans and accumulators stay on the device while their job runs.
 * Only <C> jobs (an observable, ENERGY output) are served.
 */
typedef struct stn_server stn_server;

typedef struct {
    uint64_t hbm_budget;     /* device bytes the server may hold (>= 64 MiB) */
    double job_share;        /* largest fraction of the budget one job's chunk may use, (0, 1] */
    uint32_t n_streams;      /* job streams, 1..8: stream 0 for small jobs, the others for large ones; one
                                more stream carries table uploads and tuning runs.  Keep n_streams + 1
                                within the process's hardware queues (GPU_MAX_HW_QUEUES) */
    uint32_t max_active;     /* jobs admitted at once, 1..64 */
    uint32_t plan_cache;     /* idle plans kept for jobs with identical inputs (0: none) */
    uint32_t precision;      /* 64 (complex64) or 128 (complex128) for every job */
    uint32_t chunk_max;      /* trajectories per chunk cap (0: the plan's max batch) */
    uint32_t drain_on_destroy; /* 1: stn_server_destroy waits for every submitted job */
    uint32_t reserve_cus;    /* CUs the persistent kernels (tiled statevector, lightcone networks in
                                HBM) leave free for other jobs' kernels */
    uint32_t graphs;         /* 1: chunk contractions replay HIP graphs (stn_plan_set_graphs); off by
                                default, since a graph launch costs more host time than the one to six
                                kernel launches of a contraction it replaces */
    uint32_t gang;           /* 1: ready chunks of whole-state-in-LDS jobs on the shared stream are
                                contracted together by one multi-batch launch (stn_contract_many) */
} stn_server_opts;

typedef struct {
    uint64_t job_id;         /* as returned by stn_server_submit */
    uint64_t tag;            /* the caller's tag */
    uint32_t status;         /* stn_status of the job (planning or device failure) */
    uint32_t plan_kind;      /* lowering used */
    uint32_t width;          /* its contraction width */
    uint32_t chunk;          /* trajectories per chunk */
    uint64_t K, k_done;
    uint64_t chunks;         /* chunks issued */
    double energy_mean;      /* <C>_hat over k = 0 .. K-1 */
    double energy_se;        /* std(<C>_k, ddof=1)/sqrt(K) */
    double t_submit;         /* seconds on the server clock (stn_server_clock) */
    double t_admit;
    double t_done;
    char error[96];          /* message when status != STN_OK */
} stn_job_result;

typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t active;         /* jobs admitted and not finished */
    uint64_t waiting;        /* jobs submitted and not admitted */
    uint64_t trajectories;   /* trajectories of completed jobs */
    uint64_t chunks;         /* chunks issued */
    uint64_t max_active_jobs;/* most jobs admitted at the same time */
    uint64_t plan_cache_hits, plan_cache_misses, plans_cached;
    uint64_t autotuned;      /* plan shapes whose launch shape was timed (then reused for the shape) */
    uint64_t bytes_in_use, bytes_cached, bytes_peak;   /* device memory reserved at create: in use, free, peak in use */
    double clock;            /* server clock when read */
    uint64_t gang_launches;  /* multi-batch launches (stn_contract_many) of several jobs' chunks */
    uint64_t gang_chunks;    /* chunks contracted by them */
} stn_server_stats;

/* Defaults: 64 GiB budget, job_share 0.5, 3 streams, 16 active jobs, 64
 * cached plans, complex64, drain on destroy, 32 reserved CUs, graphs off,
 * multi-batch launches on. */
void stn_server_opts_default(stn_server_opts* opts);
/* Starts the server's threads on the calling thread's current device. */
stn_status stn_server_create(const stn_server_opts* opts, stn_server** out);
/* Queues a job (inputs are copied; returns at once).  The job's draws are
 * those of stn_sample(plan, seed, 0, K).  observable is required. */
stn_status stn_server_submit(stn_server* server, const stn_circuit* circuit, const stn_noise_model* noise,
                             const stn_observable* observable, uint64_t seed, uint64_t K, uint64_t tag,
                             uint64_t* job_id);
/* Moves up to cap finished jobs' results to out (completion order), waiting
 * up to wait_s seconds for the first one when none is ready. */
stn_status stn_server_poll(stn_server* server, stn_job_result* out, uint32_t cap, uint32_t* n_out, double wait_s);
/* Waits until every submitted job has finished (STN_E_STATE on timeout). */
stn_status stn_server_drain(stn_server* server, double timeout_s);
stn_status stn_server_stats_read(stn_server* server, stn_server_stats* out);
/* Seconds since the server was created (the clock of t_submit / t_done). */
double stn_server_clock(const stn_server* server);
/* Message of the last non-OK status of a stn_server_* call on this thread. */
const char* stn_server_last_error(void);
/* Stops the threads (after draining, when drain_on_destroy) and frees the
 * server, its cached plans and its device pool. */
void stn_server_destroy(stn_server* server);

#ifdef __cplusplus
}
#endif

#endif /* STN_H */
