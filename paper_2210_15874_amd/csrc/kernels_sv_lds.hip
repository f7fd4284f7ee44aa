// Whole-trajectory-in-LDS statevector contraction (Sec. III-G: each noisy
// circuit of the ensemble is simulated to its statevector).  One workgroup
// owns one trajectory: its 2^n amplitudes live in LDS for the whole circuit
// (n <= 13 in complex64, n <= 12 in complex128: 64 KiB), and the gate list is
// interpreted in order.  After every gate the trajectory's picked Kraus
// operator of each of the gate's channels is applied literally (a Pauli as a
// signed permutation with its global phase dropped, any other operator as
// the dense K_j / sqrt(q_j)).  The trajectory index is the grid dimension, so
// every launch contracts the whole batch.
//
// Epilogue: optionally the final statevector, then the energy <psi|C|psi> of
// C = sum_t w_t [z_u != z_v]: each amplitude's term in binary64 into LDS, and
// a pairwise tree over the 2^n terms, so the result does not depend on the
// workgroup size (a launch shape the autotuner picks).
#include "sv_ops.h"

namespace stn {

namespace {

template <class R> struct Cx;
template <> struct Cx<float> { using T = float2; };
template <> struct Cx<double> { using T = double2; };

// One trajectory of one plan in the workgroup's LDS (psi: 2^n amplitudes,
// plus 2^n binary64 terms for complex128): the gate list with the picked
// Kraus operators of `row`, then the optional state and the energy.
template <class R, int kThreads>
__device__ __forceinline__ void lds_trajectory(typename Cx<R>::T* psi, uint32_t n, const LdsOp* __restrict__ ops,
                                               uint32_t n_ops, const typename Cx<R>::T* __restrict__ vals,
                                               const LdsOp* __restrict__ site_ops,
                                               const uint32_t* __restrict__ site_off,
                                               const uint8_t* __restrict__ row,
                                               const uint32_t* __restrict__ obs_uv,
                                               const double* __restrict__ obs_w, uint32_t n_terms,
                                               double* __restrict__ energy, typename Cx<R>::T* __restrict__ state) {
    using V = typename Cx<R>::T;
    const uint32_t tid = threadIdx.x;
    const uint32_t N = 1u << n;
    for (uint32_t i = tid; i < N; i += kThreads) {
        V v;
        v.x = i == 0 ? R(1) : R(0);
        v.y = R(0);
        psi[i] = v;
    }
    __syncthreads();
    for (uint32_t oi = 0; oi < n_ops; ++oi) {
        LdsOp o = ops[oi];
        if (o.kind == OP_SITE) o = site_ops[site_off[o.site] + row[o.site]];
        apply_lds_op<V>(psi, N, o, vals, tid, kThreads);
        __syncthreads();
    }
    // energy <psi|C|psi> in binary64: per-amplitude terms, then a fixed tree
    if (state)
        for (uint32_t i = tid; i < N; i += kThreads) state[i] = psi[i];
    double* e = reinterpret_cast<double*>(psi) + (sizeof(V) == 8 ? 0 : 2 * (size_t)N);
    for (uint32_t i = tid; i < N; i += kThreads) {
        const V v = psi[i];   // complex64: e[i] takes psi[i]'s own 8 bytes
        const double pr = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
        double c = 0.0;
        for (uint32_t t = 0; t < n_terms; ++t)
            c += ((i >> obs_uv[2 * t]) ^ (i >> obs_uv[2 * t + 1])) & 1 ? obs_w[t] : 0.0;
        e[i] = pr * c;
    }
    __syncthreads();
    for (uint32_t h = N / 2; h > 0; h >>= 1) {
        for (uint32_t i = tid; i < h; i += kThreads) e[i] += e[i + h];
        __syncthreads();
    }
    if (tid == 0) *energy = e[0];
}

template <class R, int kThreads>
__global__ __launch_bounds__(kThreads) void k_sv_lds(uint32_t n, const LdsOp* __restrict__ ops, uint32_t n_ops,
                                                    const typename Cx<R>::T* __restrict__ vals,
                                                    const LdsOp* __restrict__ site_ops,
                                                    const uint32_t* __restrict__ site_off,
                                                    const uint8_t* __restrict__ idx, uint32_t S,
                                                    const uint32_t* __restrict__ obs_uv,
                                                    const double* __restrict__ obs_w, uint32_t n_terms,
                                                    double* __restrict__ energy,
                                                    typename Cx<R>::T* __restrict__ states) {
    using V = typename Cx<R>::T;
    extern __shared__ char smem_raw[];
    const uint32_t b = blockIdx.x;
    lds_trajectory<R, kThreads>(reinterpret_cast<V*>(smem_raw), n, ops, n_ops, vals, site_ops, site_off,
                                idx + (size_t)b * S, obs_uv, obs_w, n_terms, energy + b,
                                states ? states + ((size_t)b << n) : nullptr);
}

// Several plans' batches in one launch: a queue of (batch, trajectory) items,
// numbered batch after batch (batch j owns items [item0_j, item0_j + K_j)).
// Persistent workgroups take the next item from an atomic counter until it
// passes the total, so every workgroup exits once the queue is empty.
template <class R, int kThreads>
__global__ __launch_bounds__(kThreads) void k_sv_lds_queue(const LdsQueue q, unsigned long long* __restrict__ counter) {
    const LdsJob* jobs = q.job;
    const uint32_t n_jobs = q.n_jobs;
    const unsigned long long total = q.total;
    using V = typename Cx<R>::T;
    extern __shared__ __align__(16) char smem_raw[];
    __shared__ unsigned long long s_item;
    __shared__ uint32_t s_job;
    while (true) {
        // a barrier first: the previous item is finished everywhere (its LDS
        // and s_item reads), and nothing the fetching thread does below is
        // next to the same thread's energy store of that item without a
        // barrier between them (the compiler could otherwise route that
        // thread around a different loop than the others)
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long it = atomicAdd(counter, 1ull);
            uint32_t lo = 0, hi = n_jobs - 1;   // last job with item0 <= it
            if (it < total)
                while (lo < hi) {
                    const uint32_t mid = (lo + hi + 1) / 2;
                    if (jobs[mid].item0 <= it) lo = mid;
                    else hi = mid - 1;
                }
            s_item = it;
            s_job = lo;
        }
        __syncthreads();
        // the same item for the whole workgroup, read as a uniform (scalar)
        // value so that the loop exit is a uniform branch
        const uint32_t ilo = __builtin_amdgcn_readfirstlane((uint32_t)s_item);
        const uint32_t ihi = __builtin_amdgcn_readfirstlane((uint32_t)(s_item >> 32));
        const uint32_t j = __builtin_amdgcn_readfirstlane(s_job);
        const unsigned long long it = ((unsigned long long)ihi << 32) | ilo;
        if (it >= total) break;
        const LdsJob& J = jobs[j];
        const uint64_t b = it - J.item0;
        V* st = static_cast<V*>(J.states);
        lds_trajectory<R, kThreads>(reinterpret_cast<V*>(smem_raw), J.n, J.ops, J.n_ops,
                                    static_cast<const V*>(J.vals), J.site_ops, J.site_off, J.idx + b * J.S,
                                    J.obs_uv, J.obs_w, J.n_terms, J.energy + b, st ? st + (b << J.n) : nullptr);
    }
}

__global__ void k_zero_counter(unsigned long long* c) { *c = 0ull; }

template <class R>
using LdsFn = void (*)(uint32_t, const LdsOp*, uint32_t, const typename Cx<R>::T*, const LdsOp*, const uint32_t*,
                       const uint8_t*, uint32_t, const uint32_t*, const double*, uint32_t, double*,
                       typename Cx<R>::T*);

struct LdsKernel {
    void* f;
    uint32_t threads;
};

// launch shapes the autotuner chooses from (variant 0 is the default)
constexpr uint32_t kLdsVariants = 4;
template <class R>
LdsKernel lds_kernel(uint32_t v) {
    switch (v) {
        case 1: return {(void*)k_sv_lds<R, 128>, 128};
        case 2: return {(void*)k_sv_lds<R, 512>, 512};
        case 3: return {(void*)k_sv_lds<R, 1024>, 1024};
        default: return {(void*)k_sv_lds<R, 256>, 256};
    }
}

}  // namespace

void launch_sv_lds(stn_plan* p, stn_batch* b, hipStream_t s) {
    const uint32_t n = p->n;
    const size_t N = (size_t)1 << n;
    const bool dense = p->opts.outputs & (STN_OUT_RHO | STN_OUT_DIAG | STN_OUT_STATES);
    const bool dbl = p->opts.precision == 128;
    const size_t elem = dbl ? 16 : 8;
    if (dense) {
        b->d_states.ensure(&p->alloc, N * b->K * elem);
        b->has_states = true;
    }
    // complex128 needs room for the binary64 terms beside the state
    const size_t lds = N * elem + (dbl ? N * 8 : 0);
    const uint32_t S = (uint32_t)p->sites.size();
    const uint32_t T = (uint32_t)p->obs_u.size();
    const uint32_t v = std::min<uint32_t>(p->variant, kLdsVariants - 1);
    const LdsKernel ker = dbl ? lds_kernel<double>(v) : lds_kernel<float>(v);
    static bool attr_set[2][kLdsVariants] = {};
    if (!attr_set[dbl][v]) {
        STN_HIP(hipFuncSetAttribute((const void*)ker.f, hipFuncAttributeMaxDynamicSharedMemorySize, 98304));
        attr_set[dbl][v] = true;
    }
    // the grid dimension is capped; larger batches run in slices
    for (uint32_t k0 = 0; k0 < b->K; k0 += 65535) {
        const uint32_t nb = std::min<uint32_t>(65535, b->K - k0);
        prof_begin(p, STN_K_SV_LDS, s);
        if (dbl) {
            hipLaunchKernelGGL(reinterpret_cast<LdsFn<double>>(ker.f), dim3(nb), dim3(ker.threads), lds, s, n,
                               p->d_lds_ops.as<LdsOp>(), (uint32_t)p->lds_ops.size(), p->d_lds_vals64.as<double2>(),
                               p->d_site_ops.as<LdsOp>(), p->d_site_op_off.as<uint32_t>(),
                               b->d_idx.as<uint8_t>() + (size_t)k0 * S, S, p->d_obs.as<uint32_t>(),
                               p->d_obs_w.as<double>(), T, b->d_energy.as<double>() + k0,
                               dense ? b->d_states.as<double2>() + (size_t)k0 * N : nullptr);
        } else {
            hipLaunchKernelGGL(reinterpret_cast<LdsFn<float>>(ker.f), dim3(nb), dim3(ker.threads), lds, s, n,
                               p->d_lds_ops.as<LdsOp>(), (uint32_t)p->lds_ops.size(), p->d_lds_vals32.as<float2>(),
                               p->d_site_ops.as<LdsOp>(), p->d_site_op_off.as<uint32_t>(),
                               b->d_idx.as<uint8_t>() + (size_t)k0 * S, S, p->d_obs.as<uint32_t>(),
                               p->d_obs_w.as<double>(), T, b->d_energy.as<double>() + k0,
                               dense ? b->d_states.as<float2>() + (size_t)k0 * N : nullptr);
        }
        STN_HIP(hipGetLastError());
        prof_end(p, STN_K_SV_LDS, s, (double)nb * ((dense ? N * elem : 0) + S + 8.0), (double)nb * p->flops_per_traj);
    }
}

uint32_t lds_variants() { return kLdsVariants; }

void launch_sv_lds_many(stn_plan* const* plans, stn_batch* const* batches, uint32_t count, hipStream_t s) {
    if (count == 0) return;
    const bool dbl = plans[0]->opts.precision == 128;
    const size_t elem = dbl ? 16 : 8;
    std::vector<LdsJob> jobs(count);
    for (uint32_t i = 0; i < count; ++i) {
        stn_plan* p = plans[i];
        stn_batch* b = batches[i];
        const size_t N = (size_t)1 << p->n;
        const bool dense = p->opts.outputs & (STN_OUT_RHO | STN_OUT_DIAG | STN_OUT_STATES);
        if (dense) {
            b->d_states.ensure(&p->alloc, N * b->K * elem);
            b->has_states = true;
        }
        LdsJob& J = jobs[i];
        J.ops = p->d_lds_ops.as<LdsOp>();
        J.vals = dbl ? (const void*)p->d_lds_vals64.p : (const void*)p->d_lds_vals32.p;
        J.site_ops = p->d_site_ops.as<LdsOp>();
        J.site_off = p->d_site_op_off.as<uint32_t>();
        J.idx = b->d_idx.as<uint8_t>();
        J.obs_uv = p->d_obs.as<uint32_t>();
        J.obs_w = p->d_obs_w.as<double>();
        J.energy = b->d_energy.as<double>();
        J.states = dense ? b->d_states.p : nullptr;
        J.item0 = 0;
        J.n = p->n;
        J.n_ops = (uint32_t)p->lds_ops.size();
        J.S = (uint32_t)p->sites.size();
        J.n_terms = (uint32_t)p->obs_u.size();
    }
    // the counter lives with the first batch; the descriptors travel as
    // kernel arguments, kLdsQueueJobs batches per launch (no host copy, so
    // the call does not wait for earlier work on the stream)
    stn_batch* owner = batches[0];
    owner->d_queue.ensure(&plans[0]->alloc, 256);
    auto* counter = static_cast<unsigned long long*>(owner->d_queue.p);
    const uint32_t v = std::min<uint32_t>(plans[0]->variant, kLdsVariants - 1);
    const uint32_t threads = v == 1 ? 128 : v == 2 ? 512 : v == 3 ? 1024 : 256;
    using QFn = void (*)(const LdsQueue, unsigned long long*);
    QFn f;
    if (dbl) f = v == 1 ? k_sv_lds_queue<double, 128> : v == 2 ? k_sv_lds_queue<double, 512>
               : v == 3 ? k_sv_lds_queue<double, 1024> : k_sv_lds_queue<double, 256>;
    else f = v == 1 ? k_sv_lds_queue<float, 128> : v == 2 ? k_sv_lds_queue<float, 512>
             : v == 3 ? k_sv_lds_queue<float, 1024> : k_sv_lds_queue<float, 256>;
    static bool attr_set[2][kLdsVariants] = {};
    if (!attr_set[dbl][v]) {
        STN_HIP(hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, 98304));
        attr_set[dbl][v] = true;
    }
    int dev = 0, cus = 0;
    STN_HIP(hipGetDevice(&dev));
    STN_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    for (uint32_t g0 = 0; g0 < count; g0 += kLdsQueueJobs) {
        const uint32_t ng = std::min<uint32_t>(kLdsQueueJobs, count - g0);
        LdsQueue q{};
        uint64_t tot = 0;
        size_t lds = 0;
        for (uint32_t i = 0; i < ng; ++i) {
            q.job[i] = jobs[g0 + i];
            q.job[i].item0 = tot;
            tot += batches[g0 + i]->K;
            lds = std::max(lds, ((size_t)1 << jobs[g0 + i].n) * elem + (dbl ? ((size_t)8 << jobs[g0 + i].n) : 0));
        }
        q.n_jobs = ng;
        q.total = tot;
        hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, s, counter);
        STN_HIP(hipGetLastError());
        // workgroups resident at once: LDS (160 KiB per CU) and at most 8 per CU
        const uint64_t per_cu = std::max<uint64_t>(1, std::min<uint64_t>(8, (160u << 10) / (lds + 1024)));
        const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(tot, per_cu * (uint64_t)cus));
        hipLaunchKernelGGL(f, dim3(grid), dim3(threads), lds, s, q, counter);
        STN_HIP(hipGetLastError());
    }
}

// loads this file's device code (the runtime does so at the first use of
// one of its kernels)
void warm_code_sv_lds() {
    hipFuncAttributes a{};
    (void)hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_sv_lds<float, 256>));
}

}  // namespace stn
