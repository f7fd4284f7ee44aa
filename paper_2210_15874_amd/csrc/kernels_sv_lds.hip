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
#include "stn_internal.h"

namespace stn {

namespace {

template <class R> struct Cx;
template <> struct Cx<float> { using T = float2; };
template <> struct Cx<double> { using T = double2; };

template <class V> __device__ __forceinline__ V cmul(V a, V b) {
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <class V> __device__ __forceinline__ V cadd(V a, V b) {
    a.x += b.x;
    a.y += b.y;
    return a;
}
template <class V> __device__ __forceinline__ V cneg_if(V a, bool neg) {
    if (neg) { a.x = -a.x; a.y = -a.y; }
    return a;
}

// index with a zero bit inserted at position q
__device__ __forceinline__ uint32_t ins0(uint32_t p, uint32_t q) {
    const uint32_t lo = p & ((1u << q) - 1u);
    return ((p ^ lo) << 1) | lo;
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
    V* psi = reinterpret_cast<V*>(smem_raw);
    const uint32_t b = blockIdx.x;
    const uint32_t tid = threadIdx.x;
    const uint32_t N = 1u << n;
    for (uint32_t i = tid; i < N; i += kThreads) {
        V v;
        v.x = i == 0 ? R(1) : R(0);
        v.y = R(0);
        psi[i] = v;
    }
    __syncthreads();
    const uint8_t* row = idx + (size_t)b * S;
    for (uint32_t oi = 0; oi < n_ops; ++oi) {
        LdsOp o = ops[oi];
        if (o.kind == OP_SITE) o = site_ops[site_off[o.site] + row[o.site]];
        switch (o.kind) {
            case OP_DENSE1: {
                const V m0 = vals[o.mat], m1 = vals[o.mat + 1], m2 = vals[o.mat + 2], m3 = vals[o.mat + 3];
                const uint32_t bit = 1u << o.q0;
                for (uint32_t p = tid; p < N / 2; p += kThreads) {
                    const uint32_t i0 = ins0(p, o.q0), i1 = i0 | bit;
                    const V a = psi[i0], c = psi[i1];
                    psi[i0] = cadd(cmul(m0, a), cmul(m1, c));
                    psi[i1] = cadd(cmul(m2, a), cmul(m3, c));
                }
                break;
            }
            case OP_DENSE2: {
                const uint32_t qa = o.q0 < o.q1 ? o.q0 : o.q1, qb = o.q0 < o.q1 ? o.q1 : o.q0;
                const uint32_t b0 = 1u << o.q0, b1 = 1u << o.q1;
                for (uint32_t p = tid; p < N / 4; p += kThreads) {
                    const uint32_t i = ins0(ins0(p, qa), qb);
                    const uint32_t ix[4] = {i, i | b0, i | b1, i | b0 | b1};
                    V v[4];
#pragma unroll
                    for (int l = 0; l < 4; ++l) v[l] = psi[ix[l]];
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        V acc = cmul(vals[o.mat + 4 * l], v[0]);
#pragma unroll
                        for (int m = 1; m < 4; ++m) acc = cadd(acc, cmul(vals[o.mat + 4 * l + m], v[m]));
                        psi[ix[l]] = acc;
                    }
                }
                break;
            }
            case OP_DIAG1: {
                const V d0 = vals[o.mat], d1 = vals[o.mat + 1];
                for (uint32_t i = tid; i < N; i += kThreads) psi[i] = cmul((i >> o.q0) & 1 ? d1 : d0, psi[i]);
                break;
            }
            case OP_DIAG2: {
                V d[4];
#pragma unroll
                for (int l = 0; l < 4; ++l) d[l] = vals[o.mat + l];
                for (uint32_t i = tid; i < N; i += kThreads)
                    psi[i] = cmul(d[((i >> o.q0) & 1) | (((i >> o.q1) & 1) << 1)], psi[i]);
                break;
            }
            case OP_PAULI: {
                const uint32_t x = (uint32_t)o.xmask, z = (uint32_t)o.zmask;
                if (x == 0) {
                    for (uint32_t i = tid; i < N; i += kThreads) psi[i] = cneg_if(psi[i], __popc(i & z) & 1);
                } else {
                    const uint32_t lb = __ffs(x) - 1;
                    for (uint32_t p = tid; p < N / 2; p += kThreads) {
                        const uint32_t i = ins0(p, lb), j = i ^ x;
                        const V a = psi[i], c = psi[j];
                        psi[j] = cneg_if(a, __popc(i & z) & 1);
                        psi[i] = cneg_if(c, __popc(j & z) & 1);
                    }
                }
                break;
            }
            default: break;  // identity
        }
        __syncthreads();
    }
    // energy <psi|C|psi> in binary64: per-amplitude terms, then a fixed tree
    if (states)
        for (uint32_t i = tid; i < N; i += kThreads) states[(size_t)b * N + i] = psi[i];
    double* e = reinterpret_cast<double*>(smem_raw) + (sizeof(V) == 8 ? 0 : 2 * (size_t)N);
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
    if (tid == 0) energy[b] = e[0];
}

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

}  // namespace stn
