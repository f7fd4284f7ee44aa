// Lightcone tensor-network contraction (Sec. III-A bucket elimination,
// batched over trajectories as Sec. III-G's ensemble).
//
// One workgroup contracts one (term, trajectory) network entirely in LDS:
// the steps planned by lightcone.cpp run in order; a step computes, for every
// index o of its output, sum_x prod_i T_i[index_i(o, x)] over the summed
// variable x, where each input's index gathers its variables' bits from
// (o, x).  Gate tensors are read from a host table holding both sign variants
// of every gate (binary64, rounded once to the contraction precision) and
// picked by the trajectory's sign bit; the bra side takes the conjugate.  The
// result of a term is <Z_u Z_v> of the trajectory's noiseless-structure state;
// k_tn_energy forms sum_t w_t (1 - f_t <Z_u Z_v>_t) / 2 in binary64 with the
// final Pauli frame's sign f_t, in term order.
#include <cmath>

#include "lightcone.h"

namespace stn {

namespace {

constexpr int kMaxPos = 24;              // largest step input rank (HBM tier)
constexpr int kLdsBytes = 64 * 1024;     // LDS tier: the whole arena in LDS
constexpr uint32_t kMaxSliceBits = 16;   // at most 2^16 slices of one term

// An input's local index from the step index: its bits come in runs of
// consecutive positions, loc |= ((full >> src) & (2^len - 1)) << dst.
struct TnIn {
    int32_t kind, gate, conj, arena, nrun, snrun;
    uint8_t src[kMaxPos], dst[kMaxPos], len[kMaxPos];
    uint8_t ssrc[4], sdst[4], slen[4];   // runs taken from the slice index (sliced variables)
};

struct TnStep {
    int32_t in_off, n_in, out_bits, sum, out_arena;
};

struct TnTerm {
    int32_t step_off, n_steps, result;
};

// one slice of one term's network: the work items are (slice, trajectory)
struct TnSlice {
    int32_t term;
    uint32_t slice;
};

template <class R> struct Cx;
template <> struct Cx<float> { using T = float2; };
template <> struct Cx<double> { using T = double2; };

template <class V> __device__ __forceinline__ V cmul(V a, V b) {
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

// The steps of term t for trajectory b with intermediates in `arena` (LDS or
// this workgroup's slice of global memory).  Each output element of a step
// is one thread's sum over the eliminated variable, so the result does not
// depend on the workgroup size.  __syncthreads() orders the steps (its
// workgroup-scope fences cover global memory too).
template <class R, int kTnThreads>
__device__ __forceinline__ double run_term(typename Cx<R>::T* arena, const TnTerm tm,
                                           const TnStep* __restrict__ steps, const TnIn* __restrict__ ins,
                                           const typename Cx<R>::T* __restrict__ gtab, const uint32_t* sg,
                                           uint32_t slice) {
    using V = typename Cx<R>::T;
    for (int s = 0; s < tm.n_steps; ++s) {
        const TnStep st = steps[tm.step_off + s];
        const uint32_t nout = 1u << st.out_bits;
        for (uint32_t o = threadIdx.x; o < nout; o += kTnThreads) {
            V acc;
            acc.x = R(0);
            acc.y = R(0);
            for (int x = 0; x <= st.sum; ++x) {
                const uint32_t full = o | ((uint32_t)x << st.out_bits);
                V prod;
                prod.x = R(1);
                prod.y = R(0);
                for (int i = 0; i < st.n_in; ++i) {
                    const TnIn& in = ins[st.in_off + i];
                    uint32_t loc = 0;
                    for (int r = 0; r < in.nrun; ++r)
                        loc |= ((full >> in.src[r]) & ((1u << in.len[r]) - 1u)) << in.dst[r];
                    for (int r = 0; r < in.snrun; ++r)
                        loc |= ((slice >> in.ssrc[r]) & ((1u << in.slen[r]) - 1u)) << in.sdst[r];
                    V val;
                    if (in.kind == TN_INTER) {
                        val = arena[in.arena + loc];
                    } else if (in.kind == TN_GATE) {
                        const uint32_t neg = (sg[in.gate >> 5] >> (in.gate & 31)) & 1u;
                        val = gtab[((size_t)in.gate * 2 + neg) * 16 + loc];
                        if (in.conj) val.y = -val.y;
                    } else if (in.kind == TN_OBS) {
                        val.x = ((loc ^ (loc >> 1)) & 1u) ? R(-1) : R(1);
                        val.y = R(0);
                    } else {
                        val.x = loc == 0 ? R(1) : R(0);
                        val.y = R(0);
                    }
                    prod = cmul(prod, val);
                }
                acc.x += prod.x;
                acc.y += prod.y;
            }
            arena[st.out_arena + o] = acc;
        }
        __syncthreads();
    }
    const double r = (double)arena[tm.result].x;
    __syncthreads();   // the arena is reused by the next work item
    return r;
}

// LDS tier: one workgroup per (slice of a term, trajectory), the arena in LDS.
template <class R, int kTnThreads>
__global__ __launch_bounds__(kTnThreads) void k_tn(const TnTerm* __restrict__ terms, const TnStep* __restrict__ steps,
                                                   const TnIn* __restrict__ ins,
                                                   const typename Cx<R>::T* __restrict__ gtab,
                                                   const uint32_t* __restrict__ signs, uint32_t words,
                                                   double* __restrict__ zz, const TnSlice* __restrict__ slices,
                                                   uint32_t F) {
    using V = typename Cx<R>::T;
    extern __shared__ char smem[];
    const uint32_t f = blockIdx.x, b = blockIdx.y;
    const TnSlice sl = slices[f];
    const double r = run_term<R, kTnThreads>(reinterpret_cast<V*>(smem), terms[sl.term], steps, ins, gtab,
                                             signs + (size_t)b * words, sl.slice);
    if (threadIdx.x == 0) zz[(size_t)b * F + f] = r;
}

// HBM tier: persistent workgroups, each with a private arena of `stride`
// slots in global memory, take work items (slice of a term, trajectory) in
// turn.
template <class R, int kTnThreads>
__global__ __launch_bounds__(kTnThreads) void k_tn_hbm(const TnTerm* __restrict__ terms,
                                                       const TnStep* __restrict__ steps,
                                                       const TnIn* __restrict__ ins,
                                                       const typename Cx<R>::T* __restrict__ gtab,
                                                       const uint32_t* __restrict__ signs, uint32_t words,
                                                       double* __restrict__ zz, const TnSlice* __restrict__ slices,
                                                       uint32_t F, uint32_t nb,
                                                       typename Cx<R>::T* __restrict__ garena, uint32_t stride) {
    typename Cx<R>::T* arena = garena + (size_t)blockIdx.x * stride;
    const uint32_t items = F * nb;
    for (uint32_t item = blockIdx.x; item < items; item += gridDim.x) {
        const uint32_t f = item % F, b = item / F;
        const TnSlice sl = slices[f];
        const double r = run_term<R, kTnThreads>(arena, terms[sl.term], steps, ins, gtab,
                                                 signs + (size_t)b * words, sl.slice);
        if (threadIdx.x == 0) zz[(size_t)b * F + f] = r;
    }
}

// energy[b] = sum_t w_t (1 - f_t zz_t) / 2, f_t = (-1)^(F_x[u] xor F_x[v]),
// zz_t = the sum of term t's slices zz[b][toff[t] .. toff[t+1]) in order
__global__ __launch_bounds__(64) void k_tn_energy(const double* __restrict__ zz, uint32_t T,
                                                  const uint32_t* __restrict__ toff, uint32_t F,
                                                  const uint32_t* __restrict__ uv, const double* __restrict__ w,
                                                  const uint64_t* __restrict__ frame, uint32_t B,
                                                  double* __restrict__ energy) {
    const uint32_t b = blockIdx.x * 64 + threadIdx.x;
    if (b >= B) return;
    const uint64_t fx = frame[2 * (size_t)b];
    double e = 0.0;
    for (uint32_t t = 0; t < T; ++t) {
        double z = 0.0;
        for (uint32_t f = toff[t]; f < toff[t + 1]; ++f) z += zz[(size_t)b * F + f];
        const double sg = (((fx >> uv[2 * t]) ^ (fx >> uv[2 * t + 1])) & 1ull) ? -1.0 : 1.0;
        e += w[t] * (1.0 - sg * z) * 0.5;
    }
    energy[b] = e;
}

template <class R>
using TnFn = void (*)(const TnTerm*, const TnStep*, const TnIn*, const typename Cx<R>::T*, const uint32_t*,
                      uint32_t, double*, const TnSlice*, uint32_t);

struct TnKernel {
    void* f;
    uint32_t threads;
};

// launch shapes the autotuner chooses from (variant 0 is the default)
constexpr uint32_t kTnVariants = 3;
template <class R>
TnKernel tn_kernel(uint32_t v) {
    switch (v) {
        case 1: return {(void*)k_tn<R, 64>, 64};
        case 2: return {(void*)k_tn<R, 128>, 128};
        default: return {(void*)k_tn<R, 256>, 256};
    }
}

template <class R>
using TnHbmFn = void (*)(const TnTerm*, const TnStep*, const TnIn*, const typename Cx<R>::T*, const uint32_t*,
                         uint32_t, double*, const TnSlice*, uint32_t, uint32_t, typename Cx<R>::T*, uint32_t);

// one persistent workgroup per free CU: the default is the widest
template <class R>
TnKernel tn_hbm_kernel(uint32_t v) {
    switch (v) {
        case 1: return {(void*)k_tn_hbm<R, 256>, 256};
        case 2: return {(void*)k_tn_hbm<R, 512>, 512};
        default: return {(void*)k_tn_hbm<R, 1024>, 1024};
    }
}

struct TnDevice {
    std::vector<TnNetwork> nets;
    int arena = 0;
    bool hbm = false;           // intermediates in global memory (persistent workgroups)
    uint32_t stride = 0;        // HBM tier: arena slots per workgroup
    uint32_t grid = 0;          // HBM tier: persistent workgroups
    uint32_t F = 0;             // slices of all terms (work items per trajectory)
    DevBuf terms, steps, ins, gtab32, gtab64, zz, garena, slices, toff;
};

// tensor values of gate g over its local index, for sign s (0: theta, 1: -theta)
void gate_tensor(const GateRec& g, int s, cd* out) {
    for (int i = 0; i < 16; ++i) out[i] = 0;
    const double th = s ? -g.theta : g.theta;
    const cd I1(0, 1);
    std::vector<cd> m;
    const double c = std::cos(th / 2), sn = std::sin(th / 2);
    switch (g.kind) {
        case STN_G_RX: m = {c, -I1 * sn, -I1 * sn, c}; break;
        case STN_G_RY: m = {c, -sn, sn, c}; break;
        case STN_G_RZ: m = {std::exp(-I1 * (th / 2)), 0, 0, std::exp(I1 * (th / 2))}; break;
        case STN_G_ZZ: {
            const cd e = std::exp(-I1 * th);
            m.assign(16, 0);
            m[0] = 1; m[5] = e; m[10] = e; m[15] = 1;
            break;
        }
        default: m = g.m; break;
    }
    const bool diag = g.kind == STN_G_RZ || g.kind == STN_G_Z || g.kind == STN_G_ZZ;
    if (g.nq == 1) {
        if (diag) {
            out[0] = m[0];
            out[1] = m[3];
        } else {
            // local index: bit 0 = input, bit 1 = output
            for (int in = 0; in < 2; ++in)
                for (int o = 0; o < 2; ++o) out[in | (o << 1)] = m[o * 2 + in];
        }
    } else {
        if (diag) {
            for (int l = 0; l < 4; ++l) out[l] = m[l * 4 + l];
        } else {
            // local index: in0, in1, out0, out1
            for (int in = 0; in < 4; ++in)
                for (int o = 0; o < 4; ++o) out[in | (o << 2)] = m[o * 4 + in];
        }
    }
}

}  // namespace

// Builds the networks of every observable term; records width and cost.
void build_lightcone(stn_plan* p) {
    if (!p->frame_ok) fail(STN_E_UNSUPPORTED, "lightcone lowering needs Pauli noise and Pauli-rotation gates after the noise");
    if (p->obs_u.empty()) fail(STN_E_UNSUPPORTED, "lightcone lowering needs an observable");
    auto* d = new TnDevice();
    p->lc = d;
    p->lc_free = [](void* v) { delete static_cast<TnDevice*>(v); };
    const size_t elem = p->opts.precision == 128 ? 16 : 8;
    double cost = 0;
    int width = 0;
    int max_rank = 0;
    bool aborted = false;
    const int rank_cap = p->opts.lc_max_rank ? std::min<int>((int)p->opts.lc_max_rank, kMaxPos - 1) : kMaxPos - 1;
    const int slice_cap = (int)std::min<uint32_t>(p->opts.lc_slice_bits, kMaxSliceBits);
    for (size_t t = 0; t < p->obs_u.size(); ++t) {
        d->nets.push_back(build_term(p, (uint32_t)t, p->obs_u[t], p->obs_v[t], p->opts.order_restarts,
                                     p->opts.order_seed, rank_cap, slice_cap));
        const TnNetwork& net = d->nets.back();
        if (net.steps.empty() && !std::isfinite(net.cost)) {
            max_rank = std::max(max_rank, net.width);   // stopped early: too wide for this lowering
            width = std::max(width, net.width);
            cost = HUGE_VAL;
            aborted = true;
            break;
        }
        for (auto& st : net.steps)
            for (auto& in : st.inputs) max_rank = std::max(max_rank, (int)in.pos.size());
        d->arena = std::max(d->arena, net.arena);
        width = std::max(width, net.width);
        cost += net.cost;
    }
    // the networks' size is known even where this lowering cannot run them
    p->lc_width = (uint32_t)width;
    p->lc_flops_per_traj = 8.0 * cost;
    if (aborted || max_rank > kMaxPos)
        fail(STN_E_UNSUPPORTED, "lightcone step rank above " + std::to_string(rank_cap + 1) + " (width " +
                                    std::to_string(width) + (slice_cap ? ", after slicing " + std::to_string(slice_cap) +
                                    " variables" : "") + ")");
    p->width = (uint32_t)width;
    size_t steps = 0;
    double inter_bytes = 0;   // intermediates read and written per trajectory
    for (auto& net : d->nets) {
        steps += net.steps.size();
        for (auto& st : net.steps) {
            inter_bytes += std::ldexp((double)elem, (int)st.out_vars.size() + net.slice_bits);
            for (auto& in : st.inputs)
                if (in.kind == TN_INTER) inter_bytes += std::ldexp((double)elem, (int)in.pos.size() + net.slice_bits);
        }
    }
    p->n_steps = (uint32_t)steps;
    uint64_t F = 0;
    int sb = 0;
    for (auto& net : d->nets) {
        F += 1ull << net.slice_bits;
        sb = std::max(sb, net.slice_bits);
    }
    if (F > (1u << 20)) fail(STN_E_UNSUPPORTED, "more than 2^20 lightcone slices");
    d->F = (uint32_t)F;
    p->lc_slices = (uint32_t)F;
    p->lc_slice_bits = (uint32_t)sb;
    p->flops_per_traj = 8.0 * cost;             // one complex multiply-add per input per index
    if ((size_t)d->arena * elem <= (size_t)kLdsBytes) {
        d->hbm = false;
        p->bytes_per_traj = 8.0 * F;                // per-slice result; everything else stays in LDS
        p->lc_est_s = p->flops_per_traj / 8e12;
    } else {
        // HBM tier: persistent workgroups with private arenas within the budget
        d->hbm = true;
        d->stride = (uint32_t)((d->arena + 63) / 64 * 64);
        const double budget = p->opts.hbm_budget ? (double)p->opts.hbm_budget : 64.0 * (1ull << 30);
        const double per_wg = (double)d->stride * elem;
        d->grid = (uint32_t)std::min(512.0, std::floor(budget / 2 / per_wg));
        if (d->grid < 32) fail(STN_E_UNSUPPORTED, "lightcone intermediates exceed the memory budget (width " +
                                                      std::to_string(width) + ")");
        p->bytes_per_traj = inter_bytes + 8.0 * F;
        p->lc_est_s = inter_bytes / 1.5e12 + p->flops_per_traj / 4e12;
        p->lc_arena_bytes = (double)d->grid * per_wg;
    }
}

void upload_lightcone(stn_plan* p, hipStream_t s) {
    auto* d = static_cast<TnDevice*>(p->lc);
    std::vector<TnTerm> terms;
    std::vector<TnStep> steps;
    std::vector<TnIn> ins;
    std::vector<TnSlice> slices;
    std::vector<uint32_t> toff;
    for (auto& net : d->nets) {
        toff.push_back((uint32_t)slices.size());
        for (uint32_t sl = 0; sl < (1u << net.slice_bits); ++sl) slices.push_back({(int32_t)terms.size(), sl});
        TnTerm tm{(int32_t)steps.size(), (int32_t)net.steps.size(), net.result};
        for (auto& st : net.steps) {
            TnStep ds{(int32_t)ins.size(), (int32_t)st.inputs.size(), (int32_t)st.out_vars.size(),
                      st.elim >= 0 ? 1 : 0, st.out_arena};
            for (auto& in : st.inputs) {
                TnIn di{};
                di.kind = in.kind;
                di.gate = in.gate;
                di.conj = in.conj;
                di.arena = in.arena;
                di.nrun = 0;
                di.snrun = 0;
                // runs of local bits whose source bits (step index, or slice
                // index for negative positions) are consecutive too
                for (size_t k = 0; k < in.pos.size();) {
                    const bool sl = in.pos[k] < 0;
                    const int src = sl ? -1 - in.pos[k] : in.pos[k];
                    size_t e = k + 1;
                    while (e < in.pos.size() && (in.pos[e] < 0) == sl &&
                           (sl ? -1 - in.pos[e] : in.pos[e]) == src + (int)(e - k))
                        ++e;
                    if (sl) {
                        if (di.snrun >= 4) fail(STN_E_INVALID, "too many sliced runs in one input");
                        di.ssrc[di.snrun] = (uint8_t)src;
                        di.sdst[di.snrun] = (uint8_t)k;
                        di.slen[di.snrun] = (uint8_t)(e - k);
                        di.snrun++;
                    } else {
                        di.src[di.nrun] = (uint8_t)src;
                        di.dst[di.nrun] = (uint8_t)k;
                        di.len[di.nrun] = (uint8_t)(e - k);
                        di.nrun++;
                    }
                    k = e;
                }
                ins.push_back(di);
            }
            steps.push_back(ds);
        }
        terms.push_back(tm);
    }
    toff.push_back((uint32_t)slices.size());
    if (ins.empty()) ins.push_back(TnIn{});
    std::vector<float2> g32(p->gates.size() * 32 + 1);
    std::vector<double2> g64(p->gates.size() * 32 + 1);
    for (size_t g = 0; g < p->gates.size(); ++g)
        for (int sgn = 0; sgn < 2; ++sgn) {
            cd vals[16];
            gate_tensor(p->gates[g], sgn, vals);
            for (int l = 0; l < 16; ++l) {
                g32[(g * 2 + sgn) * 16 + l] = make_float2((float)vals[l].real(), (float)vals[l].imag());
                g64[(g * 2 + sgn) * 16 + l] = make_double2(vals[l].real(), vals[l].imag());
            }
        }
    upload(d->terms, &p->alloc, terms.data(), terms.size() * sizeof(TnTerm), s);
    upload(d->steps, &p->alloc, steps.data(), steps.size() * sizeof(TnStep), s);
    upload(d->ins, &p->alloc, ins.data(), ins.size() * sizeof(TnIn), s);
    upload(d->gtab32, &p->alloc, g32.data(), g32.size() * sizeof(float2), s);
    upload(d->gtab64, &p->alloc, g64.data(), g64.size() * sizeof(double2), s);
    upload(d->slices, &p->alloc, slices.data(), slices.size() * sizeof(TnSlice), s);
    upload(d->toff, &p->alloc, toff.data(), toff.size() * sizeof(uint32_t), s);
}

void launch_lightcone(stn_plan* p, stn_batch* b, hipStream_t s) {
    auto* d = static_cast<TnDevice*>(p->lc);
    const uint32_t T = (uint32_t)d->nets.size();
    const uint32_t F = d->F;
    const bool dbl = p->opts.precision == 128;
    const size_t elem = dbl ? 16 : 8;
    const size_t lds = (size_t)d->arena * elem;
    const uint32_t B = std::min<uint32_t>(b->K, 65535);
    d->zz.ensure(&p->alloc, (size_t)B * F * 8);
    const uint32_t v = std::min<uint32_t>(p->variant, kTnVariants - 1);
    const TnKernel ker = d->hbm ? (dbl ? tn_hbm_kernel<double>(v) : tn_hbm_kernel<float>(v))
                                : (dbl ? tn_kernel<double>(v) : tn_kernel<float>(v));
    static bool attr[2][kTnVariants] = {};
    if (!d->hbm && !attr[dbl][v]) {
        STN_HIP(hipFuncSetAttribute(ker.f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes));
        attr[dbl][v] = true;
    }
    if (d->hbm) d->garena.ensure(&p->alloc, (size_t)d->grid * d->stride * elem);
    double cost = 0;
    for (auto& net : d->nets) cost += net.cost;
    for (uint32_t c0 = 0; c0 < b->K; c0 += B) {
        const uint32_t nb = std::min(B, b->K - c0);
        const uint32_t* sg = b->d_signs.as<uint32_t>() + (size_t)c0 * b->words;
        prof_begin(p, STN_K_TN_STEP, s);
        if (d->hbm) {
            // a job server may keep some CUs free for other jobs' kernels
            uint32_t grid = (uint32_t)std::min<uint64_t>(d->grid, (uint64_t)F * nb);
            if (p->grid_cap) grid = std::min(grid, p->grid_cap);
            if (dbl)
                hipLaunchKernelGGL(reinterpret_cast<TnHbmFn<double>>(ker.f), dim3(grid), dim3(ker.threads), 0, s,
                                   d->terms.as<TnTerm>(), d->steps.as<TnStep>(), d->ins.as<TnIn>(),
                                   d->gtab64.as<double2>(), sg, b->words, d->zz.as<double>(),
                                   d->slices.as<TnSlice>(), F, nb, d->garena.as<double2>(), d->stride);
            else
                hipLaunchKernelGGL(reinterpret_cast<TnHbmFn<float>>(ker.f), dim3(grid), dim3(ker.threads), 0, s,
                                   d->terms.as<TnTerm>(), d->steps.as<TnStep>(), d->ins.as<TnIn>(),
                                   d->gtab32.as<float2>(), sg, b->words, d->zz.as<double>(),
                                   d->slices.as<TnSlice>(), F, nb, d->garena.as<float2>(), d->stride);
        } else if (dbl) {
            hipLaunchKernelGGL(reinterpret_cast<TnFn<double>>(ker.f), dim3(F, nb), dim3(ker.threads), lds, s,
                               d->terms.as<TnTerm>(), d->steps.as<TnStep>(), d->ins.as<TnIn>(),
                               d->gtab64.as<double2>(), sg, b->words, d->zz.as<double>(), d->slices.as<TnSlice>(), F);
        } else {
            hipLaunchKernelGGL(reinterpret_cast<TnFn<float>>(ker.f), dim3(F, nb), dim3(ker.threads), lds, s,
                               d->terms.as<TnTerm>(), d->steps.as<TnStep>(), d->ins.as<TnIn>(),
                               d->gtab32.as<float2>(), sg, b->words, d->zz.as<double>(), d->slices.as<TnSlice>(), F);
        }
        STN_HIP(hipGetLastError());
        prof_end(p, STN_K_TN_STEP, s, (double)nb * p->bytes_per_traj, (double)nb * 8.0 * cost);
        hipLaunchKernelGGL(k_tn_energy, dim3((nb + 63) / 64), dim3(64), 0, s, d->zz.as<double>(), T,
                           d->toff.as<uint32_t>(), F, p->d_obs.as<uint32_t>(), p->d_obs_w.as<double>(),
                           b->d_frame.as<uint64_t>() + 2 * (size_t)c0, nb, b->d_energy.as<double>() + c0);
        STN_HIP(hipGetLastError());
    }
}

uint32_t tn_variants() { return kTnVariants; }

}  // namespace stn
