// Lightcone tensor-network contraction (Sec. III-A bucket elimination,
// batched over trajectories as Sec. III-G's ensemble).
//
// A work item is one (slice of a term's network, trajectory); persistent
// workgroups take items in turn and run the term's steps in order.  A step
// computes, for every index o of its output, sum_x prod_i T_i[index_i(o, x)]
// over the summed variable x.  Gate tensors come from a host table holding
// both sign variants of every gate (binary64, rounded once to the
// contraction precision), picked by the trajectory's sign bit; the bra side
// takes the conjugate.  Intermediates live in an LDS arena when they are
// small and in the workgroup's global-memory arena otherwise.
//
// Per step, a workgroup first multiplies the step's small factors (gate
// tensors, the observable, |0>, rank <= 2 intermediates) into one table over
// the step bits they use (at most 2^10 entries, in LDS); every output element
// then reads that table and its larger inputs once per value of x.  An
// input's local index is a bit selection of the step index, so it splits into
// a per-thread part (the low step bits, fixed for the whole step) and a
// uniform part for the higher bits, which the element loop visits in Gray
// code order: each iteration flips one step bit and so one local bit of each
// input.  Each output element is one thread's sum, in a fixed order that
// does not depend on the launch shape.  The result of a term is <Z_u Z_v> of
// the trajectory's noiseless-structure state; k_tn_energy forms
// sum_t w_t (1 - f_t <Z_u Z_v>_t) / 2 in binary64 with the final Pauli
// frame's sign f_t, in term order.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <exception>
#include <mutex>
#include <thread>

#include "lightcone.h"

namespace stn {

namespace {

constexpr int kStepBits = 24;            // output variables + the summed one (rank cap 23)
constexpr int kMaxMain = 6;              // inputs read per output element
constexpr int kTabBits = 10;             // small-factor table: at most 2^10 entries
constexpr int kLdsArenaBytes = 64 * 1024;   // intermediates in LDS
constexpr uint32_t kMaxSliceBits = 16;   // at most 2^16 slices of one term

// An input read per output element: its local index is the OR over the step
// (and slice) index bits that are set of bit[b] (sbit[b]).
struct TnMain {
    int32_t kind, gate, conj, off, lds, pad;
    uint32_t bit[kStepBits];
    uint32_t sbit[kMaxSliceBits];
};

// A factor of the step's table: its local index is the OR over the table
// (and slice) index bits that are set of tbit[t] (sbit[b]).
struct TnSmall {
    int32_t kind, gate, conj, off, lds, pad;
    uint32_t tbit[kTabBits];
    uint32_t sbit[kMaxSliceBits];
};

struct TnStep {
    int32_t out_bits, nsum, out_off, out_lds;   // nsum: summed variables, step bits out_bits ..
    int32_t main0, n_main, small0, n_small;
    int32_t tab_bits, generic, pad[2];   // generic: a per-element input is not an intermediate
    uint32_t tbit[kStepBits];   // table-index value of each step bit
};

struct TnTerm {
    int32_t step0, n_steps, result, result_lds;
    int32_t slice_bits, pad[3];
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

template <class V> __device__ __forceinline__ V cone() {
    V r;
    r.x = 1;
    r.y = 0;
    return r;
}

// value of an input of any kind at local index loc
template <class V>
__device__ __forceinline__ V tn_value(int kind, int gate, int conj, int off, int lds, uint32_t loc,
                                      const V* lds_arena, const V* garena, const V* __restrict__ gtab,
                                      const uint32_t* sg) {
    V v;
    if (kind == TN_INTER) {
        v = lds ? lds_arena[off + loc] : garena[off + loc];
    } else if (kind == TN_GATE) {
        const uint32_t neg = (sg[gate >> 5] >> (gate & 31)) & 1u;
        v = gtab[((size_t)gate * 2 + neg) * 16 + loc];
        if (conj) v.y = -v.y;
    } else if (kind == TN_OBS) {
        v.x = ((loc ^ (loc >> 1)) & 1u) ? -1 : 1;
        v.y = 0;
    } else {
        v.x = loc == 0 ? 1 : 0;
        v.y = 0;
    }
    return v;
}

// The output elements of a step whose NM per-element inputs are all
// intermediates (src: flat pointers, LDS or global), summing 2^LOGX values
// of its summed variables (xi / xt: each input's and the table's local-index
// offset of every such value).  Output bits below klog are the thread's; the
// loop visits the higher bits in blocks of 2^LOGU iterations: the block
// index in Gray code order (one step bit, so one local bit of each input,
// flips from block to block) and the 2^LOGU low loop bits in every
// combination inside a block, whose loads are all issued before any product
// is formed.
template <class V, int NM, int LOGU, int LOGX>
__device__ __forceinline__ void step_elements(const TnStep& st, const TnMain* __restrict__ mn, const V* tab,
                                              int has_tab, V* out, const V* const (&src)[kMaxMain],
                                              const uint32_t (&li)[kMaxMain], const uint32_t (&xi)[kMaxMain][2],
                                              uint32_t lt, const uint32_t (&xt)[2], uint32_t iters, int klog,
                                              uint32_t olo) {
    constexpr uint32_t U = 1u << LOGU;
    constexpr int X = 1 << LOGX;
    uint32_t fl[LOGU + 1][NM + 1];
#pragma unroll
    for (int k = 0; k < LOGU; ++k) {
#pragma unroll
        for (int i = 0; i < NM; ++i) fl[k][i] = mn[i].bit[klog + k];
        fl[k][NM] = st.tbit[klog + k];
    }
    uint32_t lj[NM + 1];
#pragma unroll
    for (int i = 0; i <= NM; ++i) lj[i] = 0;
    uint32_t oj = 0;
    const uint32_t blocks = iters >> LOGU;
    for (uint32_t m = 0; m < blocks; ++m) {
        if (m) {
            const int b = klog + LOGU + __builtin_ctz(m);
            oj ^= 1u << b;
#pragma unroll
            for (int i = 0; i < NM; ++i) lj[i] ^= mn[i].bit[b];
            lj[NM] ^= st.tbit[b];
        }
        if constexpr (U * X * (NM + 1) > (sizeof(V) > 8 ? 8 : 16)) {
            // too many values to hold at once: one summed value after another
            static_assert(U == 1, "unrolled blocks stay within the register budget");
            V acc;
            acc.x = 0;
            acc.y = 0;
#pragma unroll
            for (int x = 0; x < X; ++x) {
                const uint32_t ox = ((x & 1) ? xt[0] : 0u) ^ ((x & 2) ? xt[1] : 0u);
                V v = has_tab ? tab[lt ^ lj[NM] ^ ox] : cone<V>();
#pragma unroll
                for (int i = 0; i < NM; ++i)
                    v = cmul(v, src[i][li[i] ^ lj[i] ^ ((x & 1) ? xi[i][0] : 0u) ^ ((x & 2) ? xi[i][1] : 0u)]);
                acc.x += v.x;
                acc.y += v.y;
            }
            out[oj | olo] = acc;
            continue;
        }
        V val[U][X][NM > 0 ? NM : 1];
        V tv[U][X];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            uint32_t d[NM + 1];
#pragma unroll
            for (int i = 0; i <= NM; ++i) {
                d[i] = lj[i];
#pragma unroll
                for (int k = 0; k < LOGU; ++k)
                    if ((u >> k) & 1u) d[i] ^= fl[k][i];
            }
#pragma unroll
            for (int x = 0; x < X; ++x) {
                const uint32_t ox = ((x & 1) ? xt[0] : 0u) ^ ((x & 2) ? xt[1] : 0u);
                tv[u][x] = has_tab ? tab[lt ^ d[NM] ^ ox] : cone<V>();
#pragma unroll
                for (int i = 0; i < NM; ++i)
                    val[u][x][i] = src[i][li[i] ^ d[i] ^ ((x & 1) ? xi[i][0] : 0u) ^ ((x & 2) ? xi[i][1] : 0u)];
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            V acc;
            acc.x = 0;
            acc.y = 0;
#pragma unroll
            for (int x = 0; x < X; ++x) {
                V v = tv[u][x];
#pragma unroll
                for (int i = 0; i < NM; ++i) v = cmul(v, val[u][x][i]);
                acc.x += v.x;
                acc.y += v.y;
            }
            out[oj | (u << klog) | olo] = acc;
        }
    }
}

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

// block size of the element loop: more loads in flight when a step reads few
// values per output, bounded by the loop's length (a power of two)
template <class V, int NM, int LOGX>
__device__ __forceinline__ void step_elements_u(const TnStep& st, const TnMain* __restrict__ mn, const V* tab,
                                                int has_tab, V* out, const V* const (&src)[kMaxMain],
                                                const uint32_t (&li)[kMaxMain], const uint32_t (&xi)[kMaxMain][2],
                                                uint32_t lt, const uint32_t (&xt)[2], uint32_t iters, int klog,
                                                uint32_t olo) {
    constexpr int kValues = (sizeof(V) > 8 ? 8 : 16) / ((1 << LOGX) * (NM + 1));
    constexpr int kMaxU = ilog2c(kValues) < 2 ? ilog2c(kValues) : 2;
    const int lg = __builtin_ctz(iters);
    const int u = lg < kMaxU ? lg : kMaxU;
    if (u >= 2 && kMaxU >= 2)
        step_elements<V, NM, (kMaxU >= 2 ? 2 : 0), LOGX>(st, mn, tab, has_tab, out, src, li, xi, lt, xt, iters, klog, olo);
    else if (u == 1 && kMaxU >= 1)
        step_elements<V, NM, (kMaxU >= 1 ? 1 : 0), LOGX>(st, mn, tab, has_tab, out, src, li, xi, lt, xt, iters, klog, olo);
    else
        step_elements<V, NM, 0, LOGX>(st, mn, tab, has_tab, out, src, li, xi, lt, xt, iters, klog, olo);
}

template <class V, int NM>
__device__ __forceinline__ void step_elements_any(const TnStep& st, const TnMain* __restrict__ mn, const V* tab,
                                                  int has_tab, V* out, const V* const (&src)[kMaxMain],
                                                  const uint32_t (&li)[kMaxMain], const uint32_t (&xi)[kMaxMain][2],
                                                  uint32_t lt, const uint32_t (&xt)[2], int nsum, uint32_t iters,
                                                  int klog, uint32_t olo, bool wide) {
    // (complex128 plans are lowered without merged steps: nsum <= 1)
    constexpr int kX = sizeof(V) > 8 ? 1 : 2;
    if (wide) {
        if (nsum >= 2) step_elements_u<V, NM, kX>(st, mn, tab, has_tab, out, src, li, xi, lt, xt, iters, klog, olo);
        else step_elements_u<V, NM, 1>(st, mn, tab, has_tab, out, src, li, xi, lt, xt, iters, klog, olo);
    } else {
        if (nsum >= 2) step_elements<V, NM, 0, kX>(st, mn, tab, has_tab, out, src, li, xi, lt, xt, 1u, klog, olo);
        else if (nsum == 1) step_elements<V, NM, 0, 1>(st, mn, tab, has_tab, out, src, li, xi, lt, xt, 1u, klog, olo);
        else step_elements<V, NM, 0, 0>(st, mn, tab, has_tab, out, src, li, xi, lt, xt, 1u, klog, olo);
    }
}

// The element loop of one step for one trajectory of the group: pointers to
// that trajectory's arenas, table and output.
// (WIDE: the step has at least as many outputs as threads, the pointers are
// the same for the whole workgroup and the loop is unrolled; otherwise each
// thread computes one output of its own trajectory)
template <class V, bool WIDE>
__device__ __forceinline__ void step_item(const TnStep& st, const TnMain* __restrict__ mn, int n_main, int n_small,
                                          const V* tab, V* lds, V* ga, const V* __restrict__ gtab,
                                          const uint32_t* sg, const uint32_t (&li)[kMaxMain],
                                          const uint32_t (&xi)[kMaxMain][2], uint32_t lt, const uint32_t (&xt)[2],
                                          int nsum, uint32_t iters, int klog, uint32_t olo) {
    V* out = st.out_lds ? lds + st.out_off : ga + st.out_off;
    if (!st.generic) {
        const V* src[kMaxMain];
#pragma unroll
        for (int i = 0; i < kMaxMain; ++i) {
            src[i] = lds;
            if (i < n_main) src[i] = mn[i].lds ? (const V*)lds + mn[i].off : (const V*)ga + mn[i].off;
        }
        switch (n_main) {
            case 0: step_elements_any<V, 0>(st, mn, tab, n_small, out, src, li, xi, lt, xt, nsum, iters, klog, olo, WIDE); break;
            case 1: step_elements_any<V, 1>(st, mn, tab, n_small, out, src, li, xi, lt, xt, nsum, iters, klog, olo, WIDE); break;
            case 2: step_elements_any<V, 2>(st, mn, tab, n_small, out, src, li, xi, lt, xt, nsum, iters, klog, olo, WIDE); break;
            case 3: step_elements_any<V, 3>(st, mn, tab, n_small, out, src, li, xi, lt, xt, nsum, iters, klog, olo, WIDE); break;
            case 4: step_elements_any<V, 4>(st, mn, tab, n_small, out, src, li, xi, lt, xt, nsum, iters, klog, olo, WIDE); break;
            case 5: step_elements_any<V, 5>(st, mn, tab, n_small, out, src, li, xi, lt, xt, nsum, iters, klog, olo, WIDE); break;
            default: step_elements_any<V, 6>(st, mn, tab, n_small, out, src, li, xi, lt, xt, nsum, iters, klog, olo, WIDE); break;
        }
        return;
    }
    // some per-element input is not an intermediate: every value through tn_value
    uint32_t oj = 0, ljt = 0;
    uint32_t lj[kMaxMain];
#pragma unroll
    for (int i = 0; i < kMaxMain; ++i) lj[i] = 0;
    for (uint32_t j = 0; j < iters; ++j) {
        if (j) {
            const int b = klog + __builtin_ctz(j);
            oj ^= 1u << b;
            ljt ^= st.tbit[b];
            for (int i = 0; i < n_main; ++i) lj[i] ^= mn[i].bit[b];
        }
        V acc;
        acc.x = 0;
        acc.y = 0;
        for (int x = 0; x < (1 << nsum); ++x) {
            V v = n_small ? tab[lt ^ ljt ^ ((x & 1) ? xt[0] : 0u) ^ ((x & 2) ? xt[1] : 0u)] : cone<V>();
            for (int i = 0; i < n_main; ++i)
                v = cmul(v, tn_value<V>(mn[i].kind, mn[i].gate, mn[i].conj, mn[i].off, mn[i].lds,
                                        li[i] ^ lj[i] ^ ((x & 1) ? xi[i][0] : 0u) ^ ((x & 2) ? xi[i][1] : 0u), lds,
                                        ga, gtab, sg));
            acc.x += v.x;
            acc.y += v.y;
        }
        out[oj | olo] = acc;
    }
}

// The steps of one work item: ng trajectories (the group's valid ones) of
// one slice of one term, in lockstep.  Trajectory t of the group has the LDS
// arena lds + t lds_item, the table tabs + t tab_item and the global-memory
// arena ga + t g_item.  Steps with at least as many outputs as threads run
// the trajectories one after another; smaller steps run several side by
// side (thread = trajectory slot, output index).  __syncthreads() orders the
// steps (its workgroup-scope fences cover global memory too).
template <class R>
__device__ __forceinline__ void run_group(typename Cx<R>::T* lds, typename Cx<R>::T* tabs, typename Cx<R>::T* ga,
                                          const TnTerm tm, const TnStep* __restrict__ steps,
                                          const TnMain* __restrict__ mains, const TnSmall* __restrict__ smalls,
                                          const typename Cx<R>::T* __restrict__ gtab, const uint32_t* signs,
                                          uint32_t words, uint32_t slice, uint32_t ng, uint32_t lds_item,
                                          uint32_t tab_item, uint32_t g_item, double* zz, uint32_t F) {
    using V = typename Cx<R>::T;
    const uint32_t nthreads = blockDim.x;
    const int klog = __builtin_ctz(nthreads);
    const uint32_t tid = threadIdx.x;
    for (int s = 0; s < tm.n_steps; ++s) {
        const TnStep& st = steps[tm.step0 + s];
        const int out_bits = st.out_bits, nsum = st.nsum, n_main = st.n_main, n_small = st.n_small;
        const TnMain* __restrict__ mn = mains + st.main0;
        // 1. the small factors' product table of every trajectory
        if (n_small) {
            const int tb = st.tab_bits;
            const uint32_t total = ng << tb;
            for (uint32_t e = tid; e < total; e += nthreads) {
                const uint32_t t = e >> tb, j = e & ((1u << tb) - 1u);
                V* la = lds + t * lds_item;
                V* gat = ga ? ga + (size_t)t * g_item : ga;
                const uint32_t* sg = signs + (size_t)t * words;
                V v = cone<V>();
                for (int f = 0; f < n_small; ++f) {
                    const TnSmall& sm = smalls[st.small0 + f];
                    uint32_t loc = 0;
                    for (int q = 0; q < tb; ++q)
                        if ((j >> q) & 1u) loc |= sm.tbit[q];
                    for (int b = 0; b < tm.slice_bits; ++b)
                        if ((slice >> b) & 1u) loc |= sm.sbit[b];
                    v = cmul(v, tn_value<V>(sm.kind, sm.gate, sm.conj, sm.off, sm.lds, loc, la, gat, gtab, sg));
                }
                tabs[t * tab_item + j] = v;
            }
            __syncthreads();
        }
        // 2. per-thread parts of every index (low step bits and slice bits)
        const int tbits = out_bits < klog ? out_bits : klog;
        const uint32_t olo = tid & ((1u << tbits) - 1u);
        uint32_t li[kMaxMain], xi[kMaxMain][2];
        uint32_t lt = 0, xt[2] = {0, 0};
#pragma unroll
        for (int i = 0; i < kMaxMain; ++i) {
            li[i] = 0;
            xi[i][0] = xi[i][1] = 0;
        }
        // (descriptor values are uniform: loaded once, then masked per thread)
        for (int b = 0; b < tbits; ++b) {
            const uint32_t m = ((olo >> b) & 1u) ? ~0u : 0u;
            lt |= st.tbit[b] & m;
#pragma unroll
            for (int i = 0; i < kMaxMain; ++i)
                if (i < n_main) li[i] |= mn[i].bit[b] & m;
        }
        if (tm.slice_bits) {
#pragma unroll
            for (int i = 0; i < kMaxMain; ++i)
                if (i < n_main)
                    for (int b = 0; b < tm.slice_bits; ++b)
                        if ((slice >> b) & 1u) li[i] |= mn[i].sbit[b];
        }
        // local-index bits of the summed variables (value bit k = step bit out_bits + k)
#pragma unroll
        for (int k = 0; k < 2; ++k)
            if (k < nsum) {
                xt[k] = st.tbit[out_bits + k];
#pragma unroll
                for (int i = 0; i < kMaxMain; ++i)
                    if (i < n_main) xi[i][k] = mn[i].bit[out_bits + k];
            }
        // 3. the output elements of every trajectory
        if (out_bits >= klog) {
            const uint32_t iters = 1u << (out_bits - klog);
            for (uint32_t t = 0; t < ng; ++t)
                step_item<V, true>(st, mn, n_main, n_small, tabs + t * tab_item, lds + t * lds_item,
                                   ga ? ga + (size_t)t * g_item : ga, gtab, signs + (size_t)t * words, li, xi, lt, xt,
                                   nsum, iters, klog, olo);
        } else {
            const uint32_t per = nthreads >> out_bits;
            for (uint32_t t = tid >> out_bits; t < ng; t += per)
                step_item<V, false>(st, mn, n_main, n_small, tabs + t * tab_item, lds + t * lds_item,
                                    ga ? ga + (size_t)t * g_item : ga, gtab, signs + (size_t)t * words, li, xi, lt,
                                    xt, nsum, 1u, klog, olo);
        }
        __syncthreads();
    }
    for (uint32_t t = tid; t < ng; t += nthreads)
        zz[(size_t)t * F] = (double)(tm.result_lds ? lds[t * lds_item + tm.result]
                                                   : ga[(size_t)t * g_item + tm.result]).x;
    __syncthreads();   // the arenas are reused by the next work item
}

// Persistent workgroups take work items (slice of a term, group of TB
// consecutive trajectories) in turn.  LDS: TB arenas of lds_item slots, then
// TB tables of tab_item slots; garena: grid x TB x stride slots of global
// memory (NULL when every intermediate fits the LDS arena).
template <class R>
__global__ __launch_bounds__(1024) void k_tn(const TnTerm* __restrict__ terms, const TnStep* __restrict__ steps,
                                             const TnMain* __restrict__ mains, const TnSmall* __restrict__ smalls,
                                             const typename Cx<R>::T* __restrict__ gtab,
                                             const uint32_t* __restrict__ signs, uint32_t words,
                                             double* __restrict__ zz, const TnSlice* __restrict__ slices, uint32_t F,
                                             uint32_t nb, uint32_t TB, typename Cx<R>::T* garena_all,
                                             uint32_t stride, uint32_t lds_item, uint32_t tab_item) {
    using V = typename Cx<R>::T;
    extern __shared__ char smem[];
    V* lds = reinterpret_cast<V*>(smem);
    V* tabs = lds + TB * lds_item;
    V* ga = garena_all ? garena_all + (size_t)blockIdx.x * TB * stride : nullptr;
    const uint32_t groups = (nb + TB - 1) / TB;
    const uint32_t items = F * groups;
    for (uint32_t item = blockIdx.x; item < items; item += gridDim.x) {
        const uint32_t f = item % F, g = item / F;
        const uint32_t b0 = g * TB, ng = min(TB, nb - b0);
        const TnSlice sl = slices[f];
        run_group<R>(lds, tabs, ga, terms[sl.term], steps, mains, smalls, gtab, signs + (size_t)b0 * words, words,
                     sl.slice, ng, lds_item, tab_item, stride, zz + (size_t)b0 * F + f, F);
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
using TnFn = void (*)(const TnTerm*, const TnStep*, const TnMain*, const TnSmall*, const typename Cx<R>::T*,
                      const uint32_t*, uint32_t, double*, const TnSlice*, uint32_t, uint32_t, uint32_t,
                      typename Cx<R>::T*, uint32_t, uint32_t, uint32_t);

struct TnKernel {
    void* f;
    uint32_t threads;
};

// Launch shapes the autotuner chooses from (variant 0 is the default):
// networks held in LDS take small workgroups, networks with intermediates in
// global memory one or two large persistent workgroups per CU.
constexpr uint32_t kTnVariants = 3;
template <class R>
TnKernel tn_kernel(bool hbm, uint32_t v) {
    static const uint32_t hbm_threads[kTnVariants] = {1024, 256, 512};
    static const uint32_t lds_threads[kTnVariants] = {256, 64, 128};
    return {(void*)k_tn<R>, (hbm ? hbm_threads : lds_threads)[v < kTnVariants ? v : 0]};
}

struct TnDevice {
    std::vector<TnNetwork> nets;
    std::vector<TnTerm> h_terms;
    std::vector<TnStep> h_steps;
    std::vector<TnMain> h_mains;
    std::vector<TnSmall> h_smalls;
    uint32_t TB = 1;            // trajectories per work item (contracted in lockstep)
    int arena = 0;              // global-memory slots per trajectory
    int lds_slots = 0;          // LDS arena slots per trajectory
    int tab_slots = 1;          // small-factor table entries per trajectory
    bool hbm = false;           // some intermediates in global memory (persistent workgroups with arenas)
    uint32_t stride = 0;        // global-memory arena slots per workgroup
    uint32_t grid = 0;          // persistent workgroups (global-memory tier)
    uint32_t F = 0;             // slices of all terms (work items per trajectory)
    uint32_t resident[2][kTnVariants] = {};   // workgroups the device holds at once, per precision and shape
    uint32_t per_cu[2][kTnVariants] = {};     // ... and per CU
    DevBuf terms, steps, mains, smalls, gtab32, gtab64, zz, garena, slices, toff;
};

// Step descriptors of one network: small factors (every input that is not an
// intermediate, and intermediates of rank <= 2) go into the step's table
// while the table's step bits stay within tab_cap; the other inputs are read
// per output element.
void describe(TnDevice* d, const TnNetwork& net, int tab_cap) {
    TnTerm tm{};
    tm.step0 = (int32_t)d->h_steps.size();
    tm.n_steps = (int32_t)net.steps.size();
    tm.result = net.result;
    tm.result_lds = net.result_lds;
    tm.slice_bits = net.slice_bits;
    for (const TnStepRec& sr : net.steps) {
        TnStep st{};
        st.out_bits = (int32_t)sr.out_vars.size();
        st.nsum = sr.nsum;
        st.out_off = sr.out_arena;
        st.out_lds = sr.out_lds;
        std::vector<int> order(sr.inputs.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        auto step_bits = [&](const TnInputRec& in) {
            uint32_t m = 0;
            for (int q : in.pos)
                if (q >= 0) m |= 1u << q;
            return m;
        };
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return __builtin_popcount(step_bits(sr.inputs[a])) < __builtin_popcount(step_bits(sr.inputs[b]));
        });
        uint32_t U = 0;
        std::vector<int> small, main;
        for (int i : order) {
            const TnInputRec& in = sr.inputs[i];
            const bool cand = in.kind != TN_INTER || in.pos.size() <= 2;
            const uint32_t u2 = U | step_bits(in);
            if (cand && __builtin_popcount(u2) <= tab_cap) {
                U = u2;
                small.push_back(i);
            } else {
                main.push_back(i);
            }
        }
        if ((int)main.size() > kMaxMain)
            fail(STN_E_UNSUPPORTED, "lightcone step with more than " + std::to_string(kMaxMain) + " large inputs");
        int tb[kStepBits + 1];
        int nt = 0;
        for (int b = 0; b <= kStepBits; ++b) tb[b] = -1;
        for (int b = 0; b < kStepBits; ++b)
            if ((U >> b) & 1u) {
                tb[b] = nt;
                st.tbit[b] = 1u << nt;
                ++nt;
            }
        st.tab_bits = nt;
        d->tab_slots = std::max(d->tab_slots, 1 << nt);
        st.small0 = (int32_t)d->h_smalls.size();
        st.n_small = (int32_t)small.size();
        for (int i : small) {
            const TnInputRec& in = sr.inputs[i];
            TnSmall sm{};
            sm.kind = in.kind;
            sm.gate = in.gate;
            sm.conj = in.conj;
            sm.off = in.arena;
            sm.lds = in.lds;
            for (size_t k = 0; k < in.pos.size(); ++k) {
                if (in.pos[k] >= 0)
                    sm.tbit[tb[in.pos[k]]] = 1u << k;
                else
                    sm.sbit[-1 - in.pos[k]] = 1u << k;
            }
            d->h_smalls.push_back(sm);
        }
        st.main0 = (int32_t)d->h_mains.size();
        st.n_main = (int32_t)main.size();
        for (int i : main)
            if (sr.inputs[i].kind != TN_INTER) st.generic = 1;
        for (int i : main) {
            const TnInputRec& in = sr.inputs[i];
            TnMain mn{};
            mn.kind = in.kind;
            mn.gate = in.gate;
            mn.conj = in.conj;
            mn.off = in.arena;
            mn.lds = in.lds;
            for (size_t k = 0; k < in.pos.size(); ++k) {
                if (in.pos[k] >= 0)
                    mn.bit[in.pos[k]] = 1u << k;
                else
                    mn.sbit[-1 - in.pos[k]] = 1u << k;
            }
            d->h_mains.push_back(mn);
        }
        d->h_steps.push_back(st);
    }
    d->h_terms.push_back(tm);
}

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

// Cost model of the trajectory group size (calibrated on n = 22..29, p = 2
// Erdos-Renyi jobs): a step costs a workgroup about kStepSeconds whatever its
// size (descriptor loads, table, barriers), shared by the group's
// trajectories; global-memory intermediates move at kArenaBytesPerS over the
// device.
constexpr double kStepSeconds = 3e-6;
constexpr double kArenaBytesPerS = 3e12;
constexpr double kFlopsPerS = 8e13;      // element arithmetic, mostly hidden under the memory traffic
constexpr int kTabBytes = 16 * 1024;     // small-factor tables of all trajectories of a group
constexpr uint32_t kGroupSizes[] = {1, 2, 4, 8, 16};

// Builds the networks of every observable term; records width and cost.
// Each term's order is lowered once per group size (the LDS arena of a
// trajectory shrinks as the group grows, so more intermediates may go to
// global memory); the group size with the smallest estimated time is kept.
thread_local uint32_t tl_plan_threads = 0;

void build_lightcone(stn_plan* p) {
    if (!p->frame_ok) fail(STN_E_UNSUPPORTED, "lightcone lowering needs Pauli noise and Pauli-rotation gates after the noise");
    if (p->obs_u.empty()) fail(STN_E_UNSUPPORTED, "lightcone lowering needs an observable");
    auto* d = new TnDevice();
    p->lc = d;
    p->lc_free = [](void* v) { delete static_cast<TnDevice*>(v); };
    const size_t elem = p->opts.precision == 128 ? 16 : 8;
    constexpr int kSizes = (int)(sizeof(kGroupSizes) / sizeof(kGroupSizes[0]));
    std::vector<int> budgets;
    for (uint32_t tb : kGroupSizes) budgets.push_back((int)(kLdsArenaBytes / tb / elem));
    std::vector<std::vector<TnNetwork>> by_size(kSizes);
    double cost = 0;
    int width = 0;
    int max_rank = 0;
    bool aborted = false;
    const int rank_cap = p->opts.lc_max_rank ? std::min<int>((int)p->opts.lc_max_rank, kStepBits - 1) : kStepBits - 1;
    const int slice_cap = (int)std::min<uint32_t>(p->opts.lc_slice_bits, kMaxSliceBits);
    // Terms are independent and each is built deterministically (its own
    // seeded restarts), so they are built on a few host threads and then
    // taken in term order; a caller-supplied order function is called on
    // this thread, in term order.  Once a term is too wide no new term is
    // started (every earlier term has been).
    const size_t T = p->obs_u.size();
    std::vector<std::vector<TnNetwork>> built(T);
    std::vector<std::exception_ptr> errs(T);
    std::atomic<size_t> next{0};
    std::atomic<bool> stop{false};
    auto worker = [&] {
        for (size_t t; !stop.load() && (t = next.fetch_add(1)) < T;) {
            try {
                built[t] = build_term(p, (uint32_t)t, p->obs_u[t], p->obs_v[t], p->opts.order_restarts,
                                      p->opts.order_seed, rank_cap, slice_cap, budgets);
                if (built[t][0].steps.empty() && !std::isfinite(built[t][0].cost)) stop = true;
            } catch (...) {
                errs[t] = std::current_exception();
                stop = true;
            }
        }
    };
    const size_t hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t cap = tl_plan_threads ? tl_plan_threads : 8;
    const size_t nthreads = p->opts.lc_order_fn ? 1 : std::min<size_t>({T, hw, cap});
    if (nthreads <= 1) {
        worker();
    } else {
        std::vector<std::thread> pool;
        for (size_t i = 0; i < nthreads; ++i) pool.emplace_back(worker);
        for (auto& th : pool) th.join();
    }
    for (size_t t = 0; t < T; ++t) {
        if (errs[t]) std::rethrow_exception(errs[t]);
        std::vector<TnNetwork>& nets = built[t];
        const TnNetwork& net = nets[0];
        if (net.steps.empty() && !std::isfinite(net.cost)) {
            max_rank = std::max(max_rank, net.width);   // stopped early: too wide for this lowering
            width = std::max(width, net.width);
            cost = HUGE_VAL;
            aborted = true;
            break;
        }
        for (auto& st : net.steps)
            for (auto& in : st.inputs) max_rank = std::max(max_rank, (int)in.pos.size());
        width = std::max(width, net.width);
        cost += net.cost;
        for (int k = 0; k < kSizes; ++k) by_size[k].push_back(std::move(nets[k]));
    }
    // the networks' size is known even where this lowering cannot run them
    p->lc_width = (uint32_t)width;
    p->lc_width_lb = aborted ? 1u : 0u;
    p->lc_flops_per_traj = 8.0 * cost;
    if (aborted || max_rank > kStepBits)
        fail(STN_E_UNSUPPORTED, "lightcone step rank above " + std::to_string(rank_cap + 1) + " (width " +
                                    std::to_string(width) + (slice_cap ? ", after slicing " + std::to_string(slice_cap) +
                                    " variables" : "") + ")");
    p->width = (uint32_t)width;
    const double budget = p->opts.hbm_budget ? (double)p->opts.hbm_budget : 64.0 * (1ull << 30);
    size_t steps = 0, runs = 0;   // steps of the networks; steps run per trajectory (every slice)
    for (auto& net : by_size[0]) {
        steps += net.steps.size();
        runs += net.steps.size() << net.slice_bits;
    }
    int best = -1;
    double best_est = 0, best_gbytes = 0;
    for (int k = 0; k < kSizes; ++k) {
        const uint32_t tb = kGroupSizes[k];
        double gbytes = 0;   // global-memory intermediates read and written per trajectory
        int arena = 0;
        for (auto& net : by_size[k]) {
            arena = std::max(arena, net.arena);
            for (auto& st : net.steps) {
                if (!st.out_lds) gbytes += std::ldexp((double)elem, (int)st.out_vars.size() + net.slice_bits);
                for (auto& in : st.inputs)
                    if (in.kind == TN_INTER && !in.lds)
                        gbytes += std::ldexp((double)elem, (int)in.pos.size() + net.slice_bits);
            }
        }
        // workgroups the device holds at once: one per CU with global-memory
        // intermediates (1024 threads), four of 256 threads otherwise; fewer
        // when the arenas of one per CU exceed the budget, and the device is
        // then only partly busy
        double wgs = arena ? 256.0 : 1024.0;
        if (arena) {
            const double stride = (double)((arena + 63) / 64 * 64);
            const double fit = std::floor(budget / 2 / (stride * elem * tb));
            if (fit < 32) continue;   // arenas exceed the budget
            wgs = std::min(wgs, fit);
        }
        const double busy = wgs / (arena ? 256.0 : 1024.0);
        const double est = (double)runs * kStepSeconds / (tb * wgs) +
                           (gbytes / kArenaBytesPerS + 8.0 * cost / kFlopsPerS) / busy;
        if (best < 0 || est < best_est) {
            best = k;
            best_est = est;
            best_gbytes = gbytes;
        }
    }
    if (best < 0) fail(STN_E_UNSUPPORTED, "lightcone intermediates exceed the memory budget (width " +
                                              std::to_string(width) + ")");
    d->TB = kGroupSizes[best];
    p->lc_group = d->TB;
    d->nets = std::move(by_size[best]);
    int tab_cap = 0;
    while (tab_cap < kTabBits && ((size_t)d->TB << (tab_cap + 1)) * elem <= (size_t)kTabBytes) ++tab_cap;
    for (auto& net : d->nets) {
        d->arena = std::max(d->arena, net.arena);
        d->lds_slots = std::max(d->lds_slots, net.lds_arena);
        describe(d, net, tab_cap);
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
    p->bytes_per_traj = best_gbytes + 8.0 * F;  // per-slice results; LDS intermediates are not counted
    p->lc_est_s = best_est;
    d->hbm = d->arena > 0;
    if (d->hbm) {
        // persistent workgroups with private global-memory arenas within the budget
        d->stride = (uint32_t)((d->arena + 63) / 64 * 64);
        const double per_wg = (double)d->stride * elem * d->TB;
        d->grid = (uint32_t)std::min(512.0, std::floor(budget / 2 / per_wg));
        p->lc_arena_bytes = (double)d->grid * per_wg;
    }
}

void upload_lightcone(stn_plan* p, hipStream_t s) {
    auto* d = static_cast<TnDevice*>(p->lc);
    std::vector<TnSlice> slices;
    std::vector<uint32_t> toff;
    for (size_t t = 0; t < d->nets.size(); ++t) {
        toff.push_back((uint32_t)slices.size());
        for (uint32_t sl = 0; sl < (1u << d->nets[t].slice_bits); ++sl) slices.push_back({(int32_t)t, sl});
    }
    toff.push_back((uint32_t)slices.size());
    if (d->h_mains.empty()) d->h_mains.push_back(TnMain{});
    if (d->h_smalls.empty()) d->h_smalls.push_back(TnSmall{});
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
    upload(d->terms, &p->alloc, d->h_terms.data(), d->h_terms.size() * sizeof(TnTerm), s);
    upload(d->steps, &p->alloc, d->h_steps.data(), d->h_steps.size() * sizeof(TnStep), s);
    upload(d->mains, &p->alloc, d->h_mains.data(), d->h_mains.size() * sizeof(TnMain), s);
    upload(d->smalls, &p->alloc, d->h_smalls.data(), d->h_smalls.size() * sizeof(TnSmall), s);
    upload(d->gtab32, &p->alloc, g32.data(), g32.size() * sizeof(float2), s);
    upload(d->gtab64, &p->alloc, g64.data(), g64.size() * sizeof(double2), s);
    upload(d->slices, &p->alloc, slices.data(), slices.size() * sizeof(TnSlice), s);
    upload(d->toff, &p->alloc, toff.data(), toff.size() * sizeof(uint32_t), s);
}

template <class R>
void launch_tn(stn_plan* p, TnDevice* d, const TnKernel& ker, uint32_t grid, size_t lds, const uint32_t* sg,
               uint32_t words, uint32_t nb, hipStream_t s) {
    using V = typename Cx<R>::T;
    const V* gtab = sizeof(R) == 8 ? (const V*)d->gtab64.p : (const V*)d->gtab32.p;
    hipLaunchKernelGGL(reinterpret_cast<TnFn<R>>(ker.f), dim3(grid), dim3(ker.threads), lds, s,
                       d->terms.as<TnTerm>(), d->steps.as<TnStep>(), d->mains.as<TnMain>(), d->smalls.as<TnSmall>(),
                       gtab, sg, words, d->zz.as<double>(), d->slices.as<TnSlice>(), d->F, nb, d->TB,
                       d->hbm ? d->garena.as<V>() : (V*)nullptr, d->stride, (uint32_t)d->lds_slots,
                       (uint32_t)d->tab_slots);
}

void launch_lightcone(stn_plan* p, stn_batch* b, hipStream_t s) {
    auto* d = static_cast<TnDevice*>(p->lc);
    const uint32_t T = (uint32_t)d->nets.size();
    const uint32_t F = d->F;
    const bool dbl = p->opts.precision == 128;
    const size_t elem = dbl ? 16 : 8;
    const size_t lds = (size_t)d->TB * (d->lds_slots + d->tab_slots) * elem;
    const uint32_t B = std::min<uint32_t>(b->K, 65535);
    d->zz.ensure(&p->alloc, (size_t)B * F * 8);
    const uint32_t v = std::min<uint32_t>(p->variant, kTnVariants - 1);
    const TnKernel ker = dbl ? tn_kernel<double>(d->hbm, v) : tn_kernel<float>(d->hbm, v);
    if (lds > 64 * 1024) {
        static std::mutex mu;
        static std::vector<void*> raised;
        std::lock_guard<std::mutex> lk(mu);
        if (std::find(raised.begin(), raised.end(), ker.f) == raised.end()) {
            STN_HIP(hipFuncSetAttribute(ker.f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        kLdsArenaBytes + kTabBytes));
            raised.push_back(ker.f);
        }
    }
    // persistent workgroups: as many as the device holds at once (the
    // global-memory tier also within its arena budget)
    uint32_t& res = d->resident[dbl][v];
    if (!res) {
        int dev = 0, cus = 0, per_cu = 0;
        STN_HIP(hipGetDevice(&dev));
        STN_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        STN_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ker.f, (int)ker.threads, lds));
        res = (uint32_t)std::max(1, per_cu) * (uint32_t)std::max(1, cus);
        d->per_cu[dbl][v] = (uint32_t)std::max(1, per_cu);
    }
    const uint32_t max_grid = d->hbm ? std::min(d->grid, res) : res;
    if (d->hbm) d->garena.ensure(&p->alloc, (size_t)max_grid * d->TB * d->stride * elem);
    double cost = 0;
    for (auto& net : d->nets) cost += net.cost;
    for (uint32_t c0 = 0; c0 < b->K; c0 += B) {
        const uint32_t nb = std::min(B, b->K - c0);
        const uint32_t* sg = b->d_signs.as<uint32_t>() + (size_t)c0 * b->words;
        const uint64_t items = (uint64_t)F * ((nb + d->TB - 1) / d->TB);
        uint32_t grid = (uint32_t)std::min<uint64_t>(max_grid, items);
        // a job server may keep some CUs free for other jobs' kernels
        if (p->grid_cap) grid = std::min(grid, std::max(1u, p->grid_cap * d->per_cu[dbl][v]));
        prof_begin(p, STN_K_TN_STEP, s);
        if (dbl)
            launch_tn<double>(p, d, ker, grid, lds, sg, b->words, nb, s);
        else
            launch_tn<float>(p, d, ker, grid, lds, sg, b->words, nb, s);
        STN_HIP(hipGetLastError());
        prof_end(p, STN_K_TN_STEP, s, (double)nb * p->bytes_per_traj, (double)nb * 8.0 * cost);
        hipLaunchKernelGGL(k_tn_energy, dim3((nb + 63) / 64), dim3(64), 0, s, d->zz.as<double>(), T,
                           d->toff.as<uint32_t>(), F, p->d_obs.as<uint32_t>(), p->d_obs_w.as<double>(),
                           b->d_frame.as<uint64_t>() + 2 * (size_t)c0, nb, b->d_energy.as<double>() + c0);
        STN_HIP(hipGetLastError());
    }
}

uint32_t tn_variants() { return kTnVariants; }

// loads this file's device code (the runtime does so at the first use of
// one of its kernels)
void warm_code_tn() {
    hipFuncAttributes a{};
    (void)hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_tn<float>));
}

}  // namespace stn
