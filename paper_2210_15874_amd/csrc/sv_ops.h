// One operator of the statevector interpreters (whole state in LDS, and the
// LDS tiles of the gate-by-gate lowering) applied to N = 2^m amplitudes in
// LDS, qubit q = bit q of the local index.  The workgroup's threads share the
// work; the caller synchronises before the next operator.  A Pauli is a
// signed permutation with its global phase dropped; every other operator is
// applied as its dense or diagonal matrix from the value table.
#pragma once

#include "stn_internal.h"

namespace stn {

template <class V> __device__ __forceinline__ V op_cmul(V a, V b) {
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <class V> __device__ __forceinline__ V op_cadd(V a, V b) {
    a.x += b.x;
    a.y += b.y;
    return a;
}
template <class V> __device__ __forceinline__ V op_neg_if(V a, bool neg) {
    if (neg) { a.x = -a.x; a.y = -a.y; }
    return a;
}

// index with a zero bit inserted at position q
__device__ __forceinline__ uint32_t op_ins0(uint32_t p, uint32_t q) {
    const uint32_t lo = p & ((1u << q) - 1u);
    return ((p ^ lo) << 1) | lo;
}

// The loops over amplitude pairs (or amplitudes) take kOpUnroll of a
// thread's items per round, all loads before any arithmetic, so that the LDS
// latency of one item overlaps the others' (worth it where few waves share a
// SIMD: the tiles of the gate-by-gate lowering); items of one operator are
// disjoint, so the order of the loads and stores within a round is free.
template <class V, uint32_t kOpUnroll = 1>
__device__ __forceinline__ void apply_lds_op(V* psi, uint32_t N, const LdsOp& o, const V* __restrict__ vals,
                                             uint32_t tid, uint32_t nthreads) {
    switch (o.kind) {
        case OP_DENSE1: {
            const V m0 = vals[o.mat], m1 = vals[o.mat + 1], m2 = vals[o.mat + 2], m3 = vals[o.mat + 3];
            const uint32_t bit = 1u << o.q0;
            for (uint32_t p0 = tid; p0 < N / 2; p0 += kOpUnroll * nthreads) {
                uint32_t i0[kOpUnroll];
                V a[kOpUnroll], c[kOpUnroll];
#pragma unroll
                for (uint32_t u = 0; u < kOpUnroll; ++u) {
                    const uint32_t p = p0 + u * nthreads;
                    i0[u] = op_ins0(p < N / 2 ? p : 0u, o.q0);
                    if (p < N / 2) { a[u] = psi[i0[u]]; c[u] = psi[i0[u] | bit]; }
                }
#pragma unroll
                for (uint32_t u = 0; u < kOpUnroll; ++u) {
                    if (p0 + u * nthreads >= N / 2) continue;
                    psi[i0[u]] = op_cadd(op_cmul(m0, a[u]), op_cmul(m1, c[u]));
                    psi[i0[u] | bit] = op_cadd(op_cmul(m2, a[u]), op_cmul(m3, c[u]));
                }
            }
            break;
        }
        case OP_DENSE2: {
            const uint32_t qa = o.q0 < o.q1 ? o.q0 : o.q1, qb = o.q0 < o.q1 ? o.q1 : o.q0;
            const uint32_t b0 = 1u << o.q0, b1 = 1u << o.q1;
            for (uint32_t p = tid; p < N / 4; p += nthreads) {
                const uint32_t i = op_ins0(op_ins0(p, qa), qb);
                const uint32_t ix[4] = {i, i | b0, i | b1, i | b0 | b1};
                V v[4];
#pragma unroll
                for (int l = 0; l < 4; ++l) v[l] = psi[ix[l]];
#pragma unroll
                for (int l = 0; l < 4; ++l) {
                    V acc = op_cmul(vals[o.mat + 4 * l], v[0]);
#pragma unroll
                    for (int m = 1; m < 4; ++m) acc = op_cadd(acc, op_cmul(vals[o.mat + 4 * l + m], v[m]));
                    psi[ix[l]] = acc;
                }
            }
            break;
        }
        case OP_DIAG1: {
            const V d0 = vals[o.mat], d1 = vals[o.mat + 1];
            for (uint32_t i0 = tid; i0 < N; i0 += kOpUnroll * nthreads) {
                V a[kOpUnroll];
#pragma unroll
                for (uint32_t u = 0; u < kOpUnroll; ++u)
                    if (i0 + u * nthreads < N) a[u] = psi[i0 + u * nthreads];
#pragma unroll
                for (uint32_t u = 0; u < kOpUnroll; ++u) {
                    const uint32_t i = i0 + u * nthreads;
                    if (i < N) psi[i] = op_cmul((i >> o.q0) & 1 ? d1 : d0, a[u]);
                }
            }
            break;
        }
        case OP_DIAG2: {
            const V d0 = vals[o.mat], d1 = vals[o.mat + 1], d2 = vals[o.mat + 2], d3 = vals[o.mat + 3];
            for (uint32_t i0 = tid; i0 < N; i0 += kOpUnroll * nthreads) {
                V a[kOpUnroll];
#pragma unroll
                for (uint32_t u = 0; u < kOpUnroll; ++u)
                    if (i0 + u * nthreads < N) a[u] = psi[i0 + u * nthreads];
#pragma unroll
                for (uint32_t u = 0; u < kOpUnroll; ++u) {
                    const uint32_t i = i0 + u * nthreads;
                    if (i >= N) continue;
                    // selects, not an indexed local array (which would live in scratch)
                    const bool qa = (i >> o.q0) & 1, qb = (i >> o.q1) & 1;
                    const V lo = qa ? d1 : d0, hi = qa ? d3 : d2;
                    psi[i] = op_cmul(qb ? hi : lo, a[u]);
                }
            }
            break;
        }
        case OP_PAULI: {
            const uint32_t x = (uint32_t)o.xmask, z = (uint32_t)o.zmask;
            if (x == 0) {
                for (uint32_t i0 = tid; i0 < N; i0 += kOpUnroll * nthreads) {
                    V a[kOpUnroll];
#pragma unroll
                    for (uint32_t u = 0; u < kOpUnroll; ++u)
                        if (i0 + u * nthreads < N) a[u] = psi[i0 + u * nthreads];
#pragma unroll
                    for (uint32_t u = 0; u < kOpUnroll; ++u) {
                        const uint32_t i = i0 + u * nthreads;
                        if (i < N) psi[i] = op_neg_if(a[u], __popc(i & z) & 1);
                    }
                }
            } else {
                const uint32_t lb = __ffs(x) - 1;
                for (uint32_t p0 = tid; p0 < N / 2; p0 += kOpUnroll * nthreads) {
                    uint32_t ii[kOpUnroll];
                    V a[kOpUnroll], c[kOpUnroll];
#pragma unroll
                    for (uint32_t u = 0; u < kOpUnroll; ++u) {
                        const uint32_t p = p0 + u * nthreads;
                        ii[u] = op_ins0(p < N / 2 ? p : 0u, lb);
                        if (p < N / 2) { a[u] = psi[ii[u]]; c[u] = psi[ii[u] ^ x]; }
                    }
#pragma unroll
                    for (uint32_t u = 0; u < kOpUnroll; ++u) {
                        if (p0 + u * nthreads >= N / 2) continue;
                        const uint32_t i = ii[u], j = i ^ x;
                        psi[j] = op_neg_if(a[u], __popc(i & z) & 1);
                        psi[i] = op_neg_if(c[u], __popc(j & z) & 1);
                    }
                }
            }
            break;
        }
        default: break;  // identity
    }
}

// diagonal operators (and the identity): applied element by element
__device__ __forceinline__ bool op_is_diagonal(const LdsOp& o) {
    return o.kind == OP_DIAG1 || o.kind == OP_DIAG2 || (o.kind == OP_PAULI && o.xmask == 0) || o.kind == OP_IDENT;
}

// A run of diagonal operators ops[0 .. cnt) in one pass over the tile: each
// element is read once, multiplied by every operator's factor in order, and
// written once (instead of one pass and one barrier per operator).
template <class V, uint32_t kOpUnroll = 1>
__device__ __forceinline__ void apply_lds_diag_run(V* psi, uint32_t N, const LdsOp* ops, uint32_t cnt,
                                                   const V* __restrict__ vals, uint32_t tid, uint32_t nthreads) {
    for (uint32_t i0 = tid; i0 < N; i0 += kOpUnroll * nthreads) {
        V a[kOpUnroll];
#pragma unroll
        for (uint32_t u = 0; u < kOpUnroll; ++u)
            if (i0 + u * nthreads < N) a[u] = psi[i0 + u * nthreads];
        for (uint32_t k = 0; k < cnt; ++k) {
            const LdsOp o = ops[k];
            if (o.kind == OP_DIAG1) {
                const V d0 = vals[o.mat], d1 = vals[o.mat + 1];
#pragma unroll
                for (uint32_t u = 0; u < kOpUnroll; ++u) a[u] = op_cmul(((i0 + u * nthreads) >> o.q0) & 1 ? d1 : d0, a[u]);
            } else if (o.kind == OP_DIAG2) {
                const V d0 = vals[o.mat], d1 = vals[o.mat + 1], d2 = vals[o.mat + 2], d3 = vals[o.mat + 3];
#pragma unroll
                for (uint32_t u = 0; u < kOpUnroll; ++u) {
                    const uint32_t i = i0 + u * nthreads;
                    const bool qa = (i >> o.q0) & 1, qb = (i >> o.q1) & 1;
                    const V lo = qa ? d1 : d0, hi = qa ? d3 : d2;
                    a[u] = op_cmul(qb ? hi : lo, a[u]);
                }
            } else if (o.kind == OP_PAULI) {
                const uint32_t z = (uint32_t)o.zmask;
#pragma unroll
                for (uint32_t u = 0; u < kOpUnroll; ++u) a[u] = op_neg_if(a[u], __popc((i0 + u * nthreads) & z) & 1);
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < kOpUnroll; ++u)
            if (i0 + u * nthreads < N) psi[i0 + u * nthreads] = a[u];
    }
}

// Up to three one-qubit dense operators on distinct qubits (in order, no
// identities between them) in one pass over groups of 2^K elements: a group
// holds every combination of the K qubits, so applying the operators one
// after another inside it does the same arithmetic, element by element, as
// one pass per operator.
template <class V, int K>
__device__ __forceinline__ void apply_lds_dense1_run(V* psi, uint32_t N, const LdsOp& o0, const LdsOp& o1,
                                                     const LdsOp& o2, const V* __restrict__ vals, uint32_t tid,
                                                     uint32_t nthreads) {
    const uint32_t q[3] = {o0.q0, o1.q0, o2.q0};
    const uint32_t mat[3] = {o0.mat, o1.mat, o2.mat};
    uint32_t qs[K];   // the qubits in increasing order (for inserting the zero bits)
#pragma unroll
    for (int t = 0; t < K; ++t) qs[t] = q[t];
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
        for (int b = a + 1; b < K; ++b)
            if (qs[b] < qs[a]) { const uint32_t x = qs[a]; qs[a] = qs[b]; qs[b] = x; }
    V m[K][4];
#pragma unroll
    for (int t = 0; t < K; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) m[t][e] = vals[mat[t] + e];
    for (uint32_t g = tid; g < (N >> K); g += nthreads) {
        uint32_t base = g;
#pragma unroll
        for (int t = 0; t < K; ++t) base = op_ins0(base, qs[t]);
        V v[1 << K];
#pragma unroll
        for (uint32_t j = 0; j < (1u << K); ++j) {
            uint32_t i = base;
#pragma unroll
            for (int t = 0; t < K; ++t)
                if ((j >> t) & 1u) i |= 1u << q[t];
            v[j] = psi[i];
        }
#pragma unroll
        for (int t = 0; t < K; ++t)
#pragma unroll
            for (uint32_t j = 0; j < (1u << K); ++j) {
                if ((j >> t) & 1u) continue;
                const V a = v[j], c = v[j | (1u << t)];
                v[j] = op_cadd(op_cmul(m[t][0], a), op_cmul(m[t][1], c));
                v[j | (1u << t)] = op_cadd(op_cmul(m[t][2], a), op_cmul(m[t][3], c));
            }
#pragma unroll
        for (uint32_t j = 0; j < (1u << K); ++j) {
            uint32_t i = base;
#pragma unroll
            for (int t = 0; t < K; ++t)
                if ((j >> t) & 1u) i |= 1u << q[t];
            psi[i] = v[j];
        }
    }
}

}  // namespace stn
