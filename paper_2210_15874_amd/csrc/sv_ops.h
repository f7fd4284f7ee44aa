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

template <class V>
__device__ __forceinline__ void apply_lds_op(V* psi, uint32_t N, const LdsOp& o, const V* __restrict__ vals,
                                             uint32_t tid, uint32_t nthreads) {
    switch (o.kind) {
        case OP_DENSE1: {
            const V m0 = vals[o.mat], m1 = vals[o.mat + 1], m2 = vals[o.mat + 2], m3 = vals[o.mat + 3];
            const uint32_t bit = 1u << o.q0;
            for (uint32_t p = tid; p < N / 2; p += nthreads) {
                const uint32_t i0 = op_ins0(p, o.q0), i1 = i0 | bit;
                const V a = psi[i0], c = psi[i1];
                psi[i0] = op_cadd(op_cmul(m0, a), op_cmul(m1, c));
                psi[i1] = op_cadd(op_cmul(m2, a), op_cmul(m3, c));
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
            for (uint32_t i = tid; i < N; i += nthreads) psi[i] = op_cmul((i >> o.q0) & 1 ? d1 : d0, psi[i]);
            break;
        }
        case OP_DIAG2: {
            const V d0 = vals[o.mat], d1 = vals[o.mat + 1], d2 = vals[o.mat + 2], d3 = vals[o.mat + 3];
            for (uint32_t i = tid; i < N; i += nthreads) {
                // selects, not an indexed local array (which would live in scratch)
                const bool a = (i >> o.q0) & 1, b = (i >> o.q1) & 1;
                const V lo = a ? d1 : d0, hi = a ? d3 : d2;
                psi[i] = op_cmul(b ? hi : lo, psi[i]);
            }
            break;
        }
        case OP_PAULI: {
            const uint32_t x = (uint32_t)o.xmask, z = (uint32_t)o.zmask;
            if (x == 0) {
                for (uint32_t i = tid; i < N; i += nthreads) psi[i] = op_neg_if(psi[i], __popc(i & z) & 1);
            } else {
                const uint32_t lb = __ffs(x) - 1;
                for (uint32_t p = tid; p < N / 2; p += nthreads) {
                    const uint32_t i = op_ins0(p, lb), j = i ^ x;
                    const V a = psi[i], c = psi[j];
                    psi[j] = op_neg_if(a, __popc(i & z) & 1);
                    psi[i] = op_neg_if(c, __popc(j & z) & 1);
                }
            }
            break;
        }
        default: break;  // identity
    }
}

}  // namespace stn
