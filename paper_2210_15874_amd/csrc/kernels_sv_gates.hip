// Gate-by-gate HBM statevector contraction: any circuit, any channel, for
// states too large for LDS (Sec. III-G: each noisy circuit of the ensemble is
// simulated to its statevector; Eq. (1): after a gate, each of its channels
// contributes one Kraus operator, picked per trajectory).  The batch's states
// psi[k][x] (complex64 or complex128, 2^n per trajectory, trajectory-major)
// stay in HBM; every entry of the plan's operator list (the gate list with a
// noise-site entry after each gate's channels) is one launch over the whole
// batch.  A launch's item is one group of amplitudes that the operator mixes:
// a pair over q0 (one-qubit operators) or a quadruple over (q0, q1) (two-qubit
// ones).  At a noise site each trajectory resolves its own operator (identity,
// a Pauli as a signed permutation with its global phase dropped, or the dense
// K_j / sqrt(q_j)), always on the site's qubits, so a launch's items are the
// same for every trajectory.  Each launch reads and writes the batch once; no
// operators are fused.
//
// Energy: <psi|C|psi>, C = sum_t w_t [z_u != z_v], per trajectory: each
// workgroup sums |psi(x)|^2 C(x) over one contiguous slice in binary64 in a
// fixed order and tree, then one lane per trajectory adds the slices in
// order, so the value does not depend on the launch.
#include "stn_internal.h"

namespace stn {

namespace {

template <class R> struct Cg;
template <> struct Cg<float> { using T = float2; };
template <> struct Cg<double> { using T = double2; };

template <class V> __device__ __forceinline__ V gmul(V a, V b) {
    V r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <class V> __device__ __forceinline__ V gadd(V a, V b) {
    a.x += b.x;
    a.y += b.y;
    return a;
}
template <class V> __device__ __forceinline__ V gneg(V a, bool neg) {
    if (neg) { a.x = -a.x; a.y = -a.y; }
    return a;
}

__device__ __forceinline__ uint64_t insert0(uint64_t p, uint32_t q) {
    const uint64_t lo = p & ((1ull << q) - 1ull);
    return ((p ^ lo) << 1) | lo;
}

constexpr uint32_t kGateThreads = 256;
constexpr uint32_t kEnergySlices = 64;   // workgroups per trajectory in the energy sum

template <class V>
__global__ __launch_bounds__(256) void k_gates_init(V* __restrict__ psi, uint64_t total, uint32_t n) {
    const uint64_t mask = (1ull << n) - 1ull;
    for (uint64_t i = (uint64_t)blockIdx.x * kGateThreads + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * kGateThreads) {
        V v;
        v.x = (i & mask) == 0 ? 1 : 0;
        v.y = 0;
        psi[i] = v;
    }
}

// One operator-list entry over the batch: grid (group chunks, trajectory).
// nq = 1: groups are pairs over q0; nq = 2: quadruples, local index bit 0 =
// q0, bit 1 = q1.  A workgroup serves one trajectory, so it resolves the
// operator once (a trajectory that drew the identity returns at once) and
// keeps its values in registers.  Each lane takes kGroupsPerLane groups per
// round and issues all their loads before any store (distinct groups never
// share an amplitude), so more bytes are in flight per lane.
constexpr uint32_t kGroupsPerLane = 4;
constexpr uint32_t kGateChunksMax = 2048;   // enough workgroups for one trajectory at n = 30

template <class V>
__global__ __launch_bounds__(256) void k_gates_op(V* __restrict__ psi, uint32_t n, LdsOp op, uint32_t nq,
                                                  const V* __restrict__ vals, const LdsOp* __restrict__ site_ops,
                                                  const uint32_t* __restrict__ site_off,
                                                  const uint8_t* __restrict__ idx, uint32_t S) {
    const uint64_t k = blockIdx.y;
    LdsOp o = op;
    if (op.kind == OP_SITE) o = site_ops[site_off[op.site] + idx[k * S + op.site]];
    if (o.kind == OP_IDENT) return;   // the same for the whole workgroup; no barrier follows
    const uint32_t qa = nq == 2 ? min(op.q0, op.q1) : op.q0, qb = nq == 2 ? max(op.q0, op.q1) : 0;
    const uint64_t groups = 1ull << (n - nq);
    V* base = psi + k * (1ull << n);
    const uint64_t b0 = 1ull << op.q0, b1 = nq == 2 ? 1ull << op.q1 : 0;
    const uint32_t nv = o.kind == OP_DENSE2 ? 16 : (o.kind == OP_DENSE1 || o.kind == OP_DIAG2) ? 4
                      : o.kind == OP_DIAG1 ? 2 : 0;
    V m[16];
#pragma unroll
    for (uint32_t t = 0; t < 16; ++t) {
        m[t].x = 0;
        m[t].y = 0;
        if (t < nv) m[t] = vals[o.mat + t];
    }
    const uint64_t span = (uint64_t)kGateThreads * kGroupsPerLane;
    for (uint64_t g0 = (uint64_t)blockIdx.x * span + threadIdx.x; g0 < groups; g0 += (uint64_t)gridDim.x * span) {
        uint64_t ix[kGroupsPerLane][4];
        V a[kGroupsPerLane][4];
        bool act[kGroupsPerLane];
#pragma unroll
        for (uint32_t r = 0; r < kGroupsPerLane; ++r) {
            const uint64_t g = g0 + (uint64_t)r * kGateThreads;
            act[r] = g < groups;
            if (!act[r]) continue;
            const uint64_t i = nq == 1 ? insert0(g, qa) : insert0(insert0(g, qa), qb);
            ix[r][0] = i;
            ix[r][1] = i | b0;
            ix[r][2] = i | b1;
            ix[r][3] = i | b0 | b1;
            a[r][0] = base[ix[r][0]];
            a[r][1] = base[ix[r][1]];
            if (nq == 2) {
                a[r][2] = base[ix[r][2]];
                a[r][3] = base[ix[r][3]];
            }
        }
#pragma unroll
        for (uint32_t r = 0; r < kGroupsPerLane; ++r) {
            if (!act[r]) continue;
            V res[4];
            switch (o.kind) {
                case OP_DENSE1:   // on q0 (a one-qubit site or gate)
                    res[0] = gadd(gmul(m[0], a[r][0]), gmul(m[1], a[r][1]));
                    res[1] = gadd(gmul(m[2], a[r][0]), gmul(m[3], a[r][1]));
                    break;
                case OP_DENSE2:
#pragma unroll
                    for (uint32_t l = 0; l < 4; ++l) {
                        V acc = gmul(m[4 * l], a[r][0]);
#pragma unroll
                        for (uint32_t c = 1; c < 4; ++c) acc = gadd(acc, gmul(m[4 * l + c], a[r][c]));
                        res[l] = acc;
                    }
                    break;
                case OP_DIAG1:
                    res[0] = gmul(m[0], a[r][0]);
                    res[1] = gmul(m[1], a[r][1]);
                    break;
                case OP_DIAG2:
#pragma unroll
                    for (uint32_t l = 0; l < 4; ++l) res[l] = gmul(m[l], a[r][l]);
                    break;
                default: {        // OP_PAULI: amplitude at x moves to x ^ X with sign (-1)^|x & Z|
                    const uint64_t X = o.xmask, Z = o.zmask;
#pragma unroll
                    for (uint32_t t = 0; t < 4; ++t) {
                        V v = a[r][0];
                        uint64_t src = ix[r][0];
#pragma unroll
                        for (uint32_t l = 1; l < 4; ++l)
                            if (l < (1u << nq) && (ix[r][l] ^ X) == ix[r][t]) {
                                v = a[r][l];
                                src = ix[r][l];
                            }
                        res[t] = gneg(v, __popcll(src & Z) & 1);
                    }
                    break;
                }
            }
            base[ix[r][0]] = res[0];
            base[ix[r][1]] = res[1];
            if (nq == 2) {
                base[ix[r][2]] = res[2];
                base[ix[r][3]] = res[3];
            }
        }
    }
}

__device__ double gates_block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t s = kGateThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    return red[0];
}

// grid (kEnergySlices, K): slice partials of sum_x |psi(x)|^2 C(x)
template <class V>
__global__ __launch_bounds__(256) void k_gates_energy(const V* __restrict__ psi, uint32_t n,
                                                      const uint32_t* __restrict__ uv, const double* __restrict__ w,
                                                      uint32_t n_terms, double* __restrict__ part) {
    __shared__ double red[kGateThreads];
    const uint64_t N = 1ull << n;
    const uint64_t per = (N + kEnergySlices - 1) / kEnergySlices;
    const uint64_t a = min<uint64_t>(N, blockIdx.x * per), b = min<uint64_t>(N, a + per);
    const V* base = psi + (uint64_t)blockIdx.y * N;
    double s = 0.0;
    for (uint64_t x = a + threadIdx.x; x < b; x += kGateThreads) {
        double c = 0.0;
        for (uint32_t t = 0; t < n_terms; ++t)
            if (((x >> uv[2 * t]) ^ (x >> uv[2 * t + 1])) & 1) c += w[t];
        const V v = base[x];
        s += ((double)v.x * v.x + (double)v.y * v.y) * c;
    }
    const double tot = gates_block_sum(s, red);
    if (threadIdx.x == 0) part[(uint64_t)blockIdx.y * kEnergySlices + blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_gates_energy_sum(const double* __restrict__ part, uint32_t K,
                                                          double* __restrict__ energy) {
    const uint32_t k = blockIdx.x * kGateThreads + threadIdx.x;
    if (k >= K) return;
    double s = 0.0;
    for (uint32_t j = 0; j < kEnergySlices; ++j) s += part[(uint64_t)k * kEnergySlices + j];
    energy[k] = s;
}

template <class V> void run_gates(stn_plan* p, stn_batch* b, hipStream_t s, const V* vals) {
    const uint32_t n = p->n, K = b->K;
    const uint64_t N = 1ull << n;
    V* psi = b->d_states.as<V>();
    const uint32_t cap = 256 * 16;
    auto grid = [&](uint64_t items) {
        return (uint32_t)std::min<uint64_t>((items + kGateThreads - 1) / kGateThreads, cap);
    };
    hipLaunchKernelGGL(k_gates_init<V>, dim3(grid(N * K)), dim3(kGateThreads), 0, s, psi, N * K, n);
    STN_HIP(hipGetLastError());
    const uint32_t S = (uint32_t)p->sites.size();
    for (LdsOp op : p->lds_ops) {
        uint32_t nq;
        if (op.kind == OP_SITE) {   // the entry names the site; its groups are over the site's qubits
            const SiteRec& site = p->sites[op.site];
            nq = site.nq;
            op.q0 = site.q0;
            op.q1 = site.q1;
        } else if (op.kind == OP_IDENT) {
            continue;
        } else {
            nq = (op.kind == OP_DENSE2 || op.kind == OP_DIAG2) ? 2 : 1;
        }
        const uint64_t span = (uint64_t)kGateThreads * kGroupsPerLane;
        const uint32_t chunks = (uint32_t)std::min<uint64_t>(((N >> nq) + span - 1) / span, kGateChunksMax);
        hipLaunchKernelGGL(k_gates_op<V>, dim3(chunks, K), dim3(kGateThreads), 0, s, psi, n, op, nq, vals,
                           p->d_site_ops.as<LdsOp>(), p->d_site_op_off.as<uint32_t>(), b->d_idx.as<uint8_t>(), S);
        STN_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_gates_energy<V>, dim3(kEnergySlices, K), dim3(kGateThreads), 0, s, psi, n,
                       p->d_obs.as<uint32_t>(), p->d_obs_w.as<double>(), (uint32_t)p->obs_u.size(),
                       b->d_gates_part.as<double>());
    STN_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gates_energy_sum, dim3((K + kGateThreads - 1) / kGateThreads), dim3(kGateThreads), 0, s,
                       b->d_gates_part.as<double>(), K, b->d_energy.as<double>());
    STN_HIP(hipGetLastError());
}

}  // namespace

void launch_sv_gates(stn_plan* p, stn_batch* b, hipStream_t s) {
    const uint32_t n = p->n;
    if (n < 2 || n > kGatesMaxQubits) fail(STN_E_UNSUPPORTED, "gate-by-gate lowering needs 2 <= n <= 30");
    if (b->K > 65535) fail(STN_E_INVALID, "gate-by-gate lowering: at most 65535 trajectories per batch");
    const bool dbl = p->opts.precision == 128;
    const size_t elem = dbl ? 16 : 8;
    b->d_states.ensure(&p->alloc, ((size_t)b->K << n) * elem);
    b->d_gates_part.ensure(&p->alloc, (size_t)b->K * kEnergySlices * 8);
    prof_begin(p, STN_K_SV_PASS, s);
    if (dbl) run_gates<double2>(p, b, s, p->d_lds_vals64.as<double2>());
    else run_gates<float2>(p, b, s, p->d_lds_vals32.as<float2>());
    // bytes counted: entries that read and write every trajectory's state (gates,
    // and noise sites none of whose operators is the identity).  Sites whose
    // identity operator most trajectories draw are left out, so the figure is a
    // lower bound on the bytes moved.
    double full = 0;
    for (const LdsOp& op : p->lds_ops) {
        if (op.kind == OP_IDENT) continue;
        if (op.kind != OP_SITE) {
            full += 1;
            continue;
        }
        bool any_ident = false;
        for (uint32_t j = p->site_op_off[op.site]; j < p->site_op_off[op.site + 1]; ++j)
            any_ident |= p->site_ops[j].kind == OP_IDENT;
        full += any_ident ? 0 : 1;
    }
    prof_end(p, STN_K_SV_PASS, s, std::ldexp((double)b->K * elem, (int)n) * (2.0 * full + 2.0), 0.0);
}

}  // namespace stn
