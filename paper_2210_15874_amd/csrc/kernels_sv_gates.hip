// Gate-by-gate HBM statevector contraction: any circuit, any channel, for
// states too large for LDS (Sec. III-G: each noisy circuit of the ensemble is
// simulated to its statevector; Eq. (1): after a gate, each of its channels
// contributes one Kraus operator, picked per trajectory).  The batch's states
// psi[k][x] (complex64 or complex128, 2^n per trajectory, trajectory-major)
// stay in HBM.  The plan's operator list (the gates in order, with a
// noise-site entry after each gate for each of its channels) is cut into
// groups of consecutive entries whose qubits, together with the four lowest
// storage bits, fit one tile of 13 storage bits (12 in complex128).  Each
// group is one launch: a workgroup serves one trajectory, resolves the
// group's operators for it once (at a noise site the trajectory's own
// operator: identity, a Pauli as a signed permutation with its global phase
// dropped, or the dense K_j / sqrt(q_j)), then for each of its tiles loads the
// 2^13 amplitudes into LDS, applies the group's operators in order and stores
// them back.  A group all of whose operators are the identity for a
// trajectory leaves that trajectory untouched.  The first group generates
// |0..0> instead of loading.
//
// Energy: <psi|C|psi>, C = sum_t w_t [z_u != z_v], per trajectory: each
// workgroup sums |psi(x)|^2 C(x) over one contiguous slice in binary64 in a
// fixed order and tree, then one lane per trajectory adds the slices in
// order, so the value does not depend on the launch.
#include <algorithm>

#include "sv_ops.h"

namespace stn {

namespace {

template <class R> struct Cg;
template <> struct Cg<float> { using T = float2; };
template <> struct Cg<double> { using T = double2; };

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

constexpr uint32_t kTileLog = 9;                  // 512 threads: 4 waves per SIMD at two workgroups per CU
constexpr uint32_t kTileThreads = 1u << kTileLog;

// a thread's tile elements: tile index tid + r * kTileThreads, r < tile_per<V>
// (tiles of at most 13 bits in complex64, 12 in complex128)
template <class V> constexpr uint32_t tile_per() { return (sizeof(V) > 8 ? (1u << 12) : (1u << 13)) / kTileThreads; }

// storage bits of the tile bits above the thread bits, for round r (uniform)
__device__ __forceinline__ uint64_t tile_hi(const GateGroup& g, uint32_t r) {
    uint64_t z = 0;
    for (uint32_t l = kTileLog; l < g.nbits; ++l)
        if ((r >> (l - kTileLog)) & 1u) z |= 1ull << g.tb[l];
    return z;
}

__device__ __forceinline__ uint64_t tile_hi2(const GateGroup& g, uint32_t r) {
    uint64_t z = 0;
    for (uint32_t l = kTileLog + 1; l < g.nbits; ++l)
        if ((r >> (l - kTileLog - 1)) & 1u) z |= 1ull << g.tb[l];
    return z;
}

__device__ __forceinline__ uint64_t remap_mask(uint64_t m, const uint8_t* local) {
    uint64_t r = 0;
    for (; m; m &= m - 1) r |= 1ull << local[__builtin_ctzll(m)];
    return r;
}

// One group over the batch: grid (tile chunks, trajectory).  LDS: the tile
// (2^g.nbits amplitudes) and the group's operators resolved for this
// trajectory.
template <class V>
__global__ __launch_bounds__(kTileThreads) void k_gates_tile(V* __restrict__ psi, uint32_t n, const GateGroup g, int init,
                                                    const LdsOp* __restrict__ gops, const V* __restrict__ vals,
                                                    const LdsOp* __restrict__ site_ops,
                                                    const uint32_t* __restrict__ site_off,
                                                    const uint8_t* __restrict__ idx, uint32_t S) {
    extern __shared__ __align__(16) char smem[];
    const uint32_t T = 1u << g.nbits;
    V* tile = reinterpret_cast<V*>(smem);
    LdsOp* ops = reinterpret_cast<LdsOp*>(tile + T);
    __shared__ int s_any;
    const uint32_t tid = threadIdx.x;
    const uint64_t k = blockIdx.y;
    if (tid == 0) s_any = 0;
    __syncthreads();
    // this trajectory's operators on tile-local qubits
    for (uint32_t i = tid; i < g.n_ops; i += kTileThreads) {
        LdsOp o = gops[g.op0 + i];
        if (o.kind == OP_SITE) {
            o = site_ops[site_off[o.site] + idx[k * S + o.site]];
            o.q0 = g.local[o.q0 & 31u];
            o.q1 = g.local[o.q1 & 31u];
            o.xmask = remap_mask(o.xmask, g.local);
            o.zmask = remap_mask(o.zmask, g.local);
        }
        if (o.kind != OP_IDENT) s_any = 1;
        ops[i] = o;
    }
    __syncthreads();
    if (!s_any && !init) return;   // the same for the whole workgroup
    // storage index = tile base | spread(local index), spread(j) = sum_l bit l of j << tb[l]
    uint64_t fixed = (1ull << n) - 1ull;
    for (uint32_t l = 0; l < g.nbits; ++l) fixed &= ~(1ull << g.tb[l]);
    uint64_t zt = 0;
    for (uint32_t l = 0; l < g.nbits && l < kTileLog; ++l)
        if ((tid >> l) & 1u) zt |= 1ull << g.tb[l];
    uint64_t zt2 = 0;   // pair layout: tile bits 1 .. kTileLog from the thread index
    for (uint32_t l = 1; l < g.nbits && l <= kTileLog; ++l)
        if ((tid >> (l - 1)) & 1u) zt2 |= 1ull << g.tb[l];
    const uint32_t nt = 1u << (n - g.nbits);
    V* st = psi + (k << n);
    for (uint32_t t = blockIdx.x; t < nt; t += gridDim.x) {
        uint64_t base = 0;
        {
            uint32_t v = t;
            for (uint64_t m = fixed; m; m &= m - 1, v >>= 1)
                if (v & 1u) base |= m & (~m + 1);
        }
        // all of a thread's loads are issued before any is written to LDS
        constexpr uint32_t kTilePer = tile_per<V>();
        // complex64: amplitude pairs along tile bit 0 = storage bit 0 (every
        // group tile holds it), one 16-byte access per pair
        constexpr bool kPairs = sizeof(V) == 8;
        V vv[kTilePer];
        if constexpr (kPairs) {
            // pair p = tid + r * threads: tile indices 2p, 2p + 1 (tiles smaller
            // than two per thread leave the upper threads idle)
#pragma unroll
            for (uint32_t r = 0; r < kTilePer / 2; ++r) {
                if ((r << (kTileLog + 1)) >= T) break;
                if (2 * (tid + (r << kTileLog)) >= T) continue;
                const uint64_t z = base | zt2 | tile_hi2(g, r);
                if (init) {
                    vv[2 * r].x = z == 0 ? 1 : 0; vv[2 * r].y = 0;
                    vv[2 * r + 1].x = 0; vv[2 * r + 1].y = 0;
                } else {
                    const float4 w = *reinterpret_cast<const float4*>(st + z);
                    vv[2 * r].x = w.x; vv[2 * r].y = w.y; vv[2 * r + 1].x = w.z; vv[2 * r + 1].y = w.w;
                }
            }
#pragma unroll
            for (uint32_t r = 0; r < kTilePer / 2; ++r) {
                if ((r << (kTileLog + 1)) >= T) break;
                if (2 * (tid + (r << kTileLog)) >= T) continue;
                const uint32_t j = 2 * (tid + (r << kTileLog));
                *reinterpret_cast<float4*>(tile + j) = make_float4(vv[2 * r].x, vv[2 * r].y, vv[2 * r + 1].x, vv[2 * r + 1].y);
            }
        } else {
#pragma unroll
            for (uint32_t r = 0; r < kTilePer; ++r) {
                if ((r << kTileLog) >= T) break;
                if (tid + (r << kTileLog) >= T) continue;   // tiles smaller than the workgroup
                const uint64_t z = base | zt | tile_hi(g, r);
                if (init) {
                    vv[r].x = z == 0 ? 1 : 0;
                    vv[r].y = 0;
                } else {
                    vv[r] = st[z];
                }
            }
#pragma unroll
            for (uint32_t r = 0; r < kTilePer; ++r) {
                if ((r << kTileLog) >= T) break;
                if (tid + (r << kTileLog) >= T) continue;
                tile[tid + (r << kTileLog)] = vv[r];
            }
        }
        __syncthreads();
        constexpr uint32_t kU = sizeof(V) > 8 ? 2u : 8u;
        for (uint32_t i = 0; i < g.n_ops;) {
            const LdsOp o = ops[i];
            if (o.kind == OP_IDENT) {   // uniform: no barrier needed
                ++i;
                continue;
            }
            // a run of diagonal operators (this trajectory's, so uniform) in one pass
            uint32_t j = i + 1;
            if (op_is_diagonal(o)) {
                while (j < g.n_ops && op_is_diagonal(ops[j])) ++j;
                if (j - i > 1) apply_lds_diag_run<V, kU>(tile, T, ops + i, j - i, vals, tid, kTileThreads);
                else apply_lds_op<V, kU>(tile, T, o, vals, tid, kTileThreads);
                __syncthreads();
                i = j;
                continue;
            }
            // up to three one-qubit dense operators on distinct qubits (identities
            // between them skipped) in one pass
            if (o.kind == OP_DENSE1) {
                constexpr int kMaxRun = sizeof(V) > 8 ? 2 : 3;   // complex128: registers for 2
                uint32_t j1 = 0, j2 = 0;   // the run's second and third operator
                int cnt = 1;
                uint32_t used = 1u << o.q0;
                for (; j < g.n_ops && cnt < kMaxRun; ++j) {
                    const LdsOp& n2 = ops[j];
                    if (n2.kind == OP_IDENT) continue;
                    if (n2.kind != OP_DENSE1 || ((used >> n2.q0) & 1u)) break;
                    used |= 1u << n2.q0;
                    if (cnt == 1) j1 = j;
                    else j2 = j;
                    ++cnt;
                }
                if (cnt == 3) apply_lds_dense1_run<V, 3>(tile, T, o, ops[j1], ops[j2], vals, tid, kTileThreads);
                else if (cnt == 2) apply_lds_dense1_run<V, 2>(tile, T, o, ops[j1], o, vals, tid, kTileThreads);
                else apply_lds_op<V, kU>(tile, T, o, vals, tid, kTileThreads);
                __syncthreads();
                i = j;
                continue;
            }
            apply_lds_op<V, kU>(tile, T, o, vals, tid, kTileThreads);
            __syncthreads();
            i = j;
        }
        if constexpr (kPairs) {
#pragma unroll
            for (uint32_t r = 0; r < kTilePer / 2; ++r) {
                if ((r << (kTileLog + 1)) >= T) break;
                if (2 * (tid + (r << kTileLog)) >= T) continue;
                const float4 w = *reinterpret_cast<const float4*>(tile + 2 * (tid + (r << kTileLog)));
                vv[2 * r].x = w.x; vv[2 * r].y = w.y; vv[2 * r + 1].x = w.z; vv[2 * r + 1].y = w.w;
            }
#pragma unroll
            for (uint32_t r = 0; r < kTilePer / 2; ++r) {
                if ((r << (kTileLog + 1)) >= T) break;
                if (2 * (tid + (r << kTileLog)) >= T) continue;
                *reinterpret_cast<float4*>(st + (base | zt2 | tile_hi2(g, r))) =
                    make_float4(vv[2 * r].x, vv[2 * r].y, vv[2 * r + 1].x, vv[2 * r + 1].y);
            }
        } else {
#pragma unroll
            for (uint32_t r = 0; r < kTilePer; ++r) {
                if ((r << kTileLog) >= T) break;
                if (tid + (r << kTileLog) >= T) continue;
                vv[r] = tile[tid + (r << kTileLog)];
            }
#pragma unroll
            for (uint32_t r = 0; r < kTilePer; ++r) {
                if ((r << kTileLog) >= T) break;
                if (tid + (r << kTileLog) >= T) continue;
                st[base | zt | tile_hi(g, r)] = vv[r];
            }
        }
        __syncthreads();   // the tile is reloaded next round
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

// C(x) = sum_t w_t [x_u != x_v], every term
__device__ __forceinline__ double cut_value(uint64_t x, const uint32_t* __restrict__ uv, const double* __restrict__ w,
                                            uint32_t n_terms) {
    double c = 0.0;
    for (uint32_t t = 0; t < n_terms; ++t)
        if (((x >> uv[2 * t]) ^ (x >> uv[2 * t + 1])) & 1) c += w[t];
    return c;
}

// grid (kEnergySlices, K): slice partials of sum_x |psi(x)|^2 C(x).  A slice
// of whole 256-amplitude rows (n >= 14) is visited by each thread in Gray
// code order of the row index: one bit q of x flips per step, and C changes
// only by the terms on qubit q (adj: per qubit, offsets [n + 1] then term
// indices), so the work per amplitude is the degree of one qubit rather than
// every term; C is recomputed from scratch every 64 steps (binary64 sums of
// +-w_t, so no drift accumulates).
template <class V>
__global__ __launch_bounds__(256) void k_gates_energy(const V* __restrict__ psi, uint32_t n,
                                                      const uint32_t* __restrict__ uv, const double* __restrict__ w,
                                                      uint32_t n_terms, const uint32_t* __restrict__ adj,
                                                      double* __restrict__ part) {
    __shared__ double red[kGateThreads];
    const uint64_t N = 1ull << n;
    const uint64_t per = (N + kEnergySlices - 1) / kEnergySlices;
    const uint64_t a = min<uint64_t>(N, blockIdx.x * per), b = min<uint64_t>(N, a + per);
    const V* base = psi + (uint64_t)blockIdx.y * N;
    double s = 0.0;
    if (per % kGateThreads == 0 && a + per <= N) {
        const uint32_t rows = (uint32_t)(per / kGateThreads);   // a power of two; a is a multiple of per
        uint64_t x = a + threadIdx.x;
        double c = 0.0;
        for (uint32_t k = 0; k < rows; ++k) {
            if (k) {
                const uint32_t q = 8 + __builtin_ctz(k);
                if ((k & 63u) == 0) {
                    x ^= 1ull << q;
                    c = cut_value(x, uv, w, n_terms);
                } else {
                    for (uint32_t e = adj[q]; e < adj[q + 1]; ++e) {
                        const uint32_t t = adj[n + 1 + e];
                        c += (((x >> uv[2 * t]) ^ (x >> uv[2 * t + 1])) & 1) ? -w[t] : w[t];
                    }
                    x ^= 1ull << q;
                }
            } else {
                c = cut_value(x, uv, w, n_terms);
            }
            const V v = base[x];
            s += ((double)v.x * v.x + (double)v.y * v.y) * c;
        }
    } else {
        for (uint64_t x = a + threadIdx.x; x < b; x += kGateThreads) {
            const V v = base[x];
            s += ((double)v.x * v.x + (double)v.y * v.y) * cut_value(x, uv, w, n_terms);
        }
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
    const uint32_t S = (uint32_t)p->sites.size();
    if (p->gate_groups.empty()) {   // no operators: the state stays |0..0>
        const uint32_t grid = (uint32_t)std::min<uint64_t>((N * K + kGateThreads - 1) / kGateThreads, 4096);
        hipLaunchKernelGGL(k_gates_init<V>, dim3(grid), dim3(kGateThreads), 0, s, psi, N * K, n);
        STN_HIP(hipGetLastError());
    }
    bool first = true;
    for (const GateGroup& g : p->gate_groups) {
        const size_t lds = (sizeof(V) << g.nbits) + sizeof(LdsOp) * kGroupMaxOps;
        static bool raised[2] = {false, false};
        if (lds > 64 * 1024 && !raised[sizeof(V) > 8]) {
            STN_HIP(hipFuncSetAttribute((const void*)k_gates_tile<V>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)((sizeof(V) << 13) + sizeof(LdsOp) * kGroupMaxOps)));
            raised[sizeof(V) > 8] = true;
        }
        // about 2048 workgroups in all; each loops over its share of a trajectory's tiles
        const uint32_t nt = 1u << (n - g.nbits);
        const uint32_t chunks = std::max<uint32_t>(1, std::min<uint32_t>(nt, (2048 + K - 1) / K));
        hipLaunchKernelGGL(k_gates_tile<V>, dim3(chunks, K), dim3(kTileThreads), lds, s, psi, n, g, first ? 1 : 0,
                           p->d_gate_group_ops.as<LdsOp>(), vals, p->d_site_ops.as<LdsOp>(),
                           p->d_site_op_off.as<uint32_t>(), b->d_idx.as<uint8_t>(), S);
        STN_HIP(hipGetLastError());
        first = false;
    }
    hipLaunchKernelGGL(k_gates_energy<V>, dim3(kEnergySlices, K), dim3(kGateThreads), 0, s, psi, n,
                       p->d_obs.as<uint32_t>(), p->d_obs_w.as<double>(), (uint32_t)p->obs_u.size(),
                       p->d_obs_adj.as<uint32_t>(), b->d_gates_part.as<double>());
    STN_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gates_energy_sum, dim3((K + kGateThreads - 1) / kGateThreads), dim3(kGateThreads), 0, s,
                       b->d_gates_part.as<double>(), K, b->d_energy.as<double>());
    STN_HIP(hipGetLastError());
}

}  // namespace

// Cuts the operator list into groups whose qubits, with the four lowest
// storage bits (runs of at least 128 bytes), fit one tile; the tile is filled
// up with the lowest remaining storage bits.  Operators keep their order.
void build_gate_groups(stn_plan* p) {
    const uint32_t n = p->n;
    const uint32_t tile_bits = std::min<uint32_t>(n, p->opts.precision == 128 ? 12u : 13u);
    const uint64_t low = n > tile_bits ? 0xFull : (1ull << n) - 1ull;
    p->gate_groups.clear();
    p->gate_group_ops.clear();
    std::vector<LdsOp> cur;
    uint64_t qs = low;
    auto qubits = [&](const LdsOp& o) -> uint64_t {
        switch (o.kind) {
            case OP_DENSE1: case OP_DIAG1: return 1ull << o.q0;
            case OP_DENSE2: case OP_DIAG2: return (1ull << o.q0) | (1ull << o.q1);
            case OP_PAULI: return o.xmask | o.zmask;
            case OP_SITE: {
                const SiteRec& st = p->sites[o.site];
                return (1ull << st.q0) | (st.nq == 2 ? 1ull << st.q1 : 0ull);
            }
            default: return 0;
        }
    };
    auto close = [&]() {
        if (cur.empty()) return;
        GateGroup g{};
        uint64_t tile = qs;
        for (uint32_t q = 0; q < n && (uint32_t)__builtin_popcountll(tile) < tile_bits; ++q) tile |= 1ull << q;
        g.nbits = (uint32_t)__builtin_popcountll(tile);
        for (int q = 0; q < 32; ++q) g.local[q] = 0xFF;
        uint32_t l = 0;
        for (uint32_t q = 0; q < n; ++q)
            if ((tile >> q) & 1ull) {
                g.tb[l] = (uint8_t)q;
                g.local[q] = (uint8_t)l;
                ++l;
            }
        // the kernels move complex64 amplitudes in pairs along tile bit 0
        if (g.tb[0] != 0) fail(STN_E_INVALID, "gate group tile without storage bit 0");
        g.op0 = (uint32_t)p->gate_group_ops.size();
        g.n_ops = (uint32_t)cur.size();
        for (LdsOp o : cur) {
            if (o.kind != OP_SITE) {   // gates on tile-local qubits now; sites are remapped per trajectory
                o.q0 = g.local[o.q0 & 31u] == 0xFF ? 0 : g.local[o.q0 & 31u];
                o.q1 = g.local[o.q1 & 31u] == 0xFF ? 0 : g.local[o.q1 & 31u];
                uint64_t x = 0, z = 0;
                for (uint64_t m = o.xmask; m; m &= m - 1) x |= 1ull << g.local[__builtin_ctzll(m)];
                for (uint64_t m = o.zmask; m; m &= m - 1) z |= 1ull << g.local[__builtin_ctzll(m)];
                o.xmask = x;
                o.zmask = z;
            }
            p->gate_group_ops.push_back(o);
        }
        p->gate_groups.push_back(g);
        cur.clear();
        qs = low;
    };
    for (const LdsOp& o : p->lds_ops) {
        if (o.kind == OP_IDENT) continue;
        const uint64_t q = qubits(o);
        if ((uint32_t)__builtin_popcountll(qs | q) > tile_bits || cur.size() >= kGroupMaxOps) close();
        qs |= q;
        cur.push_back(o);
    }
    close();
}

void upload_gate_groups(stn_plan* p, hipStream_t s) {
    std::vector<LdsOp> ops = p->gate_group_ops;
    ops.push_back(LdsOp{});
    upload(p->d_gate_group_ops, &p->alloc, ops.data(), ops.size() * sizeof(LdsOp), s);
}

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
    // bytes: every group reads and writes each trajectory's state (the first
    // one only writes), and the energy reads it once more
    prof_end(p, STN_K_SV_PASS, s, std::ldexp((double)b->K * elem, (int)n) * 2.0 * (double)p->gate_groups.size(),
             0.0);
}

// loads this file's device code (the runtime does so at the first use of
// one of its kernels)
void warm_code_sv_gates() {
    hipFuncAttributes a{};
    (void)hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_gates_tile<float2>));
}

}  // namespace stn
