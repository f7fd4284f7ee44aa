// Tiled HBM statevector contraction for QAOA-structured circuits under Pauli
// noise (Sec. III-G: every noisy circuit of the ensemble is simulated to its
// statevector; the trajectory index is the batch dimension of every launch).
//
// Every trajectory is the noiseless circuit with some rotation angles negated
// (Pauli-frame rewrite, see kernels_sample.hip) followed by a final Pauli
// frame F.  The circuit is H on every qubit, then layers of a diagonal block
// (zz gates, angle = mult * base) and a mixer block (rx per qubit).  The state
// psi[b][z] (complex64) is updated in place by passes over tiles of 2^14
// amplitudes: 14 storage bits vary inside a tile, the others are fixed.  The
// first pass of a layer holds storage bits 0..13; the next holds bits 0, 1
// and the next 12 high qubits, so a layer of n = 26 qubits costs two passes.
//
// Inside a workgroup (512 threads) the tile lives in registers, 32 amplitudes
// per thread, in three layouts L0 -> L1 -> L2 exchanged through LDS; in each
// layout the thread's 5 register bits are the qubits it rotates.  The diagonal
// phase exp(-i base m(z)) with integer m(z) = sum_e mult_e sigma_e [z_u != z_v]
// is looked up in a per-layer table (binary64 on the host, rounded once);
// m(z) is split into a per-thread part and the contributions of the 5
// register bits, so each amplitude costs a few integer adds.  An rx(theta)
// is applied as cos(theta/2) [[1, -i t], [-i t, 1]] with t = tan(theta/2),
// two FMAs per amplitude; the planner keeps |t| <= 1 by writing
// rx(theta) = -i X rx(theta - pi) and moving the X into the Pauli frame, and
// the dropped factor |cos(theta/2)| is restored in the next pass's phase
// table or in the energy.  The first pass generates |+>^n; the last pass
// accumulates sum_z |psi_z|^2 C(z xor F_x) (F flips measured bits) instead of
// storing: FP32 within a thread, binary64 across threads, tiles and
// trajectories.
//
// Passes whose tile holds only two low storage bits read 32-byte runs; the
// four workgroups that share each 128-byte line are given block indices
// x, x+8, x+16, x+24, which the dispatcher places on the same XCD at the same
// time, so each line is fetched from HBM once and served to the other three
// from that XCD's L2.
#include <cmath>

#include "stn_internal.h"

namespace stn {

namespace {

constexpr int kQ = 14;          // tile bits
constexpr int kThreads = 512;   // 9 thread bits
constexpr int kRegs = 32;       // 5 register bits
constexpr int kMaxPhase = 511;  // phase table entries (2M+1)
constexpr int kMaxEdges = 512;  // zz gates of one diagonal block

// layouts: tile-index bit of each register bit / thread bit
__device__ constexpr int L0R[5] = {0, 10, 11, 12, 13};
__device__ constexpr int L0T[9] = {1, 2, 3, 4, 5, 6, 7, 8, 9};
__device__ constexpr int L1R[5] = {1, 2, 3, 4, 5};
__device__ constexpr int L1T[9] = {0, 6, 7, 8, 9, 10, 11, 12, 13};
__device__ constexpr int L2R[5] = {0, 6, 7, 8, 9};
__device__ constexpr int L2T[9] = {1, 2, 3, 4, 5, 10, 11, 12, 13};
constexpr int hL0R[5] = {0, 10, 11, 12, 13};
constexpr int hL1R[5] = {1, 2, 3, 4, 5};
constexpr int hL2R[5] = {0, 6, 7, 8, 9};

struct Pass2 {
    uint32_t tb[kQ];            // storage bit of tile-index bit i
    uint64_t fixed_mask;        // storage bits outside the tile
    uint32_t share;             // fixed storage bits below the 128-byte line (0..2)
    uint32_t init, last, diag;
    float amp0;
    int32_t mix_gate[3][5];     // per layout and register bit: rx gate, -1 = not rotated here
    float mix_coef[3][5];       // t = tan(theta_eff/2), |t| <= 1, before the trajectory's sign
    uint32_t d_off[7], d_n[7];  // diagonal edges: [0] both endpoints fixed, [1..5] one in register r-1, [6] both in registers
    uint32_t ph_off, ph_mid;    // phase table entries [ph_off, ph_off + 2*ph_mid]
    uint32_t e_off[7], e_n[7];  // observable terms in the same categories w.r.t. L2
    double e_scale;             // squared product of the rotation factors since the last diagonal
};

__device__ __forceinline__ uint32_t swz(uint32_t t) { return t ^ (((t >> 6) & 7u) << 1); }

template <const int* T>
__device__ __forceinline__ uint32_t thread_part(uint32_t tid) {
    uint32_t t = 0;
#pragma unroll
    for (int b = 0; b < 9; ++b) t |= ((tid >> b) & 1u) << T[b];
    return t;
}

template <const int* R>
__device__ __forceinline__ uint32_t reg_part(int j) {
    uint32_t t = 0;
#pragma unroll
    for (int r = 0; r < 5; ++r) t |= (uint32_t)((j >> r) & 1) << R[r];
    return t;
}

template <const int* T>
__device__ __forceinline__ uint64_t storage_thread(const Pass2& P, uint32_t tid) {
    uint64_t z = 0;
#pragma unroll
    for (int b = 0; b < 9; ++b) z |= (uint64_t)((tid >> b) & 1u) << P.tb[T[b]];
    return z;
}

__device__ __forceinline__ uint64_t pdep64(uint64_t v, uint64_t mask) {
    uint64_t r = 0;
    for (uint64_t m = mask; m; m &= m - 1) {
        if (v & 1) r |= m & (~m + 1);
        v >>= 1;
    }
    return r;
}

__device__ __forceinline__ bool sign_bit(const uint32_t* sg, int g) { return (sg[g >> 5] >> (g & 31)) & 1u; }

// rotate register bit r of layout L: pairs (j, j | 1<<r) get
// x0' = x0 - i t x1, x1' = x1 - i t x0 (rx(theta) / cos(theta/2), t = +-tan(theta/2))
template <int L>
__device__ __forceinline__ void mix(float2 (&v)[kRegs], const Pass2& P, const uint32_t* sg) {
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        const int g = P.mix_gate[L][r];
        if (g < 0) continue;
        const float c0 = P.mix_coef[L][r];
        const float t = sign_bit(sg, g) ? -c0 : c0;
#pragma unroll
        for (int j = 0; j < kRegs; ++j) {
            if (j & (1 << r)) continue;
            const float2 a = v[j], b = v[j | (1 << r)];
            v[j] = make_float2(fmaf(t, b.y, a.x), fmaf(-t, b.x, a.y));
            v[j | (1 << r)] = make_float2(fmaf(t, a.y, b.x), fmaf(-t, a.x, b.y));
        }
    }
}

// write registers in layout A, read them back in layout B
template <const int* AR, const int* AT, const int* BR, const int* BT>
__device__ __forceinline__ void exchange(float2 (&v)[kRegs], float2* lds, uint32_t tid) {
    const uint32_t ta = swz(thread_part<AT>(tid));
#pragma unroll
    for (int j = 0; j < kRegs; ++j) lds[ta ^ swz(reg_part<AR>(j))] = v[j];
    __syncthreads();
    const uint32_t tbp = swz(thread_part<BT>(tid));
#pragma unroll
    for (int j = 0; j < kRegs; ++j) v[j] = lds[tbp ^ swz(reg_part<BR>(j))];
    __syncthreads();
}

__device__ __forceinline__ uint32_t tile_of(uint32_t x, uint32_t share) {
    // line-sharing tiles (differing only in the fixed storage bits below the
    // 128-byte line) get indices x, x+8, x+16, x+24: the same XCD, same time
    if (!share) return x;
    const uint32_t xcd = x & 7u, r = x >> 3;
    const uint32_t j = r & ((1u << share) - 1u), g = ((r >> share) << 3) | xcd;
    return (g << share) | j;
}

__device__ __forceinline__ void load_tile(float2 (&v)[kRegs], const float2* st, uint64_t z0, const Pass2& P) {
#pragma unroll
    for (int jp = 0; jp < kRegs / 2; ++jp) {
        uint64_t z = z0;
#pragma unroll
        for (int r = 1; r < 5; ++r) z |= (uint64_t)((jp >> (r - 1)) & 1) << P.tb[L0R[r]];
        const float4 w = *reinterpret_cast<const float4*>(st + z);
        v[2 * jp] = make_float2(w.x, w.y);
        v[2 * jp + 1] = make_float2(w.z, w.w);
    }
}

// Persistent pass kernel: workgroup w processes tiles w, w + G, w + 2G, ...
// (G = grid size, a multiple of 32, so a workgroup stays on its XCD's share of
// line-sharing tiles) and prefetches the next tile's amplitudes into
// registers before working on the current one.
// FL: bit 0 = first pass (generate |+>^n), bit 1 = diagonal at load,
// bit 2 = last pass (energy instead of store)
template <int FL>
__global__ __launch_bounds__(kThreads) void k_sv_pass2(float2* __restrict__ psi, const Pass2 P, uint32_t n,
                                                       uint32_t tiles_log2, uint32_t total,
                                                       const uint32_t* __restrict__ signs, uint32_t words,
                                                       const uint64_t* __restrict__ frame,
                                                       const int4* __restrict__ dedges,
                                                       const float2* __restrict__ phase,
                                                       const int2* __restrict__ eedges,
                                                       const double* __restrict__ ew,
                                                       double* __restrict__ partials) {
    __shared__ float2 lds[1 << kQ];
    __shared__ uint32_t sg[64];
    __shared__ float2 ph[kMaxPhase];
    __shared__ double red[kThreads / 64];
    __shared__ int wt[kMaxEdges];  // this trajectory's signed multiplicities of the pass's zz gates
    constexpr bool kInit = FL & 1, kDiag = FL & 2, kLast = FL & 4;
    const uint32_t tid = threadIdx.x;
    const uint32_t e0 = P.d_off[0], ne = P.d_off[6] + P.d_n[6] - P.d_off[0];
    const uint64_t zt0 = storage_thread<L0T>(P, tid), zt2 = storage_thread<L2T>(P, tid);
    const uint32_t tmask = (1u << tiles_log2) - 1u;

    if (kDiag)
        for (uint32_t i = tid; i <= 2 * P.ph_mid; i += kThreads) ph[i] = phase[P.ph_off + i];

    uint32_t x = blockIdx.x;
    if (x >= total) return;
    uint32_t f = tile_of(x, P.share);
    uint32_t b = f >> tiles_log2;
    uint64_t base = pdep64(f & tmask, P.fixed_mask);
    float2 v[kRegs];
    if (kInit) {
#pragma unroll
        for (int j = 0; j < kRegs; ++j) v[j] = make_float2(P.amp0, 0.f);
    } else {
        load_tile(v, psi + ((size_t)b << n), base | zt0, P);
    }
    uint32_t sb = 0xffffffffu;  // trajectory whose signs are in LDS
    while (true) {
        // prefetch the next tile
        const uint32_t xn = x + gridDim.x;
        const bool more = xn < total;
        uint32_t fn = 0, bn = 0;
        uint64_t basen = 0;
        float2 nx[kRegs];
        if (more) {
            fn = tile_of(xn, P.share);
            bn = fn >> tiles_log2;
            basen = pdep64(fn & tmask, P.fixed_mask);
            if (!kInit) load_tile(nx, psi + ((size_t)bn << n), basen | zt0, P);
        }
        if (b != sb) {  // uniform: a new trajectory's signs and zz weights
            __syncthreads();
            for (uint32_t w = tid; w < words; w += kThreads) sg[w] = signs[(size_t)b * words + w];
            __syncthreads();
            if (kDiag)
                for (uint32_t e = tid; e < ne; e += kThreads) {
                    const int4 E = dedges[e0 + e];
                    wt[e] = sign_bit(sg, E.w) ? -E.z : E.z;
                }
            __syncthreads();
            sb = b;
        }
        float2* st = psi + ((size_t)b << n);

        if (kDiag) {
            const uint64_t z0 = base | zt0;
            int C = 0, h[5] = {0, 0, 0, 0, 0};
            const uint32_t zl = (uint32_t)z0, zh = (uint32_t)(z0 >> 32);
            for (uint32_t e = 0; e < P.d_n[0]; ++e) {
                const int4 E = dedges[P.d_off[0] + e];
                const uint32_t bu = E.x < 32 ? zl >> E.x : zh >> (E.x - 32);
                const uint32_t bv = E.y < 32 ? zl >> E.y : zh >> (E.y - 32);
                C += ((bu ^ bv) & 1u) ? wt[P.d_off[0] + e - e0] : 0;
            }
#pragma unroll
            for (int r = 0; r < 5; ++r)
                for (uint32_t e = 0; e < P.d_n[1 + r]; ++e) {
                    const int4 E = dedges[P.d_off[1 + r] + e];
                    const int w = wt[P.d_off[1 + r] + e - e0];
                    const uint32_t bv = (E.x < 32 ? zl >> E.x : zh >> (E.x - 32)) & 1u;
                    C += bv ? w : 0;
                    h[r] += bv ? -w : w;
                }
            int m[kRegs];
#pragma unroll
            for (int j = 0; j < kRegs; ++j) {
                int a = C;
#pragma unroll
                for (int r = 0; r < 5; ++r)
                    if (j & (1 << r)) a += h[r];
                m[j] = a;
            }
            for (uint32_t e = 0; e < P.d_n[6]; ++e) {
                const int4 E = dedges[P.d_off[6] + e];
                const int w = wt[P.d_off[6] + e - e0];
#pragma unroll
                for (int j = 0; j < kRegs; ++j) m[j] += (((j >> E.x) ^ (j >> E.y)) & 1) ? w : 0;
            }
#pragma unroll
            for (int j = 0; j < kRegs; ++j) {
                const float2 p = ph[P.ph_mid + m[j]];
                const float2 a = v[j];
                v[j] = make_float2(p.x * a.x - p.y * a.y, fmaf(p.x, a.y, p.y * a.x));
            }
        }

        mix<0>(v, P, sg);
        exchange<L0R, L0T, L1R, L1T>(v, lds, tid);
        mix<1>(v, P, sg);
        exchange<L1R, L1T, L2R, L2T>(v, lds, tid);
        mix<2>(v, P, sg);

        const uint64_t z2 = base | zt2;
        if (!kLast) {
#pragma unroll
            for (int jp = 0; jp < kRegs / 2; ++jp) {
                uint64_t z = z2;
#pragma unroll
                for (int r = 1; r < 5; ++r) z |= (uint64_t)((jp >> (r - 1)) & 1) << P.tb[L2R[r]];
                *reinterpret_cast<float4*>(st + z) =
                    make_float4(v[2 * jp].x, v[2 * jp].y, v[2 * jp + 1].x, v[2 * jp + 1].y);
            }
        } else {
            // energy: sum_j |v_j|^2 C(z_j xor F_x), C(z) = sum_t w_t [z_u != z_v];
            // per amplitude in FP32 (cut values are small sums of weights), summed
            // over the thread's 32 amplitudes in FP32, then in binary64
            const uint64_t fx = frame[2 * (size_t)b];
            const uint64_t zf = z2 ^ fx;
            uint32_t fr = 0;  // frame bits on the register positions
#pragma unroll
            for (int r = 0; r < 5; ++r) fr |= (uint32_t)((fx >> P.tb[L2R[r]]) & 1u) << r;
            float C = 0.f, h[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
            for (uint32_t e = 0; e < P.e_n[0]; ++e) {
                const int2 E = eedges[P.e_off[0] + e];
                if (((zf >> E.x) ^ (zf >> E.y)) & 1u) C += (float)ew[P.e_off[0] + e];
            }
#pragma unroll
            for (int r = 0; r < 5; ++r)
                for (uint32_t e = 0; e < P.e_n[1 + r]; ++e) {
                    const int2 E = eedges[P.e_off[1 + r] + e];
                    const float w = (float)ew[P.e_off[1 + r] + e];
                    const int c = (int)(((zf >> E.x) & 1u) ^ ((fr >> r) & 1u));
                    C += c ? w : 0.f;
                    h[r] += c ? -w : w;
                }
            float cz[kRegs];
#pragma unroll
            for (int j = 0; j < kRegs; ++j) {
                float a = C;
#pragma unroll
                for (int r = 0; r < 5; ++r)
                    if (j & (1 << r)) a += h[r];
                cz[j] = a;
            }
            for (uint32_t e = 0; e < P.e_n[6]; ++e) {
                const int2 E = eedges[P.e_off[6] + e];
                const float w = (float)ew[P.e_off[6] + e];
                const bool flip = ((fr >> E.x) ^ (fr >> E.y)) & 1u;
#pragma unroll
                for (int j = 0; j < kRegs; ++j) cz[j] += ((((j >> E.x) ^ (j >> E.y)) & 1) != (int)flip) ? w : 0.f;
            }
            float accf = 0.f;
#pragma unroll
            for (int j = 0; j < kRegs; ++j) accf = fmaf(fmaf(v[j].x, v[j].x, v[j].y * v[j].y), cz[j], accf);
            double acc = (double)accf;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
            if ((tid & 63) == 0) red[tid >> 6] = acc;
            __syncthreads();
            if (tid == 0) {
                double s = 0.0;
                for (int w = 0; w < kThreads / 64; ++w) s += red[w];
                partials[f] = s * P.e_scale;
            }
        }
        if (!more) break;
        x = xn;
        f = fn;
        b = bn;
        base = basen;
        if (kInit) {
#pragma unroll
            for (int j = 0; j < kRegs; ++j) v[j] = make_float2(P.amp0, 0.f);
        } else {
#pragma unroll
            for (int j = 0; j < kRegs; ++j) v[j] = nx[j];
        }
    }
}

// energy[b] = sum over the trajectory's tiles of partials, in tile order
__global__ __launch_bounds__(256) void k_tile_sum(const double* __restrict__ partials, uint32_t tiles,
                                                  double* __restrict__ energy) {
    __shared__ double red[256];
    const uint32_t b = blockIdx.x;
    double s = 0.0;
    for (uint32_t t = threadIdx.x; t < tiles; t += 256) s += partials[(size_t)b * tiles + t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) energy[b] = red[0];
}

struct TiledTables {
    std::vector<Pass2> passes;
    std::vector<int4> dedges;
    std::vector<cd> phase;
    std::vector<int2> eedges;
    std::vector<double> ew;
};

int reg_index(const int* R, const uint32_t* tb, uint32_t q) {
    for (int r = 0; r < 5; ++r)
        if (tb[R[r]] == q) return r;
    return -1;
}

TiledTables build_tables(stn_plan* p) {
    TiledTables T;
    const uint32_t n = p->n;
    const uint64_t N = 1ull << n;
    double acc_scale = 1.0;
    for (auto& ps : p->passes) {
        Pass2 P{};
        int t = 0;
        for (uint32_t q = 0; q < n; ++q)
            if ((ps.tile_mask >> q) & 1) P.tb[t++] = q;
        if (t != kQ || P.tb[0] != 0) fail(STN_E_INVALID, "tile must hold 14 storage bits including bit 0");
        P.fixed_mask = (N - 1) & ~(uint64_t)ps.tile_mask;
        P.share = (uint32_t)__builtin_popcountll(P.fixed_mask & 0xFull);
        P.init = ps.init;
        P.last = ps.last;
        P.diag = ps.layer >= 0;
        P.amp0 = (float)std::pow(2.0, -0.5 * n);
        // diagonal (layout L0 registers)
        if (P.diag) {
            const TiledLayer& L = p->layers[ps.layer];
            std::vector<int4> cat[7];
            for (size_t e = 0; e < L.zz_gates.size(); ++e) {
                const GateRec& g = p->gates[L.zz_gates[e]];
                const int ru = reg_index(hL0R, P.tb, g.q0), rv = reg_index(hL0R, P.tb, g.q1);
                const int mult = L.zz_mult[e], gi = (int)L.zz_gates[e];
                if (ru < 0 && rv < 0) cat[0].push_back({(int)g.q0, (int)g.q1, mult, gi});
                else if (ru >= 0 && rv < 0) cat[1 + ru].push_back({(int)g.q1, 0, mult, gi});
                else if (ru < 0 && rv >= 0) cat[1 + rv].push_back({(int)g.q0, 0, mult, gi});
                else cat[6].push_back({ru, rv, mult, gi});
            }
            for (int c = 0; c < 7; ++c) {
                P.d_off[c] = (uint32_t)T.dedges.size();
                P.d_n[c] = (uint32_t)cat[c].size();
                T.dedges.insert(T.dedges.end(), cat[c].begin(), cat[c].end());
            }
            if (2 * L.mult_sum + 1 > kMaxPhase || L.zz_gates.size() > (size_t)kMaxEdges)
                fail(STN_E_UNSUPPORTED, "diagonal block too large for the phase table");
            P.ph_off = (uint32_t)T.phase.size();
            P.ph_mid = (uint32_t)L.mult_sum;
            for (int m = -L.mult_sum; m <= L.mult_sum; ++m)
                T.phase.push_back(acc_scale * std::exp(cd(0, -L.base_angle * m)));
            acc_scale = 1.0;
        }
        // rotations: each mixed qubit once, in the first layout holding it in a register
        const int* LR[3] = {hL0R, hL1R, hL2R};
        uint32_t done = 0;
        for (int l = 0; l < 3; ++l)
            for (int r = 0; r < 5; ++r) {
                P.mix_gate[l][r] = -1;
                const uint32_t q = P.tb[LR[l][r]];
                if (!((ps.mix_mask >> q) & 1) || ((done >> q) & 1)) continue;
                done |= 1u << q;
                const int g = p->layers[ps.mix_layer].rx_gate[q];
                const double th = p->gates[g].theta_eff;
                const double c = std::cos(th / 2), s = std::sin(th / 2);
                if (std::abs(s) > std::abs(c) * (1 + 1e-12)) fail(STN_E_INVALID, "rx gate not in reduced form");
                P.mix_gate[l][r] = g;
                P.mix_coef[l][r] = (float)(s / c);
                acc_scale *= std::abs(c);
            }
        if (done != ps.mix_mask) fail(STN_E_INVALID, "pass mixes a qubit outside its tile");
        // observable (layout L2 registers)
        if (P.last) {
            std::vector<int2> cat[7];
            std::vector<double> cw[7];
            for (size_t t2 = 0; t2 < p->obs_u.size(); ++t2) {
                const uint32_t u = p->obs_u[t2], v = p->obs_v[t2];
                const int ru = reg_index(hL2R, P.tb, u), rv = reg_index(hL2R, P.tb, v);
                int c = 0;
                int2 e{(int)u, (int)v};
                if (ru < 0 && rv < 0) {
                    c = 0;
                } else if (ru >= 0 && rv < 0) {
                    c = 1 + ru;
                    e = {(int)v, 0};
                } else if (ru < 0 && rv >= 0) {
                    c = 1 + rv;
                    e = {(int)u, 0};
                } else {
                    c = 6;
                    e = {ru, rv};
                }
                cat[c].push_back(e);
                cw[c].push_back(p->obs_w[t2]);
            }
            for (int c = 0; c < 7; ++c) {
                P.e_off[c] = (uint32_t)T.eedges.size();
                P.e_n[c] = (uint32_t)cat[c].size();
                T.eedges.insert(T.eedges.end(), cat[c].begin(), cat[c].end());
                T.ew.insert(T.ew.end(), cw[c].begin(), cw[c].end());
            }
            P.e_scale = acc_scale * acc_scale;
        }
        T.passes.push_back(P);
    }
    return T;
}

struct TiledDevice {
    TiledTables t;
    DevBuf dedges, phase, eedges, ew;
};

}  // namespace

void launch_sv_tiled(stn_plan* p, stn_batch* b, hipStream_t s) {
    const uint32_t n = p->n;
    const uint64_t N = 1ull << n;
    const uint32_t tiles_log2 = n - kQ;
    const uint32_t tiles = 1u << tiles_log2;
    const uint32_t B = std::min(p->max_batch, b->K);
    if (b->words > 64) fail(STN_E_UNSUPPORTED, "tiled lowering supports at most 2048 gates");
    if ((uint64_t)B * tiles > 0x7fffffffull) fail(STN_E_UNSUPPORTED, "batch slice too large");
    if (!p->tiled) {
        auto* d = new TiledDevice();
        p->tiled = d;
        p->tiled_free = [](void* v) { delete static_cast<TiledDevice*>(v); };
        d->t = build_tables(p);
        std::vector<float2> ph32;
        for (auto& c : d->t.phase) ph32.push_back(make_float2((float)c.real(), (float)c.imag()));
        if (d->t.dedges.empty()) d->t.dedges.push_back(int4{0, 0, 0, 0});
        if (ph32.empty()) ph32.push_back(make_float2(0.f, 0.f));
        if (d->t.eedges.empty()) d->t.eedges.push_back(int2{0, 0});
        if (d->t.ew.empty()) d->t.ew.push_back(0.0);
        upload(d->dedges, &p->alloc, d->t.dedges.data(), d->t.dedges.size() * sizeof(int4), s);
        upload(d->phase, &p->alloc, ph32.data(), ph32.size() * sizeof(float2), s);
        upload(d->eedges, &p->alloc, d->t.eedges.data(), d->t.eedges.size() * sizeof(int2), s);
        upload(d->ew, &p->alloc, d->t.ew.data(), d->t.ew.size() * sizeof(double), s);
        STN_HIP(hipStreamSynchronize(s));
    }
    auto* d = static_cast<TiledDevice*>(p->tiled);
    p->d_work.ensure(&p->alloc, (size_t)B * N * 8);
    p->d_partials.ensure(&p->alloc, (size_t)B * tiles * 8);
    int dev = 0, cus = 0;
    STN_HIP(hipGetDevice(&dev));
    STN_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // one resident workgroup per CU, a multiple of 32 (XCD rounds of line groups)
    const uint32_t grid_max = std::max(32u, (uint32_t)cus / 32u * 32u);
    for (uint32_t c0 = 0; c0 < b->K; c0 += B) {
        const uint32_t nb = std::min(B, b->K - c0);
        const uint32_t blocks = nb * tiles;
        for (const Pass2& P0 : d->t.passes) {
            Pass2 P = P0;
            if (blocks % (8u << P.share)) P.share = 0;  // grouping needs whole XCD rounds
            int nmix = 0;
            for (int l = 0; l < 3; ++l)
                for (int r = 0; r < 5; ++r) nmix += P.mix_gate[l][r] >= 0;
            const double elems = (double)nb * (double)N;
            prof_begin(p, STN_K_SV_PASS, s);
            const int fl = (P.init ? 1 : 0) | (P.diag ? 2 : 0) | (P.last ? 4 : 0);
            auto kern = fl == 0 ? k_sv_pass2<0> : fl == 1 ? k_sv_pass2<1> : fl == 2 ? k_sv_pass2<2>
                      : fl == 3 ? k_sv_pass2<3> : fl == 4 ? k_sv_pass2<4> : fl == 5 ? k_sv_pass2<5>
                      : fl == 6 ? k_sv_pass2<6> : k_sv_pass2<7>;
            const uint32_t grid = std::min(grid_max, blocks);
            if (P.share && grid % 32) P.share = 0;
            hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, s, p->d_work.as<float2>(), P, n,
                               tiles_log2, blocks, b->d_signs.as<uint32_t>() + (size_t)c0 * b->words, b->words,
                               b->d_frame.as<uint64_t>() + 2 * (size_t)c0, d->dedges.as<int4>(),
                               d->phase.as<float2>(), d->eedges.as<int2>(), d->ew.as<double>(),
                               p->d_partials.as<double>());
            STN_HIP(hipGetLastError());
            prof_end(p, STN_K_SV_PASS, s, elems * 8.0 * ((P.init ? 0 : 1) + (P.last ? 0 : 1)),
                     elems * (6.0 * nmix + (P.diag ? 6.0 : 0.0) + (P.last ? 4.0 : 0.0)));
        }
        prof_begin(p, STN_K_TILE_SUM, s);
        hipLaunchKernelGGL(k_tile_sum, dim3(nb), dim3(256), 0, s, p->d_partials.as<double>(), tiles,
                           b->d_energy.as<double>() + c0);
        STN_HIP(hipGetLastError());
        prof_end(p, STN_K_TILE_SUM, s, (double)nb * tiles * 8.0 + nb * 8.0, (double)nb * tiles);
    }
}

void launch_lightcone(stn_plan*, stn_batch*, hipStream_t) { fail(STN_E_UNSUPPORTED, "lightcone lowering not built"); }

}  // namespace stn
