// Complex128 twin of the tiled HBM statevector contraction (same circuits:
// H prefix, layers of zz diagonals and rx mixers, Pauli noise as gate signs
// and a final Pauli frame; Sec. III-G).  It exists to state the error of the
// complex64 path at full size and serves binary64 jobs; it is written for
// clarity over speed.
//
// The state psi[b][z] (complex128) is updated in place by passes over tiles of
// 2^12 amplitudes held in LDS (64 KiB).  The pass schedule is the complex64
// path's (alternating tile order, merged layer boundaries) with 12-bit tiles:
// a tile is the low 12 storage bits, or 3 low bits plus up to 9 high ones.
// Gates are applied literally with binary64 coefficients: rx(sigma theta)
// as [[c, -i sigma s], [-i sigma s, c]], and a layer's diagonal as
// exp(-i base m(z)) with the integer m(z) = sum_e mult_e sigma_e [z_u != z_v]
// looked up in a binary64 table.  The last pass accumulates
// sum_z |psi_z|^2 C(z xor F_x) in binary64, in a fixed order.
//
// Half-state plans (psi(~z) = psi(z) for every trajectory of these
// circuits) store only qubit n-1 = 0; a tile holding qubit n-1 (tile bit
// 11) reads and writes its qubit n-1 = 1 amplitudes at the complemented
// index, and only one tile of each complementary pair is visited.  The
// energy over the stored half is doubled.
#include <cmath>

#include "stn_internal.h"

namespace stn {

namespace {

constexpr int kQ128 = 12;
constexpr int kT128 = 512;
constexpr int kTBits = 9;                          // thread bits of the tile index
constexpr int kPerThread = (1 << kQ128) / kT128;   // 8
constexpr int kMaxEdges128 = 1024;

struct Pass128 {
    uint32_t tb[kQ128];         // qubit (storage bit) of tile bit i
    uint64_t fixed_mask;        // storage bits outside the tile (half-state: the top one of a mirror tile excluded)
    uint64_t mirror;            // half-state tile holding qubit n-1: 1 << (n-1); else 0
    uint64_t half_mask;         // half-state: 2^(n-1) - 1; else all ones
    double escale;              // 2 for half-state plans (the complemented half), else 1
    int32_t diag[2];            // layer whose diagonal starts segment s (-1 none)
    int32_t nrot[2];            // rotations of segment s
    int32_t rot_bit[2][kQ128];  // tile bit rotated
    int32_t rot_gate[2][kQ128]; // its rx gate
    uint32_t init, last;
    double amp0;
};

__device__ __forceinline__ uint64_t pdep64_128(uint64_t v, uint64_t mask) {
    uint64_t r = 0;
    for (uint64_t m = mask; m; m &= m - 1) {
        if (v & 1) r |= m & (~m + 1);
        v >>= 1;
    }
    return r;
}

// rx on register bit RB of a thread's 8 elements: [[c, -i s], [-i s, c]]
template <int RB>
__device__ __forceinline__ void rot8(double2 (&v)[8], double c, double sn) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (j & (1 << RB)) continue;
        const double2 a = v[j], w = v[j | (1 << RB)];
        v[j] = make_double2(c * a.x + sn * w.y, c * a.y - sn * w.x);
        v[j | (1 << RB)] = make_double2(sn * a.y + c * w.x, -sn * a.x + c * w.y);
    }
}

// LDS slot of tile index t: bits 0..3 XOR (t4, t5, t6, t6), so that in
// every layout (3 register bits 3k..3k+2, the others from the thread index)
// each 16 consecutive lanes read 16 distinct 16-byte bank groups
__device__ __forceinline__ uint32_t slot128(uint32_t t) { return t ^ ((t >> 4) & 7u) ^ (((t >> 6) & 1u) << 3); }

__device__ __forceinline__ bool flipped(const uint32_t* sg, int g) { return (sg[g >> 5] >> (g & 31)) & 1u; }

// element bit (0..2: tile bits 9..11, the bits of i in t = tid + 512 i)
// holding qubit q, or -1
__device__ __forceinline__ int elem_bit(const Pass128& P, int q) {
    return (uint32_t)q == P.tb[kTBits] ? 0 : (uint32_t)q == P.tb[kTBits + 1] ? 1 : (uint32_t)q == P.tb[kTBits + 2] ? 2 : -1;
}

__global__ __launch_bounds__(kT128) __attribute__((amdgpu_waves_per_eu(4))) void k_sv128_pass(double2* __restrict__ psi, const Pass128 P, uint32_t n,
                                                      uint32_t tiles_log2, const uint32_t* __restrict__ signs,
                                                      uint32_t words, const uint64_t* __restrict__ frame,
                                                      const int4* __restrict__ ledges,
                                                      const uint32_t* __restrict__ lofs,
                                                      const double2* __restrict__ phase,
                                                      const uint32_t* __restrict__ phmid,
                                                      const double2* __restrict__ gcs,
                                                      const int2* __restrict__ oedges,
                                                      const double* __restrict__ ow, uint32_t n_terms,
                                                      double* __restrict__ partials) {
    __shared__ double2 tile[1 << kQ128];
    __shared__ int32_t smult[kMaxEdges128];
    __shared__ double red[kT128];
    const uint32_t tid = threadIdx.x;
    const uint32_t blk = blockIdx.x;
    const uint32_t b = blk >> tiles_log2, f = blk & ((1u << tiles_log2) - 1u);
    const uint64_t base = pdep64_128(f, P.fixed_mask);
    double2* st = psi + ((size_t)b << n);
    const uint32_t* sg = signs + (size_t)b * words;

    // qubit index of tile index t = tid + 512 i: thread part | i part; its
    // storage index: the same, or the complement within the stored half
    // where it holds qubit n-1
    uint64_t zlo = base;
#pragma unroll
    for (int k = 0; k < kTBits; ++k) zlo |= (uint64_t)((tid >> k) & 1u) << P.tb[k];
    // (the element part of the index is uniform: recomputed where used
    // rather than held in registers)
    auto at = [&](int i) -> uint64_t {
        uint64_t z = zlo;
#pragma unroll
        for (int k = 0; k < kQ128 - kTBits; ++k) z |= (uint64_t)((i >> k) & 1) << P.tb[kTBits + k];
        return (z & P.mirror) ? (~z & P.half_mask) : z;
    };

#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
        const uint32_t t = tid + kT128 * i;
        tile[slot128(t)] = P.init ? make_double2(P.amp0, 0.0) : st[at(i)];
    }
    __syncthreads();

    for (int s = 0; s < 2; ++s) {
        const int L = P.diag[s];
        if (L >= 0) {
            const uint32_t e0 = lofs[L], ne = lofs[L + 1] - e0;
            for (uint32_t e = tid; e < ne; e += kT128) {
                const int4 E = ledges[e0 + e];
                smult[e] = flipped(sg, E.w) ? -E.z : E.z;
            }
            __syncthreads();
            const double2* ph = phase + phmid[L];
            // m(z) over the thread's elements: the zz gates whose qubits are
            // both outside the element bits (tile bits 9..11) give a constant,
            // those with one inside a term linear in that bit, those with both
            // inside a term of the bit pair
            int32_t m0 = 0, h[3] = {0, 0, 0}, w2[3] = {0, 0, 0};
            for (uint32_t e = 0; e < ne; ++e) {
                const int4 E = ledges[e0 + e];
                const int32_t w = smult[e];
                const int iu = elem_bit(P, E.x), iv = elem_bit(P, E.y);
                if (iu < 0 && iv < 0) {
                    m0 += (((zlo >> E.x) ^ (zlo >> E.y)) & 1u) ? w : 0;
                } else if (iu < 0 || iv < 0) {
                    const int r = iu < 0 ? iv : iu;
                    const uint32_t other = (uint32_t)(zlo >> (iu < 0 ? E.x : E.y)) & 1u;
                    m0 += other ? w : 0;
                    const int32_t d = other ? -w : w;
                    h[0] += r == 0 ? d : 0;     // (selects, not indexing: the arrays stay in registers)
                    h[1] += r == 1 ? d : 0;
                    h[2] += r == 2 ? d : 0;
                } else {
                    const int pr = iu + iv - 1;  // pairs (0,1), (0,2), (1,2)
                    w2[0] += pr == 0 ? w : 0;
                    w2[1] += pr == 1 ? w : 0;
                    w2[2] += pr == 2 ? w : 0;
                }
            }
#pragma unroll
            for (int i = 0; i < kPerThread; ++i) {
                const uint32_t t = tid + kT128 * i;
                const int b0 = i & 1, b1 = (i >> 1) & 1, b2 = (i >> 2) & 1;
                const int32_t m = m0 + (b0 ? h[0] : 0) + (b1 ? h[1] : 0) + (b2 ? h[2] : 0) +
                                  ((b0 ^ b1) ? w2[0] : 0) + ((b0 ^ b2) ? w2[1] : 0) + ((b1 ^ b2) ? w2[2] : 0);
                const double2 c = ph[m], a = tile[slot128(t)];
                tile[slot128(t)] = make_double2(c.x * a.x - c.y * a.y, c.x * a.y + c.y * a.x);
            }
            __syncthreads();
        }
        // rotations in registers: layout k gives each thread the 8 elements
        // of tile bits 3k .. 3k+2 (its other 9 bits from the thread index)
        for (int k = 0; k < kQ128 / 3; ++k) {
            bool any = false;
            for (int r = 0; r < P.nrot[s]; ++r) any |= P.rot_bit[s][r] / 3 == k;
            if (!any) continue;
            const uint32_t lo = tid & ((1u << (3 * k)) - 1u);
            const uint32_t tbase = lo | ((tid >> (3 * k)) << (3 * k + 3));
            double2 v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = tile[slot128(tbase | ((uint32_t)j << (3 * k)))];
            for (int r = 0; r < P.nrot[s]; ++r) {
                if (P.rot_bit[s][r] / 3 != k) continue;
                const int rb = P.rot_bit[s][r] - 3 * k;
                const int g = P.rot_gate[s][r];
                const double c = gcs[g].x, sn = flipped(sg, g) ? -gcs[g].y : gcs[g].y;
                // rb is uniform (a scalar branch); each case indexes the registers statically
                if (rb == 0) rot8<0>(v, c, sn);
                else if (rb == 1) rot8<1>(v, c, sn);
                else rot8<2>(v, c, sn);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) tile[slot128(tbase | ((uint32_t)j << (3 * k)))] = v[j];
            __syncthreads();
        }
    }

    if (P.last) {
        // C(z xor F_x) split as the diagonal above, on the flipped bits
        const uint64_t fx = frame[2 * (size_t)b];
        const uint64_t zf = zlo ^ fx;
        double c0 = 0.0, hc[3] = {0.0, 0.0, 0.0}, w2c[3] = {0.0, 0.0, 0.0};
        for (uint32_t e = 0; e < n_terms; ++e) {
            const int2 E = oedges[e];
            const double w = ow[e];
            const int iu = elem_bit(P, E.x), iv = elem_bit(P, E.y);
            if (iu < 0 && iv < 0) {
                if (((zf >> E.x) ^ (zf >> E.y)) & 1u) c0 += w;
            } else if (iu < 0 || iv < 0) {
                const int r = iu < 0 ? iv : iu;
                const uint32_t other = (uint32_t)(zf >> (iu < 0 ? E.x : E.y)) & 1u;
                if (other) c0 += w;
                const double d = other ? -w : w;
                hc[0] += r == 0 ? d : 0.0;
                hc[1] += r == 1 ? d : 0.0;
                hc[2] += r == 2 ? d : 0.0;
            } else {
                const int pr = iu + iv - 1;
                w2c[0] += pr == 0 ? w : 0.0;
                w2c[1] += pr == 1 ? w : 0.0;
                w2c[2] += pr == 2 ? w : 0.0;
            }
        }
        uint32_t fi = 0;   // frame bits on the element bits
#pragma unroll
        for (int r = 0; r < kQ128 - kTBits; ++r) fi |= (uint32_t)((fx >> P.tb[kTBits + r]) & 1u) << r;
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < kPerThread; ++i) {
            const uint32_t t = tid + kT128 * i;
            const uint32_t ie = (uint32_t)i ^ fi;
            const int b0 = ie & 1, b1 = (ie >> 1) & 1, b2 = (ie >> 2) & 1;
            const double cz = c0 + (b0 ? hc[0] : 0.0) + (b1 ? hc[1] : 0.0) + (b2 ? hc[2] : 0.0) +
                              ((b0 ^ b1) ? w2c[0] : 0.0) + ((b0 ^ b2) ? w2c[1] : 0.0) + ((b1 ^ b2) ? w2c[2] : 0.0);
            const double2 a = tile[slot128(t)];
            acc += (a.x * a.x + a.y * a.y) * cz;
        }
        red[tid] = acc;
        __syncthreads();
        for (uint32_t w = kT128 / 2; w > 0; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        if (tid == 0) partials[blk] = red[0] * P.escale;
    } else {
#pragma unroll
        for (int i = 0; i < kPerThread; ++i) st[at(i)] = tile[slot128(tid + kT128 * i)];
    }
}

// energy[b] = sum of the trajectory's tile partials, fixed order
__global__ __launch_bounds__(256) void k_tile_sum128(const double* __restrict__ partials, uint32_t tiles,
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

struct Tiled128Device {
    std::vector<Pass128> passes;
    DevBuf ledges, lofs, phase, phmid, gcs, oedges, ow;
};

}  // namespace

uint32_t tiled128_tile_bits() { return kQ128; }

void upload_tiled128(stn_plan* p, hipStream_t s) {
    if (p->tiled) return;
    auto* d = new Tiled128Device();
    p->tiled = d;
    p->tiled_free = [](void* v) { delete static_cast<Tiled128Device*>(v); };
    const uint32_t n = p->n;
    const uint64_t N = n >= 64 ? ~0ull : (1ull << n) - 1;
    std::vector<int4> ledges;
    std::vector<uint32_t> lofs, phmid;
    std::vector<double2> phase;
    for (auto& L : p->layers) {
        lofs.push_back((uint32_t)ledges.size());
        for (size_t e = 0; e < L.zz_gates.size(); ++e) {
            const GateRec& g = p->gates[L.zz_gates[e]];
            ledges.push_back(int4{(int)g.q0, (int)g.q1, L.zz_mult[e], (int)L.zz_gates[e]});
        }
        if (L.zz_gates.size() > (size_t)kMaxEdges128) fail(STN_E_UNSUPPORTED, "too many zz gates in one layer");
        phmid.push_back((uint32_t)phase.size() + (uint32_t)L.mult_sum);
        for (int m = -L.mult_sum; m <= L.mult_sum; ++m) {
            const cd c = std::exp(cd(0, -L.base_angle * m));
            phase.push_back(make_double2(c.real(), c.imag()));
        }
    }
    lofs.push_back((uint32_t)ledges.size());
    std::vector<double2> gcs(p->gates.size() + 1);
    for (size_t g = 0; g < p->gates.size(); ++g)
        gcs[g] = make_double2(std::cos(p->gates[g].theta / 2), std::sin(p->gates[g].theta / 2));
    std::vector<int2> oe;
    for (size_t t = 0; t < p->obs_u.size(); ++t) oe.push_back(int2{(int)p->obs_u[t], (int)p->obs_v[t]});
    std::vector<double> ow = p->obs_w;
    for (auto& ps : p->passes) {
        Pass128 P{};
        int t = 0;
        for (uint32_t q = 0; q < n; ++q)
            if ((ps.tile_mask >> q) & 1) P.tb[t++] = q;
        if (t != kQ128) fail(STN_E_INVALID, "complex128 tile must hold 12 storage bits");
        P.escale = 1.0;
        P.half_mask = ~0ull;
        if (p->sv_half) {
            const uint64_t Nh = (1ull << (n - 1)) - 1;
            P.half_mask = Nh;
            P.escale = 2.0;
            P.fixed_mask = Nh & ~(uint64_t)ps.tile_mask;
            if ((ps.tile_mask >> (n - 1)) & 1) {
                if (P.tb[kQ128 - 1] != n - 1 || !P.fixed_mask) fail(STN_E_INVALID, "half-state tile layout");
                P.mirror = 1ull << (n - 1);
                P.fixed_mask &= ~(1ull << (63 - __builtin_clzll(P.fixed_mask)));
            }
        } else {
            P.fixed_mask = N & ~(uint64_t)ps.tile_mask;
        }
        P.init = ps.init;
        P.last = ps.last;
        P.amp0 = std::pow(2.0, -0.5 * n);
        const int32_t layer[2] = {ps.mix1, ps.mix2};
        const uint32_t mask[2] = {ps.mix1_mask, ps.mix2_mask};
        P.diag[0] = ps.diag_a;
        P.diag[1] = ps.diag_b;
        for (int sgi = 0; sgi < 2; ++sgi) {
            P.nrot[sgi] = 0;
            if (layer[sgi] < 0) continue;
            for (int i = 0; i < kQ128; ++i) {
                const uint32_t q = P.tb[i];
                if (!((mask[sgi] >> q) & 1)) continue;
                const int32_t g = p->layers[layer[sgi]].rx_gate[q];
                if (g < 0) continue;
                P.rot_bit[sgi][P.nrot[sgi]] = i;
                P.rot_gate[sgi][P.nrot[sgi]] = g;
                P.nrot[sgi]++;
            }
        }
        d->passes.push_back(P);
    }
    if (ledges.empty()) ledges.push_back(int4{0, 0, 0, 0});
    if (phase.empty()) phase.push_back(make_double2(1, 0));
    if (phmid.empty()) phmid.push_back(0);
    if (oe.empty()) oe.push_back(int2{0, 0});
    ow.push_back(0.0);
    upload(d->ledges, &p->alloc, ledges.data(), ledges.size() * sizeof(int4), s);
    upload(d->lofs, &p->alloc, lofs.data(), lofs.size() * sizeof(uint32_t), s);
    upload(d->phase, &p->alloc, phase.data(), phase.size() * sizeof(double2), s);
    upload(d->phmid, &p->alloc, phmid.data(), phmid.size() * sizeof(uint32_t), s);
    upload(d->gcs, &p->alloc, gcs.data(), gcs.size() * sizeof(double2), s);
    upload(d->oedges, &p->alloc, oe.data(), oe.size() * sizeof(int2), s);
    upload(d->ow, &p->alloc, ow.data(), ow.size() * sizeof(double), s);
    STN_HIP(hipStreamSynchronize(s));
}

void launch_sv_tiled128(stn_plan* p, stn_batch* b, hipStream_t s) {
    // N: amplitudes stored per trajectory (2^(n-1) for half-state plans)
    const uint32_t n = p->n, ns = p->sv_half ? n - 1 : n;
    const uint64_t N = 1ull << ns;
    const uint32_t tiles_log2 = ns - kQ128;
    const uint32_t tiles = 1u << tiles_log2;
    const uint32_t B = std::min(p->max_batch, b->K);
    if ((uint64_t)B * tiles > 0x7fffffffull) fail(STN_E_UNSUPPORTED, "batch slice too large");
    if (!p->tiled) upload_tiled128(p, s);
    auto* d = static_cast<Tiled128Device*>(p->tiled);
    p->d_work.ensure(&p->alloc, (size_t)B * N * 16);
    p->d_partials.ensure(&p->alloc, (size_t)B * tiles * 8);
    for (uint32_t c0 = 0; c0 < b->K; c0 += B) {
        const uint32_t nb = std::min(B, b->K - c0);
        const uint32_t blocks = nb * tiles;
        for (const Pass128& P : d->passes) {
            const double elems = (double)nb * (double)N;
            prof_begin(p, STN_K_SV_PASS, s);
            hipLaunchKernelGGL(k_sv128_pass, dim3(blocks), dim3(kT128), 0, s, p->d_work.as<double2>(), P, ns,
                               tiles_log2, b->d_signs.as<uint32_t>() + (size_t)c0 * b->words, b->words,
                               b->d_frame.as<uint64_t>() + 2 * (size_t)c0, d->ledges.as<int4>(),
                               d->lofs.as<uint32_t>(), d->phase.as<double2>(), d->phmid.as<uint32_t>(),
                               d->gcs.as<double2>(), d->oedges.as<int2>(), d->ow.as<double>(),
                               (uint32_t)p->obs_u.size(), p->d_partials.as<double>());
            STN_HIP(hipGetLastError());
            prof_end(p, STN_K_SV_PASS, s, elems * 16.0 * ((P.init ? 0 : 1) + (P.last ? 0 : 1)), 0.0);
        }
        prof_begin(p, STN_K_TILE_SUM, s);
        hipLaunchKernelGGL(k_tile_sum128, dim3(nb), dim3(256), 0, s, p->d_partials.as<double>(), tiles,
                           b->d_energy.as<double>() + c0);
        STN_HIP(hipGetLastError());
        prof_end(p, STN_K_TILE_SUM, s, (double)nb * tiles * 8.0 + nb * 8.0, (double)nb * tiles);
    }
}

// loads this file's device code (the runtime does so at the first use of
// one of its kernels)
void warm_code_sv_tiled128() {
    hipFuncAttributes a{};
    (void)hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_sv128_pass));
}

}  // namespace stn
