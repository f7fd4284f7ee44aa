// Tiled HBM statevector contraction for QAOA-structured circuits under Pauli
// noise (Sec. III-G, with the trajectory index as batch dimension).
//
// Every trajectory is the noiseless circuit with some rotation angles negated
// (Pauli-frame rewrite, see kernels_sample.hip) followed by a final Pauli
// frame F.  The circuit is H on every qubit, then layers of a diagonal block
// (zz gates, angle = mult * base) and a mixer block (rx per qubit).  The state
// psi[b][z] (complex64, z = basis index) is updated in place by passes; a
// pass loads a tile of 2^13 amplitudes (13 storage bits, the rest fixed) into
// LDS, applies the layer's diagonal phase exp(-i base m(z)) with the integer
// m(z) = sum_e mult_e sigma_e [z_u != z_v] looked up in a table computed in
// binary64 on the host, rotates the tile's qubits with rx(sigma theta), and
// writes the tile back.  The first pass generates |+>^n instead of loading;
// the last pass accumulates the energy sum_z |psi_z|^2 C(z xor F_x) (the frame
// flips measured bits) in binary64 instead of storing.
#include <cmath>

#include "stn_internal.h"

namespace stn {

namespace {

constexpr int kTileBits = 13;
constexpr int kTileN = 1 << kTileBits;
constexpr int kThreads = 256;

struct PassArgs {
    uint32_t n;
    uint32_t tile_bit[kTileBits];  // storage bit of tile index bit t (ascending)
    uint32_t fixed_mask;           // storage bits outside the tile
    int32_t layer;                 // diagonal layer applied at load, -1 = none
    uint32_t edge_off, n_edges, phase_off, mult_sum;
    uint32_t n_mix;
    uint32_t mix_pos[kTileBits];   // tile index bit of each rotated qubit
    int32_t mix_gate[kTileBits];   // its rx gate index
    uint32_t init, last;
    float amp0;                    // 2^{-n/2}
};

__device__ __forceinline__ uint32_t ins0(uint32_t p, uint32_t q) {
    const uint32_t lo = p & ((1u << q) - 1u);
    return ((p ^ lo) << 1) | lo;
}

__device__ __forceinline__ uint64_t pdep64(uint64_t v, uint64_t mask) {
    uint64_t r = 0;
    for (uint64_t m = mask; m; m &= m - 1) {
        const uint64_t bit = m & (~m + 1);
        if (v & 1) r |= bit;
        v >>= 1;
    }
    return r;
}

__global__ __launch_bounds__(kThreads) void k_sv_pass(float2* __restrict__ psi, PassArgs a,
                                                      const uint32_t* __restrict__ signs, uint32_t words,
                                                      const uint64_t* __restrict__ frame,
                                                      const int4* __restrict__ edges,
                                                      const float2* __restrict__ phase,
                                                      const float2* __restrict__ rxcs,
                                                      const uint32_t* __restrict__ obs_uv,
                                                      const double* __restrict__ obs_w, uint32_t n_terms,
                                                      double* __restrict__ partials) {
    __shared__ float2 tile[kTileN];
    __shared__ uint32_t sg[64];
    __shared__ double red[kThreads];
    const uint32_t tid = threadIdx.x;
    const uint32_t b = blockIdx.y;
    const uint64_t N = 1ull << a.n;
    const uint64_t base = pdep64(blockIdx.x, a.fixed_mask);
    float2* st = psi + (size_t)b * N;
    for (uint32_t w = tid; w < words && w < 64; w += kThreads) sg[w] = signs[(size_t)b * words + w];
    __syncthreads();
    for (uint32_t i = tid; i < kTileN; i += kThreads) {
        uint64_t z = base;
#pragma unroll
        for (int t = 0; t < kTileBits; ++t) z |= (uint64_t)((i >> t) & 1) << a.tile_bit[t];
        float2 v = a.init ? make_float2(a.amp0, 0.f) : st[z];
        if (a.layer >= 0) {
            int m = 0;
            for (uint32_t e = 0; e < a.n_edges; ++e) {
                const int4 E = edges[a.edge_off + e];
                const int neg = (sg[E.w >> 5] >> (E.w & 31)) & 1;
                const int cut = (int)(((z >> E.x) ^ (z >> E.y)) & 1);
                m += cut * (neg ? -E.z : E.z);
            }
            const float2 ph = phase[a.phase_off + a.mult_sum + m];
            v = make_float2(ph.x * v.x - ph.y * v.y, ph.x * v.y + ph.y * v.x);
        }
        tile[i] = v;
    }
    __syncthreads();
    for (uint32_t q = 0; q < a.n_mix; ++q) {
        const uint32_t pos = a.mix_pos[q];
        const int32_t g = a.mix_gate[q];
        const float2 cs = rxcs[g];
        const float c = cs.x, s = ((sg[g >> 5] >> (g & 31)) & 1) ? -cs.y : cs.y;
        for (uint32_t p = tid; p < kTileN / 2; p += kThreads) {
            const uint32_t i0 = ins0(p, pos), i1 = i0 | (1u << pos);
            const float2 x0 = tile[i0], x1 = tile[i1];
            // rx: [[c, -i s], [-i s, c]]
            tile[i0] = make_float2(c * x0.x + s * x1.y, c * x0.y - s * x1.x);
            tile[i1] = make_float2(c * x1.x + s * x0.y, c * x1.y - s * x0.x);
        }
        __syncthreads();
    }
    if (a.last) {
        const uint64_t fx = frame[2 * (size_t)b];
        double acc = 0.0;
        for (uint32_t i = tid; i < kTileN; i += kThreads) {
            uint64_t z = base;
#pragma unroll
            for (int t = 0; t < kTileBits; ++t) z |= (uint64_t)((i >> t) & 1) << a.tile_bit[t];
            z ^= fx;
            double c = 0.0;
            for (uint32_t t = 0; t < n_terms; ++t)
                c += ((z >> obs_uv[2 * t]) ^ (z >> obs_uv[2 * t + 1])) & 1 ? obs_w[t] : 0.0;
            const float2 v = tile[i];
            acc += ((double)v.x * v.x + (double)v.y * v.y) * c;
        }
        red[tid] = acc;
        __syncthreads();
        for (uint32_t w = kThreads / 2; w > 0; w >>= 1) {
            if (tid < w) red[tid] += red[tid + w];
            __syncthreads();
        }
        if (tid == 0) partials[(size_t)b * gridDim.x + blockIdx.x] = red[0];
    } else {
        for (uint32_t i = tid; i < kTileN; i += kThreads) {
            uint64_t z = base;
#pragma unroll
            for (int t = 0; t < kTileBits; ++t) z |= (uint64_t)((i >> t) & 1) << a.tile_bit[t];
            st[z] = tile[i];
        }
    }
}

// energy[b] = sum over tiles of partials[b][t], in tile order
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

}  // namespace

void launch_sv_tiled(stn_plan* p, stn_batch* b, hipStream_t s) {
    const uint32_t n = p->n;
    const uint64_t N = 1ull << n;
    const uint32_t tiles = 1u << (n - kTileBits);
    const uint32_t B = std::min(p->max_batch, b->K);
    if (b->words > 64) fail(STN_E_UNSUPPORTED, "tiled lowering supports at most 2048 gates");
    if (B > 65535) fail(STN_E_UNSUPPORTED, "batch slice too large");
    p->d_work.ensure(&p->alloc, (size_t)B * N * 8);
    p->d_partials.ensure(&p->alloc, (size_t)B * tiles * 8);
    std::vector<PassArgs> args;
    for (auto& ps : p->passes) {
        PassArgs a{};
        a.n = n;
        int t = 0;
        for (uint32_t q = 0; q < n; ++q)
            if ((ps.tile_mask >> q) & 1) a.tile_bit[t++] = q;
        if (t != kTileBits) fail(STN_E_INVALID, "tile does not have 13 bits");
        a.fixed_mask = (uint32_t)((N - 1) & ~(uint64_t)ps.tile_mask);
        a.layer = ps.layer;
        if (ps.layer >= 0) {
            a.edge_off = p->layer_edge_off[ps.layer];
            a.n_edges = p->layer_edge_off[ps.layer + 1] - a.edge_off;
            a.phase_off = p->phase_off[ps.layer];
            a.mult_sum = (uint32_t)p->layers[ps.layer].mult_sum;
        }
        a.n_mix = 0;
        for (int tt = 0; tt < kTileBits; ++tt) {
            const uint32_t q = a.tile_bit[tt];
            if ((ps.mix_mask >> q) & 1) {
                a.mix_pos[a.n_mix] = (uint32_t)tt;
                a.mix_gate[a.n_mix] = p->layers[ps.mix_layer].rx_gate[q];
                ++a.n_mix;
            }
        }
        a.init = ps.init;
        a.last = ps.last;
        a.amp0 = (float)std::pow(2.0, -0.5 * n);
        args.push_back(a);
    }
    for (uint32_t c0 = 0; c0 < b->K; c0 += B) {
        const uint32_t nb = std::min(B, b->K - c0);
        for (auto& a : args) {
            const double elems = (double)nb * (double)N;
            prof_begin(p, STN_K_SV_PASS, s);
            hipLaunchKernelGGL(k_sv_pass, dim3(tiles, nb), dim3(kThreads), 0, s, p->d_work.as<float2>(), a,
                               b->d_signs.as<uint32_t>() + (size_t)c0 * b->words, b->words,
                               b->d_frame.as<uint64_t>() + 2 * (size_t)c0, p->d_layer_edges.as<int4>(),
                               p->d_phase32.as<float2>(), p->d_rx32.as<float2>(), p->d_obs.as<uint32_t>(),
                               p->d_obs_w.as<double>(), (uint32_t)p->obs_u.size(), p->d_partials.as<double>());
            STN_HIP(hipGetLastError());
            prof_end(p, STN_K_SV_PASS, s, elems * 8.0 * ((a.init ? 0 : 1) + (a.last ? 0 : 1)),
                     elems * (6.0 * a.n_mix + (a.layer >= 0 ? 6.0 : 0.0) + (a.last ? 4.0 : 0.0)));
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
