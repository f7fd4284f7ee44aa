// Kraus-operator selection (Sec. III-G: one uniform number per channel picks
// a Kraus operator) and the Pauli-frame scan.
//
// k_sample: one thread per (trajectory, site).  The 32-bit draw is word 0 of
//   Philox4x32-10 (Salmon et al., SC'11) with key = job seed and counter
//   (k low, k high, s, 0); the picked index is the number of thresholds
//   T_0..T_{J-2} that are <= r, i.e. min{ j : r < T_j }.
// k_frame: one thread per trajectory.  Walks the gates in order holding the
//   product F of the Pauli errors inserted so far (x / z bit masks, phase
//   dropped).  A Pauli rotation exp(-i theta P/2) that F anticommutes with is
//   equal, after moving F past it, to the rotation by -theta (up to a global
//   phase), so its sign bit is set; F itself moves unchanged to the end of the
//   circuit (the final frame).  A gate the planner rewrote as a rotation
//   followed by a fixed X (see GateRec::det_x) adds that X to F after the gate.
#include "stn_internal.h"

namespace stn {

namespace {

constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(kM0, c.x), lo0 = kM0 * c.x;
        const uint32_t hi1 = __umulhi(kM1, c.z), lo1 = kM1 * c.z;
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
        k.x += kW0;
        k.y += kW1;
    }
    return c;
}

__global__ __launch_bounds__(256) void k_sample(uint8_t* __restrict__ idx, const uint64_t* __restrict__ T,
                                                const uint32_t* __restrict__ off, uint32_t S, uint64_t total,
                                                uint64_t k0, uint64_t seed) {
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= total) return;
    const uint64_t k = k0 + t / S;
    const uint32_t s = (uint32_t)(t % S);
    const uint4 r4 = philox4x32_10(make_uint4((uint32_t)k, (uint32_t)(k >> 32), s, 0u),
                                   make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
    const uint64_t r = r4.x;
    uint32_t j = 0;
    const uint32_t e = off[s + 1] - 1;
    for (uint32_t o = off[s]; o < e; ++o) j += (r >= T[o]) ? 1u : 0u;
    idx[t] = (uint8_t)j;
}

__global__ __launch_bounds__(64) void k_frame(const uint8_t* __restrict__ idx, uint32_t S, uint32_t K,
                                              const uint32_t* __restrict__ site_gate,
                                              const uint32_t* __restrict__ off, const uint64_t* __restrict__ px,
                                              const uint64_t* __restrict__ pz, const uint64_t* __restrict__ gx,
                                              const uint64_t* __restrict__ gz,
                                              const uint64_t* __restrict__ dx, uint32_t G, uint32_t words,
                                              uint32_t* __restrict__ signs, uint64_t* __restrict__ frame) {
    const uint32_t k = blockIdx.x * 64 + threadIdx.x;
    if (k >= K) return;
    uint64_t x = 0, z = 0;
    uint32_t s = 0, w = 0;
    const uint8_t* row = idx + (size_t)k * S;
    for (uint32_t g = 0; g < G; ++g) {
        const uint64_t ax = gx[g], az = gz[g];
        const uint32_t anti = (uint32_t)(__popcll((x & az) ^ (z & ax)) & 1);
        w |= anti << (g & 31);
        if ((g & 31) == 31) {
            signs[(size_t)k * words + (g >> 5)] = w;
            w = 0;
        }
        x ^= dx[g];  // deterministic X of a rewritten gate, before the gate's noise
        for (; s < S && site_gate[s] == g; ++s) {
            const uint32_t o = off[s] + row[s];
            x ^= px[o];
            z ^= pz[o];
        }
    }
    if (G & 31) signs[(size_t)k * words + (G >> 5)] = w;
    frame[2 * (size_t)k] = x;
    frame[2 * (size_t)k + 1] = z;
}

}  // namespace

void launch_sample(stn_plan* p, stn_batch* b, uint64_t seed, hipStream_t s) {
    const uint32_t S = (uint32_t)p->sites.size();
    const uint64_t total = (uint64_t)b->K * S;
    if (!total) return;
    const uint64_t blocks = (total + 255) / 256;
    if (blocks > 0x7fffffffull) fail(STN_E_INVALID, "batch too large");
    prof_begin(p, STN_K_SAMPLE, s);
    hipLaunchKernelGGL(k_sample, dim3((uint32_t)blocks), dim3(256), 0, s, b->d_idx.as<uint8_t>(),
                       p->d_site_T.as<uint64_t>(), p->d_site_off.as<uint32_t>(), S, total, b->k0, seed);
    STN_HIP(hipGetLastError());
    prof_end(p, STN_K_SAMPLE, s, (double)total, 0.0);
}

void launch_frame(stn_plan* p, stn_batch* b, hipStream_t s) {
    const uint32_t S = (uint32_t)p->sites.size();
    const uint32_t G = (uint32_t)p->gates.size();
    prof_begin(p, STN_K_FRAME, s);
    hipLaunchKernelGGL(k_frame, dim3((b->K + 63) / 64), dim3(64), 0, s, b->d_idx.as<uint8_t>(), S, b->K,
                       p->d_site_gate.as<uint32_t>(), p->d_site_off.as<uint32_t>(), p->d_site_px.as<uint64_t>(),
                       p->d_site_pz.as<uint64_t>(), p->d_gate_gx.as<uint64_t>(), p->d_gate_gz.as<uint64_t>(),
                       p->d_gate_dx.as<uint64_t>(), G,
                       b->words, b->d_signs.as<uint32_t>(), b->d_frame.as<uint64_t>());
    STN_HIP(hipGetLastError());
    prof_end(p, STN_K_FRAME, s, (double)b->K * (S + 4.0 * b->words + 16.0), 0.0);
}

// loads this file's device code (the runtime does so at the first use of
// one of its kernels)
void warm_code_sample() {
    hipFuncAttributes a{};
    (void)hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_sample));
}

}  // namespace stn
