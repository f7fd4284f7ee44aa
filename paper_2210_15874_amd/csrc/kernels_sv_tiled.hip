// Tiled HBM statevector contraction for QAOA-structured circuits under Pauli
// noise (Sec. III-G: every noisy circuit of the ensemble is simulated to its
// statevector; the trajectory index is the batch dimension of every launch).
//
// Every trajectory is the noiseless circuit with some rotation angles negated
// (Pauli-frame rewrite, see kernels_sample.hip) followed by a final Pauli
// frame F.  The circuit is H on every qubit, then layers of a diagonal block
// (zz gates, angle = mult * base) and a mixer block (rx per qubit).  The state
// psi[b][z] (complex64) is updated in place by passes over tiles of 2^14 or
// 2^15 amplitudes: 14 or 15 storage bits vary inside a tile, the others are
// fixed.  The
// planner's schedule (plan.cpp, schedule_tiled) alternates the order of a
// layer's tiles so that one pass can rotate the last tile of layer l, apply
// the diagonal of layer l+1 and rotate the same tile for layer l+1: n = 26,
// p = 4 costs 5 passes per trajectory.
//
// Inside a workgroup (512 threads for 14-qubit tiles, 1024 for 15-qubit ones)
// the tile lives in registers, 32 amplitudes per thread, in three layouts
// exchanged through LDS; in each layout the
// thread's 5 register bits are the qubits it rotates.  A pass runs the
// layouts L0 -> L1 -> L2 for its first segment and L2 -> L1 -> L0 for its
// second.  The diagonal phase exp(-i base m(z)) with integer
// m(z) = sum_e mult_e sigma_e [z_u != z_v] is looked up in a per-layer table
// (binary64 on the host, rounded once); m(z) is split into a per-thread part
// and the contributions of the 5 register bits, so each amplitude costs a few
// integer adds.  An rx(theta) is applied as cos(theta/2) [[1, -i t], [-i t, 1]]
// with t = tan(theta/2), two FMAs per amplitude; the planner keeps |t| <= 1 by
// writing rx(theta) = -i X rx(theta - pi) and moving the X into the Pauli
// frame, and the dropped factor |cos(theta/2)| is restored in the next phase
// table or in the energy.  The first pass generates |+>^n; the last pass
// accumulates sum_z |psi_z|^2 C(z xor F_x) (F flips measured bits) instead of
// storing: FP32 within a thread, binary64 across threads, tiles and
// trajectories.
//
// Half-state plans keep only the amplitudes with qubit n-1 = 0: every
// trajectory's state satisfies psi(~z) = psi(z) (the circuits commute with X
// on all qubits), so psi(z', 1) is read at the complement of z' in the
// stored half.  A tile holding qubit n-1 (as tile bit 13) thus holds its own
// amplitudes and, for qubit n-1 = 1, those of the complemented tile, stored
// in reverse order; only one of each complementary pair of tiles is visited
// (the top fixed bit is 0).  Phases, rotations and the energy see the full
// index z; the energy over the half is doubled.
//
// Tiles that hold only two low storage bits read 32-byte runs; the four
// workgroups that share each 128-byte line get tile indices x, x+8, x+16,
// x+24, which the dispatcher places on the same XCD at the same time, so each
// line comes from HBM once.  14-qubit tiles leave a second tile only two low
// bits at n = 26; 15-qubit tiles leave it four (128-byte runs, whole lines).
// Workgroups are persistent.  14-qubit tiles: either one per CU, prefetching
// the next tile into registers while working on the current one, or two per
// CU with the exchange buffer halved (the launch-shape variants).  15-qubit
// tiles: one 1024-thread workgroup per CU, exchanging through the halved
// (4-byte slot) buffer of the whole tile, 135 KB.
#include <cmath>

#include "stn_internal.h"

namespace stn {

namespace {

constexpr int kQ = 14;          // tile bits (15-qubit tiles: kQ + 1)
constexpr int kThreads = 512;   // 9 thread bits (15-qubit tiles: 1024, 10)
constexpr int kRegs = 32;       // 5 register bits
constexpr int kMaxPhase = 511;  // phase table entries (2M+1) per diagonal
constexpr int kMaxEdges = 512;  // zz gates of the pass's diagonals

// layouts: tile-index bit of each register bit / thread bit
__device__ constexpr int L0R[5] = {0, 10, 11, 12, 13};
__device__ constexpr int L0T[9] = {1, 2, 3, 4, 5, 6, 7, 8, 9};
__device__ constexpr int L1R[5] = {1, 2, 3, 4, 5};
__device__ constexpr int L1T[9] = {0, 6, 7, 8, 9, 10, 11, 12, 13};
__device__ constexpr int L2R[5] = {0, 6, 7, 8, 9};
__device__ constexpr int L2T[9] = {1, 2, 3, 4, 5, 10, 11, 12, 13};
constexpr int hLR[3][5] = {{0, 10, 11, 12, 13}, {1, 2, 3, 4, 5}, {0, 6, 7, 8, 9}};
// 15-qubit tiles (1024 threads): the three layouts' register bits partition
// the tile bits, so tile bit 0 is a register bit in L0 only
__device__ constexpr int M0R[5] = {0, 11, 12, 13, 14};
__device__ constexpr int M0T[10] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10};
__device__ constexpr int M1R[5] = {1, 2, 3, 4, 5};
__device__ constexpr int M1T[10] = {0, 6, 7, 8, 9, 10, 11, 12, 13, 14};
__device__ constexpr int M2R[5] = {6, 7, 8, 9, 10};
__device__ constexpr int M2T[10] = {0, 1, 2, 3, 4, 5, 11, 12, 13, 14};
constexpr int hMR[3][5] = {{0, 11, 12, 13, 14}, {1, 2, 3, 4, 5}, {6, 7, 8, 9, 10}};

// zz gates of one diagonal, split by where their qubits sit in a layout:
// [0] both outside the registers, [1 + r] one in register bit r, [6] both in
// registers (stored as register-bit indices)
struct DiagTab {
    uint32_t off[7], n[7];
    uint32_t ph_off, ph_mid;    // phase table entries [ph_off, ph_off + 2 ph_mid]
};

struct Pass2 {
    uint32_t tb[kQ + 1];        // qubit (storage bit) of tile-index bit i
    uint64_t fixed_mask;        // storage bits outside the tile (half-state: the top one of a mirror tile excluded)
    uint64_t mirror;            // half-state tile holding qubit n-1: 1 << (n-1); else 0
    uint64_t half_mask;         // half-state: 2^(n-1) - 1
    uint32_t share;             // fixed storage bits below the 128-byte line (0..2)
    float amp0;
    int32_t mix_gate[2][3][5];  // [segment][layout][register bit]: rx gate, -1 = none (t = 0)
    float mix_coef[2][3][5];    // tan(theta_eff / 2) before the trajectory's sign
    DiagTab da, db;             // diagonal after the load (layout L0) / between the segments (L2)
    uint32_t w_off, w_n;        // zz weights of da then db: dedges[w_off .. w_off + w_n)
    uint32_t e_off[7], e_n[7];  // observable terms by category w.r.t. the final layout
    double e_scale;             // squared product of the rotation factors since the last diagonal
};

// LDS slot of tile index t: rows of 64 amplitudes shifted by 2 per row within
// a group of 8 rows, groups of 512 padded by 16.  Every layout's accesses
// then hit distinct banks, and the map is additive over disjoint bit sets,
// so a thread's 32 slots are one base address plus immediate offsets.
constexpr int kLdsSlots = 16894;  // pad(2^14 - 1) + 1
__host__ __device__ constexpr uint32_t pad(uint32_t t) { return t + 2u * ((t >> 6) & 7u) + 16u * (t >> 9); }

// The same for the exchange in two halves (real parts, then imaginary parts;
// 4-byte slots), which halves the buffer so that two workgroups fit on a CU.
// In every layout the 32 lanes of a half-wave see tile-bit offsets of
// 2-adic valuations 0..4, i.e. 32 distinct banks of 32.
constexpr int kLdsSlots4 = 16895;  // pad4(2^14 - 1) + 1
__host__ __device__ constexpr uint32_t pad4(uint32_t t) { return t + ((t >> 5) & 1u) + 2u * (t >> 6); }
// 15-qubit tiles exchange through the same map (their half-waves see tile
// bits {1..5}, {0, 6..9} and {0..4}: again 32 distinct banks)
constexpr int kLdsSlots4x15 = 33791;  // pad4(2^15 - 1) + 1
static_assert(pad4(16383) + 1 == kLdsSlots4 && pad4(32767) + 1 == kLdsSlots4x15, "exchange buffer sizes");
// blocks of 2^11 tile indices (one wave's amplitudes in layouts L1 and L2)
// map to disjoint slot ranges 2112 apart in both exchange maps
static_assert(pad(2048) == 2112 && pad(2047) < 2112 && pad4(2048) == 2112 && pad4(2047) < 2112,
              "wave blocks of the exchange maps");

template <const int* T, int NB>
__device__ __forceinline__ uint32_t thread_part(uint32_t tid) {
    uint32_t t = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) t |= ((tid >> b) & 1u) << T[b];
    return t;
}

template <const int* R>
__device__ __forceinline__ uint32_t reg_part(int j) {
    uint32_t t = 0;
#pragma unroll
    for (int r = 0; r < 5; ++r) t |= (uint32_t)((j >> r) & 1) << R[r];
    return t;
}

template <const int* T, int NB>
__device__ __forceinline__ uint64_t storage_thread(const Pass2& P, uint32_t tid) {
    uint64_t z = 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) z |= (uint64_t)((tid >> b) & 1u) << P.tb[T[b]];
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

__device__ __forceinline__ uint32_t bit_of(uint64_t z, int q) {
    return (uint32_t)(q < 32 ? ((uint32_t)z >> q) : ((uint32_t)(z >> 32) >> (q - 32))) & 1u;
}

// Rotate the register bits of layout L in segment S: pairs (j, j | 1<<r) get
// x0' = x0 - i t x1, x1' = x1 - i t x0.  A slot the pass does not rotate runs
// with t = 0 (amplitudes unchanged), so there are no data-dependent branches;
// tile bit 0 sits in two layouts and only its first slot in the segment's
// layout order is compiled (the other is SKIP).
// tt holds this trajectory's signed coefficients of the pass, [S][L][r].
template <int S, int L, int SKIP_R>
__device__ __forceinline__ void mix(float2 (&v)[kRegs], const float* tt) {
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        if (r == SKIP_R) continue;
        const float t = tt[15 * S + 5 * L + r];
#pragma unroll
        for (int j = 0; j < kRegs; ++j) {
            if (j & (1 << r)) continue;
            const float2 a = v[j], b = v[j | (1 << r)];
            v[j] = make_float2(fmaf(t, b.y, a.x), fmaf(-t, b.x, a.y));
            v[j | (1 << r)] = make_float2(fmaf(t, a.y, b.x), fmaf(-t, a.x, b.y));
        }
    }
}

// whether layouts A and B map thread bits 6 and up (the wave bits) to the
// same tile bits
template <const int* A, const int* B, int NB>
__device__ constexpr bool same_wave_bits() {
    for (int b = 6; b < NB; ++b)
        if (A[b] != B[b]) return false;
    return true;
}

// Orders one wave's LDS accesses across its lanes: a wave's LDS operations
// execute in issue order, so wave-scope fences (keeping the compiler from
// moving accesses across) suffice where no other wave touches the slots.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// write registers in layout A, read them back in layout B; TWO: through a
// buffer of 4-byte slots, real parts first.  LOCAL: A and B put the same
// tile bits on the wave bits (thread bits 6 and up), so each wave writes and
// reads only its own block of 2^11 consecutive tile indices, whose slots no
// other wave's slots interleave (both maps add 2112 per block), and no
// workgroup barrier is needed.  TRAIL: a barrier after the last read (not
// needed when the next writes to the buffer are a wave's own block, or
// start with a barrier of their own).
template <bool TWO, int NB, bool LOCAL, bool TRAIL, const int* AR, const int* AT, const int* BR, const int* BT>
__device__ __forceinline__ void exchange(float2 (&v)[kRegs], float* ldsf, uint32_t tid) {
    static_assert(!LOCAL || same_wave_bits<AT, BT, NB>(), "a wave-local exchange needs layouts with the same wave bits");
    auto sync = [] {
        if constexpr (LOCAL) wave_lds_sync();
        else __syncthreads();
    };
    if constexpr (!TWO) {
        float2* lds = reinterpret_cast<float2*>(ldsf);
        float2* wa = lds + pad(thread_part<AT, NB>(tid));
#pragma unroll
        for (int j = 0; j < kRegs; ++j) wa[pad(reg_part<AR>(j))] = v[j];
        sync();
        const float2* rb = lds + pad(thread_part<BT, NB>(tid));
#pragma unroll
        for (int j = 0; j < kRegs; ++j) v[j] = rb[pad(reg_part<BR>(j))];
        if constexpr (TRAIL) sync();
    } else {
        // the bases are recomputed here rather than kept live across the
        // pass (register budget of two workgroups per CU)
        uint32_t ta = pad4(thread_part<AT, NB>(tid)), tb = pad4(thread_part<BT, NB>(tid));
        asm volatile("" : "+v"(ta), "+v"(tb));
        float* wa = ldsf + ta;
        const float* rb = ldsf + tb;
        // the real parts are replaced while the imaginary parts still hold
        // layout A
#pragma unroll
        for (int j = 0; j < kRegs; ++j) wa[pad4(reg_part<AR>(j))] = v[j].x;
        sync();
#pragma unroll
        for (int j = 0; j < kRegs; ++j) v[j].x = rb[pad4(reg_part<BR>(j))];
        sync();
#pragma unroll
        for (int j = 0; j < kRegs; ++j) wa[pad4(reg_part<AR>(j))] = v[j].y;
        sync();
#pragma unroll
        for (int j = 0; j < kRegs; ++j) v[j].y = rb[pad4(reg_part<BR>(j))];
        if constexpr (TRAIL) sync();
    }
}

// Diagonal exp(-i base m(z)) on the registers of the layout whose register
// bits sit at storage bits rs[] and whose other bits form z0.  m6[j] is the
// part of m from zz gates with both qubits on register bits (the same for
// every thread, tabulated once per trajectory by reg_pair_table).
__device__ __forceinline__ void diag(float2 (&v)[kRegs], const DiagTab& D, uint64_t z0, const int4* dedges,
                                     const int* wt, uint32_t w_base, const float2* ph, const int* m6) {
    int C = 0, h[5] = {0, 0, 0, 0, 0};
    for (uint32_t e = 0; e < D.n[0]; ++e) {
        const int4 E = dedges[D.off[0] + e];
        C += (bit_of(z0, E.x) ^ bit_of(z0, E.y)) ? wt[D.off[0] + e - w_base] : 0;
    }
#pragma unroll
    for (int r = 0; r < 5; ++r)
        for (uint32_t e = 0; e < D.n[1 + r]; ++e) {
            const int4 E = dedges[D.off[1 + r] + e];
            const int w = wt[D.off[1 + r] + e - w_base];
            const uint32_t bv = bit_of(z0, E.x);
            C += bv ? w : 0;
            h[r] += bv ? -w : w;
        }
    // in chunks of 8 amplitudes, so that only 8 phases are live at a time
#pragma unroll
    for (int j0 = 0; j0 < kRegs; j0 += 8) {
        int m[8];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const int j = j0 + jj;
            int a = C;
#pragma unroll
            for (int r = 0; r < 5; ++r)
                if (j & (1 << r)) a += h[r];
            m[jj] = a;
        }
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const float2 p = ph[D.ph_mid + m[jj] + m6[j0 + jj]];
            const float2 a = v[j0 + jj];
            v[j0 + jj] = make_float2(p.x * a.x - p.y * a.y, fmaf(p.x, a.y, p.y * a.x));
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// m6[j] of diagonal D for register index j (threads j = 0..31 of the caller)
__device__ __forceinline__ int reg_pair_table(const DiagTab& D, const int4* dedges, const int* wt, uint32_t w_base,
                                              int j) {
    int a = 0;
    for (uint32_t e = 0; e < D.n[6]; ++e) {
        const int4 E = dedges[D.off[6] + e];
        a += (((j >> E.x) ^ (j >> E.y)) & 1) ? wt[D.off[6] + e - w_base] : 0;
    }
    return a;
}

__device__ __forceinline__ uint32_t tile_of(uint32_t x, uint32_t share) {
    if (!share) return x;
    const uint32_t xcd = x & 7u, r = x >> 3;
    const uint32_t j = r & ((1u << share) - 1u), g = ((r >> share) << 3) | xcd;
    return (g << share) | j;
}

// float4 = the amplitude pair of tile bit 0 (storage bit 0): z (bit 0 clear)
// and z | 1.  MIR (a half-state tile holding qubit n-1): where z holds qubit
// n-1 the pair is stored at ~z - 1 and ~z (so in the other order).  Qubit
// n-1 is the top tile bit: register bit 4 of layout L0 (the upper 8 register
// pairs) and the top thread bit of layout L2 (the upper half of the
// workgroup, whole waves).
template <const int* R>
__device__ __forceinline__ uint64_t reg_off(int jp, const Pass2& P, int nbits) {
    uint64_t off = 0;
#pragma unroll
    for (int r = 1; r < 5; ++r)
        if (r <= nbits) off |= (uint64_t)((jp >> (r - 1)) & 1) << P.tb[R[r]];
    return off;
}

template <const int* R, bool MIR>
__device__ __forceinline__ void load_tile(float2 (&v)[kRegs], const float2* st, uint64_t z0, const Pass2& P) {
    if constexpr (!MIR) {
#pragma unroll
        for (int jp = 0; jp < kRegs / 2; ++jp) {
            const float4 w = *reinterpret_cast<const float4*>(st + (z0 | reg_off<R>(jp, P, 4)));
            v[2 * jp] = make_float2(w.x, w.y);
            v[2 * jp + 1] = make_float2(w.z, w.w);
        }
    } else {
        static_assert(R == L0R || R == M0R, "half-state tiles are loaded in layout L0");
        const uint64_t rb = P.half_mask - 1u - z0;   // z0 holds no bit of qubit n-1 in L0
#pragma unroll
        for (int jp = 0; jp < kRegs / 2; ++jp) {
            const uint64_t off = reg_off<R>(jp, P, 3);
            if (jp < 8) {
                const float4 w = *reinterpret_cast<const float4*>(st + (z0 | off));
                v[2 * jp] = make_float2(w.x, w.y);
                v[2 * jp + 1] = make_float2(w.z, w.w);
            } else {
                const float4 w = *reinterpret_cast<const float4*>(st + (rb - off));
                v[2 * jp] = make_float2(w.z, w.w);
                v[2 * jp + 1] = make_float2(w.x, w.y);
            }
        }
    }
}

template <const int* R, bool MIR>
__device__ __forceinline__ void store_tile(const float2 (&v)[kRegs], float2* st, uint64_t z0, const Pass2& P) {
    auto plain = [&](uint64_t zb, int nbits, int j0, int j1) {
#pragma unroll
        for (int jp = 0; jp < kRegs / 2; ++jp) {
            if (jp < j0 || jp >= j1) continue;
            *reinterpret_cast<float4*>(st + (zb | reg_off<R>(jp, P, nbits))) =
                make_float4(v[2 * jp].x, v[2 * jp].y, v[2 * jp + 1].x, v[2 * jp + 1].y);
        }
    };
    auto mirrored = [&](uint64_t rb, int nbits, int j0, int j1) {
#pragma unroll
        for (int jp = 0; jp < kRegs / 2; ++jp) {
            if (jp < j0 || jp >= j1) continue;
            *reinterpret_cast<float4*>(st + (rb - reg_off<R>(jp, P, nbits))) =
                make_float4(v[2 * jp + 1].x, v[2 * jp + 1].y, v[2 * jp].x, v[2 * jp].y);
        }
    };
    if constexpr (!MIR) {
        plain(z0, 4, 0, kRegs / 2);
    } else if constexpr (R == L0R || R == M0R) {
        plain(z0, 3, 0, 8);
        mirrored(P.half_mask - 1u - z0, 3, 8, kRegs / 2);
    } else {
        // layout L2: the wave's threads all hold qubit n-1 = 1, or all 0
        if (__builtin_amdgcn_readfirstlane((uint32_t)((z0 & P.mirror) != 0)))
            mirrored(P.half_mask - 1u - (z0 & P.half_mask), 4, 0, kRegs / 2);
        else
            plain(z0, 4, 0, kRegs / 2);
    }
}

// Layout L2 of 15-qubit tiles: tile bit 0 is a thread bit, so each
// amplitude is stored on its own (8 bytes; the 64 lanes of a wave cover 64
// consecutive tile indices).  The wave's threads all hold qubit n-1 = 1, or
// all 0 (top thread bit).
template <const int* R, bool MIR>
__device__ __forceinline__ void store_tile_elems(const float2 (&v)[kRegs], float2* st, uint64_t z0, const Pass2& P) {
    auto off = [&](int j) {
        uint64_t o = 0;
#pragma unroll
        for (int r = 0; r < 5; ++r) o |= (uint64_t)((j >> r) & 1) << P.tb[R[r]];
        return o;
    };
    if (MIR && __builtin_amdgcn_readfirstlane((uint32_t)((z0 & P.mirror) != 0))) {
        const uint64_t rc = P.half_mask - (z0 & P.half_mask);
#pragma unroll
        for (int j = 0; j < kRegs; ++j) st[rc - off(j)] = v[j];
    } else {
#pragma unroll
        for (int j = 0; j < kRegs; ++j) st[z0 | off(j)] = v[j];
    }
}

// sum_j |v_j|^2 C(z_j xor F_x) for the layout with register storage bits of R
template <const int* R>
__device__ __forceinline__ float energy_part(const float2 (&v)[kRegs], const Pass2& P, uint64_t z0, uint64_t fx,
                                             const int2* eedges, const double* ew) {
    const uint64_t zf = z0 ^ fx;
    uint32_t fr = 0;  // frame bits on the register positions
#pragma unroll
    for (int r = 0; r < 5; ++r) fr |= bit_of(fx, P.tb[R[r]]) << r;
    float C = 0.f, h[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    for (uint32_t e = 0; e < P.e_n[0]; ++e) {
        const int2 E = eedges[P.e_off[0] + e];
        if (bit_of(zf, E.x) ^ bit_of(zf, E.y)) C += (float)ew[P.e_off[0] + e];
    }
#pragma unroll
    for (int r = 0; r < 5; ++r)
        for (uint32_t e = 0; e < P.e_n[1 + r]; ++e) {
            const int2 E = eedges[P.e_off[1 + r] + e];
            const float w = (float)ew[P.e_off[1 + r] + e];
            const uint32_t c = bit_of(zf, E.x) ^ ((fr >> r) & 1u);
            C += c ? w : 0.f;
            h[r] += c ? -w : w;
        }
    float acc = 0.f;
#pragma unroll
    for (int j0 = 0; j0 < kRegs; j0 += 8) {
        float cz[8];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const int j = j0 + jj;
            float a = C;
#pragma unroll
            for (int r = 0; r < 5; ++r)
                if (j & (1 << r)) a += h[r];
            cz[jj] = a;
        }
        for (uint32_t e = 0; e < P.e_n[6]; ++e) {
            const int2 E = eedges[P.e_off[6] + e];
            const float w = (float)ew[P.e_off[6] + e];
            const int flip = (int)(((fr >> E.x) ^ (fr >> E.y)) & 1u);
#pragma unroll
            for (int jj = 0; jj < 8; ++jj)
                cz[jj] += (((((j0 + jj) >> E.x) ^ ((j0 + jj) >> E.y)) & 1) != flip) ? w : 0.f;
        }
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) {
            const float2 a = v[j0 + jj];
            acc = fmaf(fmaf(a.x, a.x, a.y * a.y), cz[jj], acc);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    return acc;
}

// FL bits: 1 = first pass (generate |+>^n), 2 = diagonal after the load,
// 4 = second segment (diagonal + rotations back through L1 to L0),
// 8 = last pass (energy instead of store).
// Workgroup w processes tiles w, w + G, ... (G = grid, a multiple of 32 so
// every workgroup keeps its XCD's share of line-sharing tiles).
// TWO: two resident workgroups per CU (half the LDS, at most 128 registers,
// no prefetch): one workgroup's loads and stores overlap the other's
// arithmetic and exchanges.
template <int Q, int FL, bool TWO, bool MIR>
__global__ __launch_bounds__(Q == 15 ? 2 * kThreads : kThreads, (Q == 14 && TWO) ? 4 : 1) void k_sv_pass(float2* __restrict__ psi, const Pass2 P, uint32_t n,
                                                      uint32_t tiles_log2, uint32_t total,
                                                      const uint32_t* __restrict__ signs, uint32_t words,
                                                      const uint64_t* __restrict__ frame,
                                                      const int4* __restrict__ dedges,
                                                      const float2* __restrict__ phase,
                                                      const int2* __restrict__ eedges,
                                                      const double* __restrict__ ew,
                                                      double* __restrict__ partials) {
    // 15-qubit tiles: 1024 threads, exchange through 4-byte slots, no prefetch
    static_assert(Q == 14 || (Q == 15 && TWO), "15-qubit tiles use the split exchange");
    constexpr int NT = Q == 15 ? 2 * kThreads : kThreads, NB = Q == 15 ? 10 : 9;
    constexpr const int* R0 = Q == 15 ? M0R : L0R;
    constexpr const int* T0 = Q == 15 ? M0T : L0T;
    constexpr const int* R1 = Q == 15 ? M1R : L1R;
    constexpr const int* T1 = Q == 15 ? M1T : L1T;
    constexpr const int* R2 = Q == 15 ? M2R : L2R;
    constexpr const int* T2 = Q == 15 ? M2T : L2T;
    // 14-qubit tiles hold tile bit 0 in the registers of L0 and L2; it is
    // rotated in the segment's first of them
    constexpr int SKIP0 = Q == 15 ? 5 : 0;
    __shared__ __align__(16) float lds[Q == 15 ? kLdsSlots4x15 : (TWO ? kLdsSlots4 : 2 * kLdsSlots)];
    __shared__ uint32_t sg[64];
    __shared__ float2 pha[kMaxPhase], phb[kMaxPhase];
    __shared__ double red[NT / 64];
    __shared__ int wt[kMaxEdges];  // this trajectory's signed multiplicities of the pass's zz gates
    __shared__ float tt[32];       // this trajectory's signed rotation coefficients [segment][layout][r]
    __shared__ int m6[2][kRegs];   // register-pair parts of the two diagonals' m (see diag)
    constexpr bool kInit = FL & 1, kDiagA = FL & 2, kSeg2 = FL & 4, kLast = FL & 8;
    // the next tile is prefetched into registers when they allow it (one
    // segment); two-segment passes load it after finishing the current one
    constexpr bool kPrefetch = !kSeg2 && !TWO;
    const uint32_t tid = threadIdx.x;
    const uint64_t zt0 = storage_thread<T0, NB>(P, tid), zt2 = storage_thread<T2, NB>(P, tid);
    const uint32_t tmask = (1u << tiles_log2) - 1u;

    if (kDiagA)
        for (uint32_t i = tid; i <= 2 * P.da.ph_mid; i += NT) pha[i] = phase[P.da.ph_off + i];
    if (kSeg2)
        for (uint32_t i = tid; i <= 2 * P.db.ph_mid; i += NT) phb[i] = phase[P.db.ph_off + i];

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
        load_tile<R0, MIR>(v, psi + ((size_t)b << n), base | zt0, P);
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
            if (!kInit && kPrefetch) load_tile<R0, MIR>(nx, psi + ((size_t)bn << n), basen | zt0, P);
        }
        if (b != sb) {  // uniform: a new trajectory's signs and zz weights
            __syncthreads();
            for (uint32_t w = tid; w < words; w += NT) sg[w] = signs[(size_t)b * words + w];
            __syncthreads();
            for (uint32_t e = tid; e < P.w_n; e += NT) {
                const int4 E = dedges[P.w_off + e];
                wt[e] = sign_bit(sg, E.w) ? -E.z : E.z;
            }
            if (tid < 30) {
                const int g = (&P.mix_gate[0][0][0])[tid];
                const float c0 = g < 0 ? 0.f : (&P.mix_coef[0][0][0])[tid];
                tt[tid] = (g >= 0 && sign_bit(sg, g)) ? -c0 : c0;
            }
            __syncthreads();
            if (tid < 2 * kRegs) {
                const bool second = tid >= kRegs;
                if (second ? kSeg2 : kDiagA)
                    m6[second][tid % kRegs] =
                        reg_pair_table(second ? P.db : P.da, dedges, wt, P.w_off, (int)(tid % kRegs));
            }
            __syncthreads();
            sb = b;
        }
        float2* st = psi + ((size_t)b << n);

        if (kDiagA) diag(v, P.da, base | zt0, dedges, wt, P.w_off, pha, m6[0]);
        if constexpr (TWO) __builtin_amdgcn_sched_barrier(0);
        mix<0, 0, 5>(v, tt);
        // the previous tile's exchanges may still be reading (wave-local
        // ones their own blocks, the last one of a two-segment pass any
        // block), and this exchange's writes cover every block
        __syncthreads();
        exchange<TWO, NB, false, false, R0, T0, R1, T1>(v, lds, tid);
        mix<0, 1, 5>(v, tt);
        exchange<TWO, NB, true, true, R1, T1, R2, T2>(v, lds, tid);
        mix<0, 2, SKIP0>(v, tt);
        if (kSeg2) {
            if constexpr (TWO) __builtin_amdgcn_sched_barrier(0);
            diag(v, P.db, base | zt2, dedges, wt, P.w_off, phb, m6[1]);
            if constexpr (TWO) __builtin_amdgcn_sched_barrier(0);
            mix<1, 2, 5>(v, tt);
            exchange<TWO, NB, true, true, R2, T2, R1, T1>(v, lds, tid);
            mix<1, 1, 5>(v, tt);
            exchange<TWO, NB, false, false, R1, T1, R0, T0>(v, lds, tid);
            mix<1, 0, SKIP0>(v, tt);
        }

        if (!kLast) {
            if (kSeg2) store_tile<R0, MIR>(v, st, base | zt0, P);
            else if constexpr (Q == 15) store_tile_elems<R2, MIR>(v, st, base | zt2, P);
            else store_tile<R2, MIR>(v, st, base | zt2, P);
        } else {
            const uint64_t fx = frame[2 * (size_t)b];
            const float accf = kSeg2 ? energy_part<R0>(v, P, base | zt0, fx, eedges, ew)
                                     : energy_part<R2>(v, P, base | zt2, fx, eedges, ew);
            double acc = (double)accf;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
            if ((tid & 63) == 0) red[tid >> 6] = acc;
            __syncthreads();
            if (tid == 0) {
                double s = 0.0;
                for (int w = 0; w < NT / 64; ++w) s += red[w];
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
        } else if (kPrefetch) {
#pragma unroll
            for (int j = 0; j < kRegs; ++j) v[j] = nx[j];
        } else {
            load_tile<R0, MIR>(v, psi + ((size_t)b << n), base | zt0, P);
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

typedef void (*PassKernel)(float2*, const Pass2, uint32_t, uint32_t, uint32_t, const uint32_t*, uint32_t,
                           const uint64_t*, const int4*, const float2*, const int2*, const double*, double*);

template <int Q, bool TWO, bool MIR>
PassKernel pass_kernel_of(int fl) {
    static const PassKernel tab[16] = {
        k_sv_pass<Q, 0, TWO, MIR>,  k_sv_pass<Q, 1, TWO, MIR>,  k_sv_pass<Q, 2, TWO, MIR>,  k_sv_pass<Q, 3, TWO, MIR>,
        k_sv_pass<Q, 4, TWO, MIR>,  k_sv_pass<Q, 5, TWO, MIR>,  k_sv_pass<Q, 6, TWO, MIR>,  k_sv_pass<Q, 7, TWO, MIR>,
        k_sv_pass<Q, 8, TWO, MIR>,  k_sv_pass<Q, 9, TWO, MIR>,  k_sv_pass<Q, 10, TWO, MIR>, k_sv_pass<Q, 11, TWO, MIR>,
        k_sv_pass<Q, 12, TWO, MIR>, k_sv_pass<Q, 13, TWO, MIR>, k_sv_pass<Q, 14, TWO, MIR>, k_sv_pass<Q, 15, TWO, MIR>};
    return tab[fl & 15];
}

// q = 15: one 1024-thread workgroup per CU (two is ignored)
PassKernel pass_kernel(uint32_t q, int fl, bool two, bool mir) {
    if (q == 15) return mir ? pass_kernel_of<15, true, true>(fl) : pass_kernel_of<15, true, false>(fl);
    if (mir) return two ? pass_kernel_of<14, true, true>(fl) : pass_kernel_of<14, false, true>(fl);
    return two ? pass_kernel_of<14, true, false>(fl) : pass_kernel_of<14, false, false>(fl);
}

struct TiledTables {
    std::vector<Pass2> passes;
    std::vector<int> flags;
    std::vector<double> flops;   // algorithmic flops per amplitude of each pass
    std::vector<int4> dedges;
    std::vector<cd> phase;
    std::vector<int2> eedges;
    std::vector<double> ew;
};

// register bit of qubit q in a layout of tiles with Q qubits (-1: none)
int reg_index(uint32_t Q, int layout, const uint32_t* tb, uint32_t q) {
    const int (*lr)[5] = Q == 15 ? hMR : hLR;
    for (int r = 0; r < 5; ++r)
        if (tb[lr[layout][r]] == q) return r;
    return -1;
}

// zz gates of layer L by category w.r.t. the register bits of `layout`
DiagTab diag_table(stn_plan* p, TiledTables& T, const Pass2& P, int layer, int layout, double scale) {
    const TiledLayer& L = p->layers[layer];
    if (2 * L.mult_sum + 1 > kMaxPhase) fail(STN_E_UNSUPPORTED, "diagonal block too large for the phase table");
    DiagTab D{};
    std::vector<int4> cat[7];
    for (size_t e = 0; e < L.zz_gates.size(); ++e) {
        const GateRec& g = p->gates[L.zz_gates[e]];
        const int ru = reg_index(p->tile_bits, layout, P.tb, g.q0), rv = reg_index(p->tile_bits, layout, P.tb, g.q1);
        const int mult = L.zz_mult[e], gi = (int)L.zz_gates[e];
        if (ru < 0 && rv < 0) cat[0].push_back({(int)g.q0, (int)g.q1, mult, gi});
        else if (ru >= 0 && rv < 0) cat[1 + ru].push_back({(int)g.q1, 0, mult, gi});
        else if (ru < 0 && rv >= 0) cat[1 + rv].push_back({(int)g.q0, 0, mult, gi});
        else cat[6].push_back({ru, rv, mult, gi});
    }
    for (int c = 0; c < 7; ++c) {
        D.off[c] = (uint32_t)T.dedges.size();
        D.n[c] = (uint32_t)cat[c].size();
        T.dedges.insert(T.dedges.end(), cat[c].begin(), cat[c].end());
    }
    D.ph_off = (uint32_t)T.phase.size();
    D.ph_mid = (uint32_t)L.mult_sum;
    for (int m = -L.mult_sum; m <= L.mult_sum; ++m) T.phase.push_back(scale * std::exp(cd(0, -L.base_angle * m)));
    return D;
}

TiledTables build_tables(stn_plan* p) {
    TiledTables T;
    const uint32_t n = p->n;
    const uint64_t N = 1ull << n;
    double acc_scale = 1.0;
    // segment s visits layouts in this order; tile bit 0 (L0 slot 0 and L2
    // slot 0) is rotated at the first of them
    const int order[2][3] = {{0, 1, 2}, {2, 1, 0}};
    for (auto& ps : p->passes) {
        Pass2 P{};
        int t = 0;
        for (uint32_t q = 0; q < n; ++q)
            if ((ps.tile_mask >> q) & 1) P.tb[t++] = q;
        const uint32_t Q = p->tile_bits;
        if ((Q != 14 && Q != 15) || t != (int)Q || P.tb[0] != 0)
            fail(STN_E_INVALID, "tile must hold 14 or 15 storage bits including bit 0");
        if (p->sv_half) {
            // stored: qubits 0 .. n-2; a tile holding qubit n-1 (tile bit 13)
            // also covers the complemented tile, so its top fixed bit is 0
            const uint64_t Nh = N / 2;
            P.half_mask = Nh - 1;
            P.fixed_mask = (Nh - 1) & ~(uint64_t)ps.tile_mask;
            if ((ps.tile_mask >> (n - 1)) & 1) {
                if (P.tb[Q - 1] != n - 1 || !P.fixed_mask) fail(STN_E_INVALID, "half-state tile layout");
                P.mirror = 1ull << (n - 1);
                P.fixed_mask &= ~(1ull << (63 - __builtin_clzll(P.fixed_mask)));
            }
        } else {
            P.half_mask = ~0ull;
            P.fixed_mask = (N - 1) & ~(uint64_t)ps.tile_mask;
        }
        P.share = (uint32_t)__builtin_popcountll(P.fixed_mask & 0xFull);
        P.amp0 = (float)std::pow(2.0, -0.5 * n);
        int fl = (ps.init ? 1 : 0) | (ps.diag_a >= 0 ? 2 : 0) | (ps.mix2 >= 0 ? 4 : 0) | (ps.last ? 8 : 0);
        if (ps.diag_b >= 0 && ps.mix2 < 0) fail(STN_E_INVALID, "diagonal between segments without a second segment");
        const size_t w0 = T.dedges.size();
        double nmix = 0;
        auto rotations = [&](int seg, int layer, uint32_t mask) {
            uint32_t done = 0;
            for (int li = 0; li < 3; ++li) {
                const int l = order[seg][li];
                for (int r = 0; r < 5; ++r) {
                    P.mix_gate[seg][l][r] = -1;
                    P.mix_coef[seg][l][r] = 0.f;
                    const uint32_t q = P.tb[(Q == 15 ? hMR : hLR)[l][r]];
                    if (layer < 0 || !((mask >> q) & 1) || ((done >> q) & 1)) continue;
                    done |= 1u << q;
                    const int g = p->layers[layer].rx_gate[q];
                    const double th = p->gates[g].theta_eff;
                    const double c = std::cos(th / 2), s = std::sin(th / 2);
                    if (std::abs(s) > std::abs(c) * (1 + 1e-12)) fail(STN_E_INVALID, "rx gate not in reduced form");
                    P.mix_gate[seg][l][r] = g;
                    P.mix_coef[seg][l][r] = (float)(s / c);
                    acc_scale *= std::abs(c);
                    nmix += 1;
                }
            }
            if (layer >= 0 && done != mask) fail(STN_E_INVALID, "pass rotates a qubit outside its tile");
        };
        if (ps.diag_a >= 0) {
            P.da = diag_table(p, T, P, ps.diag_a, 0, acc_scale);
            acc_scale = 1.0;
        }
        rotations(0, ps.mix1, ps.mix1_mask);
        if (ps.mix2 >= 0) {
            P.db = diag_table(p, T, P, ps.diag_b, 2, acc_scale);
            acc_scale = 1.0;
            rotations(1, ps.mix2, ps.mix2_mask);
        } else {
            for (int l = 0; l < 3; ++l)
                for (int r = 0; r < 5; ++r) P.mix_gate[1][l][r] = -1;
        }
        P.w_off = (uint32_t)w0;
        P.w_n = (uint32_t)(T.dedges.size() - w0);
        if (P.w_n > (uint32_t)kMaxEdges) fail(STN_E_UNSUPPORTED, "too many zz gates in one pass");
        if (ps.last) {
            const int layout = ps.mix2 >= 0 ? 0 : 2;
            std::vector<int2> cat[7];
            std::vector<double> cw[7];
            for (size_t t2 = 0; t2 < p->obs_u.size(); ++t2) {
                const uint32_t u = p->obs_u[t2], v = p->obs_v[t2];
                const int ru = reg_index(p->tile_bits, layout, P.tb, u), rv = reg_index(p->tile_bits, layout, P.tb, v);
                int c = 0;
                int2 e{(int)u, (int)v};
                if (ru >= 0 && rv < 0) {
                    c = 1 + ru;
                    e = {(int)v, 0};
                } else if (ru < 0 && rv >= 0) {
                    c = 1 + rv;
                    e = {(int)u, 0};
                } else if (ru >= 0 && rv >= 0) {
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
            // half-state: the visited amplitudes are half of the whole, and
            // their complements carry equal weight and equal cut values
            P.e_scale = acc_scale * acc_scale * (p->sv_half ? 2.0 : 1.0);
        }
        T.passes.push_back(P);
        T.flags.push_back(fl);
        T.flops.push_back(6.0 * nmix + 6.0 * ((ps.diag_a >= 0) + (ps.mix2 >= 0)) + (ps.last ? 4.0 : 0.0));
    }
    return T;
}

struct TiledDevice {
    TiledTables t;
    DevBuf dedges, phase, eedges, ew;
};

}  // namespace

void upload_tiled(stn_plan* p, hipStream_t s) {
    if (p->tiled) return;
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

void launch_sv_tiled(stn_plan* p, stn_batch* b, hipStream_t s) {
    // N: amplitudes stored per trajectory (2^(n-1) for half-state plans)
    const uint32_t n = p->n, ns = p->sv_half ? n - 1 : n;
    const uint64_t N = 1ull << ns;
    const uint32_t Q = p->tile_bits, tiles_log2 = ns - Q;
    if ((Q != 14 && Q != 15) || ns < Q) fail(STN_E_INVALID, "tiled plan without a valid tile width");
    const uint32_t tiles = 1u << tiles_log2;
    const uint32_t B = std::min(p->max_batch, b->K);
    if (b->words > 64) fail(STN_E_UNSUPPORTED, "tiled lowering supports at most 2048 gates");
    if ((uint64_t)B * tiles > 0x7fffffffull) fail(STN_E_UNSUPPORTED, "batch slice too large");
    if (!p->tiled) upload_tiled(p, s);
    auto* d = static_cast<TiledDevice*>(p->tiled);
    p->d_work.ensure(&p->alloc, (size_t)B * N * 8);
    p->d_partials.ensure(&p->alloc, (size_t)B * tiles * 8);
    int dev = 0, cus = 0;
    STN_HIP(hipGetDevice(&dev));
    STN_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // 14-qubit tiles: variant 0: one workgroup per CU; 1: two per CU, the
    // second queued behind the first; 2: two resident per CU (the half-buffer
    // kernels).  15-qubit tiles: one 1024-thread workgroup per CU.  The grid
    // is a multiple of 32 (XCD rounds of line groups).
    const bool big = Q == 15;
    const bool two = !big && p->variant == 2;
    const uint32_t per_cu = (big || p->variant == 0) ? 1u : 2u;
    const uint32_t threads = big ? 2u * kThreads : (uint32_t)kThreads;
    uint32_t grid_max = std::max(32u, (uint32_t)cus / 32u * 32u) * per_cu;
    // a job server may keep some CUs free for other jobs' kernels
    if (p->grid_cap) grid_max = std::min(grid_max, std::max(32u, p->grid_cap * (two ? 2u : 1u) / 32u * 32u));
    for (uint32_t c0 = 0; c0 < b->K; c0 += B) {
        const uint32_t nb = std::min(B, b->K - c0);
        const uint32_t blocks = nb * tiles;
        for (size_t i = 0; i < d->t.passes.size(); ++i) {
            Pass2 P = d->t.passes[i];
            const int fl = d->t.flags[i];
            const uint32_t grid = std::min(grid_max, blocks);
            if (blocks % (8u << P.share) || grid % 32) P.share = 0;  // grouping needs whole XCD rounds
            const double elems = (double)nb * (double)N;
            prof_begin(p, STN_K_SV_PASS, s);
            hipLaunchKernelGGL(pass_kernel(Q, fl, two, P.mirror != 0), dim3(grid), dim3(threads), 0, s, p->d_work.as<float2>(), P, ns,
                               tiles_log2, blocks, b->d_signs.as<uint32_t>() + (size_t)c0 * b->words, b->words,
                               b->d_frame.as<uint64_t>() + 2 * (size_t)c0, d->dedges.as<int4>(),
                               d->phase.as<float2>(), d->eedges.as<int2>(), d->ew.as<double>(),
                               p->d_partials.as<double>());
            STN_HIP(hipGetLastError());
            prof_end(p, STN_K_SV_PASS, s, elems * 8.0 * ((fl & 1 ? 0 : 1) + (fl & 8 ? 0 : 1)),
                     elems * d->t.flops[i]);
        }
        prof_begin(p, STN_K_TILE_SUM, s);
        hipLaunchKernelGGL(k_tile_sum, dim3(nb), dim3(256), 0, s, p->d_partials.as<double>(), tiles,
                           b->d_energy.as<double>() + c0);
        STN_HIP(hipGetLastError());
        prof_end(p, STN_K_TILE_SUM, s, (double)nb * tiles * 8.0 + nb * 8.0, (double)nb * tiles);
    }
}

uint32_t tiled_variants(const stn_plan* p) { return (p->opts.precision == 128 || p->tile_bits == 15) ? 1u : 3u; }

// loads this file's device code (the runtime does so at the first use of
// one of its kernels)
void warm_code_sv_tiled() {
    hipFuncAttributes a{};
    (void)hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_sv_pass<15, 4, true, false>));
}

}  // namespace stn
