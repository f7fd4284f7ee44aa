// Ensemble reductions in binary64 (Sec. III-G: the probability vectors phi_k
// are averaged to sigma_approx; here generalised to the full rho_hat and the
// energy <C>).
//
// k_herk:     rho += Psi^T conj(Psi) over a batch of B statevectors, only the
//             64x64 tiles on or above the diagonal (I <= J), on the FP64
//             matrix cores.  With X = [Re Psi^T | Im Psi^T] and
//             Y = [Im Psi^T | -Re Psi^T] (N x 2B, the two parts of each
//             trajectory interleaved), Re rho = X X^T and Im rho = Y X^T: two
//             real rank-2B updates of 16x16 blocks by v_mfma_f64_16x16x4
//             (k = 4: two trajectories per step).  Amplitudes are widened to
//             binary64 before the products; every element has a single writer
//             per launch.
// k_diag:     diag += sum_b |psi_b|^2 in trajectory order.
// k_stats:    mean and standard error of the per-trajectory energies, summed
//             in a fixed order (strided per thread, then a fixed tree), two
//             passes (mean, then squared deviations).
// k_finish_*: mirror the upper triangle (rho_ji = conj(rho_ij), real
//             diagonal) and scale by 1/K into output buffers; the trace of
//             sigma from chunk sums of 2048 values added in chunk order.
// k_cdf_*, k_sample_bits: bitstrings drawn from sigma by inverse transform.
//             The running sums F of the accumulated diagonal are formed in
//             chunks of 2048 values, one workgroup per chunk: chunk totals,
//             their exclusive prefix (one workgroup, runs of totals summed in
//             thread order), then each chunk's sums from its offset.  The
//             order of every addition is fixed by the chunk size alone.  Each
//             sampling workgroup stages F in LDS (up to 2^13 values; larger F
//             is searched where it lies in device memory) and each lane
//             binary-searches the smallest x with F(x) > u F(last), or, when
//             rounding leaves none, the smallest x with F(x) >= u F(last).
//             Every index returned is in range whatever u holds.
#include <mutex>

#include "stn_internal.h"

namespace stn {

namespace {

template <class V> __device__ __forceinline__ double2 widen(V v) { return make_double2((double)v.x, (double)v.y); }

constexpr int kTile = 64;   // output tile edge
constexpr int kChunk = 16;  // trajectories per LDS stage

typedef double d4_t __attribute__((ext_vector_type(4)));

// Operand and result layout of v_mfma_f64_16x16x4_f64 (64 lanes, measured on
// gfx950 with one-hot operands): A (16x4) lane l holds A[l % 16][l / 16];
// B (4x16) lane l holds B[l / 16][l % 16]; D (16x16) lane l, component v
// holds D[l / 16 + 4 v][l % 16].
template <class V>
__global__ __launch_bounds__(256, 4) void k_herk(const V* __restrict__ Psi, uint32_t B, uint32_t N, uint32_t tiles,
                                              double2* __restrict__ rho) {
    // upper-triangle tile pair from the linear block index
    uint32_t t = blockIdx.x, I = 0;
    while (t >= tiles - I) {
        t -= tiles - I;
        ++I;
    }
    const uint32_t J = I + t;
    // staged in the amplitudes' own precision (half the LDS for complex64,
    // so more workgroups fit on a CU) and widened when read
    __shared__ V A[kChunk][kTile];   // rows i0..
    __shared__ V C[kChunk][kTile];   // cols j0..
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t rw = (wave >> 1) * 32, cw = (wave & 1) * 32;   // this wave's 32x32 sub-block
    const uint32_t l16 = lane & 15, k4 = lane >> 4;               // row/col in block, k index
    const uint32_t kb = k4 >> 1, part = k4 & 1;                    // trajectory within the step, re/im
    d4_t re[2][2], im[2][2];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            re[r][c] = d4_t{0.0, 0.0, 0.0, 0.0};
            im[r][c] = d4_t{0.0, 0.0, 0.0, 0.0};
        }
    const uint32_t i0 = I * kTile, j0 = J * kTile;
    for (uint32_t b0 = 0; b0 < B; b0 += kChunk) {
        for (uint32_t e = threadIdx.x; e < kChunk * kTile; e += 256) {
            const uint32_t bb = e / kTile, x = e % kTile;
            const bool ok = b0 + bb < B;
            V za;
            za.x = 0;
            za.y = 0;
            A[bb][x] = (ok && i0 + x < N) ? Psi[(size_t)(b0 + bb) * N + i0 + x] : za;
            C[bb][x] = (ok && j0 + x < N) ? Psi[(size_t)(b0 + bb) * N + j0 + x] : za;
        }
        __syncthreads();
#pragma unroll 2
        for (int bb = 0; bb < kChunk; bb += 2) {
            double ax[2], ay[2], bx[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const double2 a = widen(A[bb + kb][rw + 16 * r + l16]);
                ax[r] = part ? a.y : a.x;      // X[i][k]
                ay[r] = part ? -a.x : a.y;     // Y[i][k]
            }
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const double2 v = widen(C[bb + kb][cw + 16 * c + l16]);
                bx[c] = part ? v.y : v.x;      // X[j][k] as B[k][j]
            }
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    re[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[r], bx[c], re[r][c], 0, 0, 0);
                    im[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(ay[r], bx[c], im[r][c], 0, 0, 0);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint32_t i = i0 + rw + 16 * r + k4 + 4 * v, j = j0 + cw + 16 * c + l16;
                if (i < N && j < N && i <= j) {
                    double2* d = rho + (size_t)i * N + j;
                    double2 o = *d;
                    o.x += re[r][c][v];
                    o.y += im[r][c][v];
                    *d = o;
                }
            }
}

// One thread per basis state (64-thread workgroups, so that small N still
// spreads over many CUs); the sum over trajectories stays in trajectory
// order, with the loads of 8 trajectories issued ahead of their adds.
template <class V>
__global__ __launch_bounds__(64) void k_diag(const V* __restrict__ Psi, uint32_t B, uint32_t N,
                                             double* __restrict__ diag) {
    const uint32_t i = blockIdx.x * 64 + threadIdx.x;
    if (i >= N) return;
    double s = 0.0;
    uint32_t b = 0;
    for (; b + 8 <= B; b += 8) {
        double2 v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = widen(Psi[(size_t)(b + u) * N + i]);
#pragma unroll
        for (int u = 0; u < 8; ++u) s += v[u].x * v[u].x + v[u].y * v[u].y;
    }
    for (; b < B; ++b) {
        const double2 v = widen(Psi[(size_t)b * N + i]);
        s += v.x * v.x + v.y * v.y;
    }
    diag[i] += s;
}

__device__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (uint32_t w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_stats(const double* __restrict__ e, uint64_t K, double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (uint64_t k = threadIdx.x; k < K; k += 256) s += e[k];
    const double mean = block_sum(s, red) / (double)K;
    double v = 0.0;
    for (uint64_t k = threadIdx.x; k < K; k += 256) {
        const double d = e[k] - mean;
        v += d * d;
    }
    const double ss = block_sum(v, red);
    if (threadIdx.x == 0) {
        out[0] = mean;
        out[1] = K > 1 ? sqrt(ss / (double)(K - 1) / (double)K) : 0.0;
    }
}

__global__ __launch_bounds__(256) void k_finish_rho(const double2* __restrict__ rho, uint32_t N, double inv,
                                                    double2* __restrict__ out) {
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)N * N) return;
    const uint32_t i = (uint32_t)(t / N), j = (uint32_t)(t % N);
    double2 v;
    if (i < j) {
        v = rho[t];
    } else if (i > j) {
        v = rho[(size_t)j * N + i];
        v.y = -v.y;
    } else {
        v = make_double2(rho[t].x, 0.0);
    }
    out[t] = make_double2(v.x * inv, v.y * inv);
}

// sigma = diag / K in chunks of 2048 values, one workgroup each (each thread
// 8 consecutive values, summed in order, then the workgroup's fixed tree):
// parts[c] = the chunk's sum
__global__ __launch_bounds__(256) void k_finish_diag(const double* __restrict__ diag, uint32_t N, double inv,
                                                     double* __restrict__ out, double* __restrict__ parts) {
    __shared__ double red[256];
    const uint32_t a = blockIdx.x * 2048u + threadIdx.x * 8u;
    double s = 0.0;
#pragma unroll
    for (uint32_t j = 0; j < 8; ++j)
        if (a + j < N) {
            const double v = diag[a + j] * inv;
            out[a + j] = v;
            s += v;
        }
    const double tr = block_sum(s, red);
    if (threadIdx.x == 0) parts[blockIdx.x] = tr;
}

// trace = the chunk sums in order: contiguous runs per thread, then the fixed tree
__global__ __launch_bounds__(256) void k_finish_trace(const double* __restrict__ parts, uint32_t C,
                                                      double* __restrict__ trace) {
    __shared__ double red[256];
    const uint32_t per = (C + 255) / 256;
    const uint32_t a = min(C, threadIdx.x * per), b = min(C, a + per);
    double s = 0.0;
    for (uint32_t i = a; i < b; ++i) s += parts[i];
    const double tr = block_sum(s, red);
    if (threadIdx.x == 0) *trace = tr;
}

// Running sums in chunks of kCdfChunk values: thread t of chunk c owns the
// kCdfPer consecutive values from c kCdfChunk + t kCdfPer and sums them in
// order; the 256 thread sums of a chunk are offset in thread order.
constexpr uint32_t kCdfThreads = 256;
constexpr uint32_t kCdfPer = 8;
constexpr uint32_t kCdfChunk = kCdfThreads * kCdfPer;

__device__ __forceinline__ double cdf_thread_sum(const double* __restrict__ diag, uint32_t N, uint32_t a) {
    double s = 0.0;
#pragma unroll
    for (uint32_t j = 0; j < kCdfPer; ++j)
        if (a + j < N) s += diag[a + j];
    return s;
}

// exclusive prefix of the workgroup's thread sums in thread order; returns
// this thread's offset and leaves the workgroup total in *total
__device__ __forceinline__ double cdf_block_offset(double s, double* off, double* total) {
    off[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (uint32_t t = 0; t < kCdfThreads; ++t) {
            const double v = off[t];
            off[t] = r;
            r += v;
        }
        off[kCdfThreads] = r;
    }
    __syncthreads();
    *total = off[kCdfThreads];
    return off[threadIdx.x];
}

// totals[c] = the sum of chunk c
__global__ __launch_bounds__(kCdfThreads) void k_cdf_totals(const double* __restrict__ diag, uint32_t N,
                                                            double* __restrict__ totals) {
    __shared__ double off[kCdfThreads + 1];
    const uint32_t a = blockIdx.x * kCdfChunk + threadIdx.x * kCdfPer;
    double total;
    cdf_block_offset(cdf_thread_sum(diag, N, a), off, &total);
    if (threadIdx.x == 0) totals[blockIdx.x] = total;
}

// totals[0..C) -> exclusive offsets in place: each thread takes a contiguous
// run of chunk totals, the run sums are offset in thread order
__global__ __launch_bounds__(kCdfThreads) void k_cdf_offsets(double* __restrict__ totals, uint32_t C) {
    __shared__ double off[kCdfThreads + 1];
    const uint32_t per = (C + kCdfThreads - 1) / kCdfThreads;
    const uint32_t a = min(C, threadIdx.x * per), b = min(C, a + per);
    double s = 0.0;
    for (uint32_t i = a; i < b; ++i) s += totals[i];
    double total;
    double r = cdf_block_offset(s, off, &total);
    for (uint32_t i = a; i < b; ++i) {
        const double v = totals[i];
        totals[i] = r;
        r += v;
    }
}

// cdf[x] = offsets[chunk of x] + the chunk's running sum up to x
__global__ __launch_bounds__(kCdfThreads) void k_cdf_scan(const double* __restrict__ diag, uint32_t N,
                                                          const double* __restrict__ offsets,
                                                          double* __restrict__ cdf) {
    __shared__ double off[kCdfThreads + 1];
    const uint32_t a = blockIdx.x * kCdfChunk + threadIdx.x * kCdfPer;
    double total;
    double r = offsets[blockIdx.x] + cdf_block_offset(cdf_thread_sum(diag, N, a), off, &total);
#pragma unroll
    for (uint32_t j = 0; j < kCdfPer; ++j)
        if (a + j < N) {
            r += diag[a + j];
            cdf[a + j] = r;
        }
}

// Smallest x with F[x] > t over N = 2^n sums (N when none): the count of sums
// <= t, found by binary lifting (n dependent LDS reads, no divergence).
__device__ __forceinline__ uint32_t count_le(const double* F, uint32_t N, double t) {
    uint32_t pos = 0;
    for (uint32_t bit = N >> 1; bit; bit >>= 1)
        if (F[pos + bit - 1] <= t) pos += bit;
    return F[pos] <= t ? N : pos;
}

constexpr uint32_t kDrawsPerLane = 4;

constexpr uint32_t kSampleLdsMax = 8192;

template <bool kLds>
__global__ __launch_bounds__(256) void k_sample_bits(const double* __restrict__ cdf, uint32_t N,
                                                     const double* __restrict__ u, uint32_t m,
                                                     uint32_t* __restrict__ out) {
    extern __shared__ double lds_F[];
    const double* F = cdf;
    if (kLds) {
        for (uint32_t i = threadIdx.x; i < N; i += 256) lds_F[i] = cdf[i];
        __syncthreads();
        F = lds_F;
    }
    const double total = F[N - 1];
    const uint32_t span = 256 * kDrawsPerLane;
    for (uint64_t j0 = (uint64_t)blockIdx.x * span + threadIdx.x; j0 < m; j0 += (uint64_t)gridDim.x * span) {
        double t[kDrawsPerLane];
#pragma unroll
        for (uint32_t r = 0; r < kDrawsPerLane; ++r) {
            const uint64_t j = j0 + r * 256;
            t[r] = j < m ? u[j] * total : 0.0;
        }
#pragma unroll
        for (uint32_t r = 0; r < kDrawsPerLane; ++r) {
            const uint64_t j = j0 + r * 256;
            uint32_t x = count_le(F, N, t[r]);
            if (x == N) {  // u F(last) rounded up to F(last): the smallest x with F[x] >= t
                uint32_t lo = 0, hi = N - 1;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (F[mid] >= t[r]) hi = mid; else lo = mid + 1;
                }
                x = lo;
            }
            if (j < m) out[j] = x;
        }
    }
}

}  // namespace

// Running sums and chunk offsets for stn_accum_sample_noalloc: 2^20 + 512
// doubles (8 MiB + 4 KiB) per device, held until the process ends.  Host code
// uses only the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[((size_t)1 << kStaticSampleQubits) +
                                                (((size_t)1 << kStaticSampleQubits) + kCdfChunk - 1) / kCdfChunk];

double* static_sample_scratch(hipError_t* err) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double* ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *err = e != hipSuccess ? e : hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            *err = e;
            return nullptr;
        }
        ptr[dev] = static_cast<double*>(a);
    }
    return ptr[dev];
}

size_t sample_bits_scratch(uint32_t n) {
    const size_t N = (size_t)1 << n;
    return (N + (N + kCdfChunk - 1) / kCdfChunk) * sizeof(double);
}

void launch_sample_bits(stn_accum* a, const double* u, uint32_t m, uint32_t* out, double* work, hipStream_t s) {
    const uint32_t N = 1u << a->plan->n;
    const uint32_t C = (N + kCdfChunk - 1) / kCdfChunk;
    double* cdf = work;
    double* totals = work + N;
    hipLaunchKernelGGL(k_cdf_totals, dim3(C), dim3(kCdfThreads), 0, s, a->d_diag.as<double>(), N, totals);
    STN_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_cdf_offsets, dim3(1), dim3(kCdfThreads), 0, s, totals, C);
    STN_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_cdf_scan, dim3(C), dim3(kCdfThreads), 0, s, a->d_diag.as<double>(), N,
                       (const double*)totals, cdf);
    STN_HIP(hipGetLastError());
    const uint32_t blocks = std::min<uint32_t>((m + 256 * kDrawsPerLane - 1) / (256 * kDrawsPerLane), 1024);
    if (N <= kSampleLdsMax)
        hipLaunchKernelGGL(k_sample_bits<true>, dim3(blocks), dim3(256), N * sizeof(double), s, (const double*)cdf,
                           N, u, m, out);
    else
        hipLaunchKernelGGL(k_sample_bits<false>, dim3(blocks), dim3(256), 0, s, (const double*)cdf, N, u, m, out);
    STN_HIP(hipGetLastError());
}

void launch_reduce(stn_plan* p, stn_batch* b, stn_accum* a, hipStream_t s) {
    const uint32_t N = 1u << p->n;
    const bool dbl = p->opts.precision == 128;
    const uint32_t outs = p->opts.outputs;
    if (outs & STN_OUT_RHO) {
        const uint32_t tiles = (N + kTile - 1) / kTile;
        const uint32_t blocks = tiles * (tiles + 1) / 2;
        const double upper = (double)N * (N + 1) / 2;
        prof_begin(p, STN_K_HERK, s);
        if (dbl)
            hipLaunchKernelGGL(k_herk<double2>, dim3(blocks), dim3(256), 0, s, b->d_states.as<double2>(), b->K, N,
                               tiles, a->d_rho.as<double2>());
        else
            hipLaunchKernelGGL(k_herk<float2>, dim3(blocks), dim3(256), 0, s, b->d_states.as<float2>(), b->K, N,
                               tiles, a->d_rho.as<double2>());
        STN_HIP(hipGetLastError());
        prof_end(p, STN_K_HERK, s, (double)b->K * N * (dbl ? 16 : 8) + upper * 32.0, upper * b->K * 8.0);
    }
    if (outs & (STN_OUT_RHO | STN_OUT_DIAG)) {
        prof_begin(p, STN_K_DIAG, s);
        if (dbl)
            hipLaunchKernelGGL(k_diag<double2>, dim3((N + 63) / 64), dim3(64), 0, s, b->d_states.as<double2>(),
                               b->K, N, a->d_diag.as<double>());
        else
            hipLaunchKernelGGL(k_diag<float2>, dim3((N + 63) / 64), dim3(64), 0, s, b->d_states.as<float2>(),
                               b->K, N, a->d_diag.as<double>());
        STN_HIP(hipGetLastError());
        prof_end(p, STN_K_DIAG, s, (double)b->K * N * (dbl ? 16 : 8) + N * 16.0, (double)b->K * N * 4.0);
    }
    if (outs & STN_OUT_ENERGY) {
        // per-trajectory energies into the chunk that holds trajectory k
        uint64_t k = b->k0;
        const uint64_t end = b->k0 + b->K;
        while (k < end) {
            const uint64_t c = k / kEnergyChunk, stop = std::min<uint64_t>(end, (c + 1) * kEnergyChunk);
            STN_HIP(hipMemcpyAsync(a->e_chunks[c].as<double>() + (k % kEnergyChunk),
                                   b->d_energy.as<double>() + (k - b->k0), (stop - k) * 8,
                                   hipMemcpyDeviceToDevice, s));
            k = stop;
        }
    }
}

__global__ __launch_bounds__(256) void k_scatter_energy(const double* __restrict__ src,
                                                        const uint32_t* __restrict__ map, uint32_t K,
                                                        double* __restrict__ dst) {
    const uint32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k < K) dst[k] = src[map[k]];
}

void launch_scatter_energy(const double* src, const uint32_t* map, uint32_t K, double* dst, hipStream_t s) {
    if (!K) return;
    hipLaunchKernelGGL(k_scatter_energy, dim3((K + 255) / 256), dim3(256), 0, s, src, map, K, dst);
    STN_HIP(hipGetLastError());
}

void launch_energy_stats(stn_accum* a, uint64_t K, hipStream_t s) {
    hipLaunchKernelGGL(k_stats, dim3(1), dim3(256), 0, s, a->d_egather.as<double>(), K, a->d_stats.as<double>());
    STN_HIP(hipGetLastError());
}

void launch_finish_dense(stn_accum* a, hipStream_t s) {
    stn_plan* p = a->plan;
    const uint32_t N = 1u << p->n;
    const double inv = a->k_done ? 1.0 / (double)a->k_done : 0.0;
    if (p->opts.outputs & STN_OUT_RHO) {
        const size_t tot = (size_t)N * N;
        hipLaunchKernelGGL(k_finish_rho, dim3((uint32_t)((tot + 255) / 256)), dim3(256), 0, s,
                           a->d_rho.as<double2>(), N, inv, a->d_rho_out.as<double2>());
        STN_HIP(hipGetLastError());
    }
    const uint32_t C = (N + 2047) / 2048;
    a->d_parts.ensure(&a->plan->alloc, (size_t)C * 8);
    hipLaunchKernelGGL(k_finish_diag, dim3(C), dim3(256), 0, s, a->d_diag.as<double>(), N, inv,
                       a->d_diag_out.as<double>(), a->d_parts.as<double>());
    STN_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_finish_trace, dim3(1), dim3(256), 0, s, (const double*)a->d_parts.as<double>(), C,
                       a->d_stats.as<double>() + 2);
    STN_HIP(hipGetLastError());
}

// loads this file's device code (the runtime does so at the first use of
// one of its kernels)
void warm_code_reduce() {
    hipFuncAttributes a{};
    (void)hipFuncGetAttributes(&a, reinterpret_cast<const void*>(k_stats));
}

}  // namespace stn
