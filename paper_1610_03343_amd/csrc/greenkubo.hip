// Green-Kubo heat-current autocorrelation and running thermal conductivity
// from the per-step total heat current J = sum_i J_i (the potential part of
// Section 2.3, columns 11..13 of the thermo rows).
//
//   C_a(k)     = 1/(S - k) sum_{t=0}^{S-k-1} J_a(t) J_a(t + k),  a = x, y, z
//   kappa_a(K) = dtau / (k_B T^2 V) [C_a(0)/2 + C_a(1) + ... + C_a(K)/2]
//
// over S samples taken every `every` steps (every time origin is used, each
// lag averaged over its own origin count), in W/(m K).
//
// The correlation is a lag x origin product: a block owns 512 consecutive
// lags, eight per lane (k0 + 8 l + r), and walks a strided set of
// 1024-origin tiles, staging per component the two sample windows it needs
// (J(t) and J(t + k0 ..)) in LDS, zero-padded past the end so no product
// needs a bounds test.  A lane keeps the 16 samples J(t + k0 + 8 l + u),
// u < 16, in registers and slides them eight origins at a time, so each
// staged value it reads feeds eight multiply-adds.  Each lag's sum is split
// over a fixed number of origin groups and over the four waves of the block
// (each wave a contiguous quarter of every tile) in a fixed pattern, and
// the finishing pass adds the partials in order: the result is the same
// bits on every run, without atomics.
#include "mbmd_internal.h"

namespace mbmd {

constexpr int kGkR = 8;                  // consecutive lags per lane
constexpr int kGkLags = 64 * kGkR;       // lags per block
constexpr int kGkOrigins = 1024;         // origins per staged tile
constexpr int kGkWaves = kBlock / 64;
constexpr int kGkWaveOrigins = kGkOrigins / kGkWaves;
// b window index x lives at x + x / 8: a lane's reads (x = 8 l + const)
// then fall 9 doubles apart, which spreads a wave over every LDS bank
__device__ __forceinline__ int gk_pad(int x) { return x + (x >> 3); }
constexpr int kGkBWin = kGkOrigins + kGkLags;
constexpr int kGkBWinPadded = kGkBWin + kGkBWin / 8 + 1;

__global__ void __launch_bounds__(kBlock)
k_gk_compact(const double* __restrict__ thermo, int64_t S, int every, double* __restrict__ jc)
{
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= S) return;
    const double* row = thermo + s * every * kThermoCols;
    jc[s] = row[11];
    jc[S + s] = row[12];
    jc[2 * S + s] = row[13];
}

// part[(g * kGkWaves + wave) * max_lag + k][3]
__global__ void __launch_bounds__(kBlock)
k_gk_corr(const double* __restrict__ jc, int64_t S, int max_lag, double* __restrict__ part)
{
    __shared__ double a_win[kGkOrigins];
    __shared__ double b_win[kGkBWinPadded];
    const int g = blockIdx.x, G = gridDim.x;
    const int k0 = blockIdx.y * kGkLags;
    const int l = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int lb = kGkR * l;                  // this lane's first lag, less k0
    double acc[3][kGkR];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < kGkR; ++r) acc[c][r] = 0.0;
    // origins t with t + k0 < S can pair with a lag of this block
    const int64_t tend = S - k0;
    for (int64_t t0 = (int64_t)g * kGkOrigins; t0 < tend; t0 += (int64_t)G * kGkOrigins) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            __syncthreads();   // the previous window is consumed
            const double* jcc = jc + c * S;
            for (int x = threadIdx.x; x < kGkBWin; x += kBlock) {
                if (x < kGkOrigins) {
                    const int64_t ta = t0 + x;
                    a_win[x] = ta < S ? jcc[ta] : 0.0;
                }
                const int64_t tb = t0 + k0 + x;
                b_win[gk_pad(x)] = tb < S ? jcc[tb] : 0.0;
            }
            __syncthreads();
            // wave q: origins i0 .. i0 + kGkWaveOrigins - 1 of the tile; lag
            // k0 + lb + r pairs J(t0 + i) with b_win[i + lb + r]
            const int i0 = q * kGkWaveOrigins;
            double w0[kGkR], w1[kGkR];
#pragma unroll
            for (int u = 0; u < kGkR; ++u) w0[u] = b_win[gk_pad(i0 + lb + u)];
            for (int i = i0; i < i0 + kGkWaveOrigins; i += 2 * kGkR) {
                // w0 = b[i + lb ..], w1 = b[i + lb + 8 ..]; then w1, w0 for i + 8
#pragma unroll
                for (int u = 0; u < kGkR; ++u) w1[u] = b_win[gk_pad(i + lb + kGkR + u)];
#pragma unroll
                for (int u = 0; u < kGkR; ++u) {
                    const double av = a_win[i + u];
#pragma unroll
                    for (int r = 0; r < kGkR; ++r)
                        acc[c][r] = fma(av, u + r < kGkR ? w0[u + r] : w1[u + r - kGkR],
                                        acc[c][r]);
                }
#pragma unroll
                for (int u = 0; u < kGkR; ++u)
                    w0[u] = b_win[gk_pad(i + lb + 2 * kGkR + u)];
#pragma unroll
                for (int u = 0; u < kGkR; ++u) {
                    const double av = a_win[i + kGkR + u];
#pragma unroll
                    for (int r = 0; r < kGkR; ++r)
                        acc[c][r] = fma(av, u + r < kGkR ? w1[u + r] : w0[u + r - kGkR],
                                        acc[c][r]);
                }
            }
        }
    }
    double* out = part + ((int64_t)(g * kGkWaves + q) * max_lag) * 3;
#pragma unroll
    for (int r = 0; r < kGkR; ++r) {
        const int k = k0 + lb + r;
        if (k < max_lag) {
#pragma unroll
            for (int c = 0; c < 3; ++c) out[(int64_t)k * 3 + c] = acc[c][r];
        }
    }
}

// C(k) from the P = groups x waves partials, added in partial order: one
// thread per (lag, component), reading part with the same index stride.
__global__ void __launch_bounds__(kBlock)
k_gk_sum(const double* __restrict__ part, int P, int64_t S, int max_lag, double* __restrict__ hac)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;   // k * 3 + c
    const int64_t n = (int64_t)max_lag * 3;
    if (e >= n) return;
    double s = 0.0;
    for (int p = 0; p < P; ++p) s += part[(int64_t)p * n + e];
    hac[e] = s / (double)(S - e / 3);
}

// One block: the trapezoid running integral of C as a chunked scan (each
// thread a contiguous run of lags; the chunk totals are scanned in order by
// one thread).
__global__ void __launch_bounds__(kBlock)
k_gk_kappa(const double* __restrict__ hac, int max_lag, double scale, double* __restrict__ kappa)
{
    __shared__ double chunk_sum[kBlock][3];
    const int per = (max_lag + kBlock - 1) / kBlock;
    const int lo = threadIdx.x * per;
    const int hi = lo + per < max_lag ? lo + per : max_lag;
    double run[3] = {0.0, 0.0, 0.0};
    for (int k = lo > 0 ? lo : 1; k < hi; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            run[c] += 0.5 * (hac[(int64_t)(k - 1) * 3 + c] + hac[(int64_t)k * 3 + c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) chunk_sum[threadIdx.x][c] = run[c];
    __syncthreads();
    if (threadIdx.x == 0) {
        double off[3] = {0.0, 0.0, 0.0};
        for (int t = 0; t < kBlock; ++t)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double v = chunk_sum[t][c];
                chunk_sum[t][c] = off[c];
                off[c] += v;
            }
    }
    __syncthreads();
    double acc[3] = {chunk_sum[threadIdx.x][0], chunk_sum[threadIdx.x][1],
                     chunk_sum[threadIdx.x][2]};
    for (int k = lo; k < hi; ++k) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (k > 0) acc[c] += 0.5 * (hac[(int64_t)(k - 1) * 3 + c] + hac[(int64_t)k * 3 + c]);
            kappa[(int64_t)k * 3 + c] = scale * acc[c];
        }
    }
}

int gk_groups(int64_t S)
{
    const int64_t tiles = (S + kGkOrigins - 1) / kGkOrigins;
    return (int)(tiles < 64 ? tiles : 64);
}

size_t gk_scratch_bytes(int64_t S, int max_lag)
{
    return sizeof(double) * (3 * (size_t)S + (size_t)gk_groups(S) * kGkWaves * max_lag * 3);
}

hipError_t launch_green_kubo(const double* thermo, int64_t S, int every, int max_lag,
                             double scale, double* scratch, double* hac, double* kappa,
                             hipStream_t s)
{
    if (!thermo || !scratch || !hac || S < 1 || every < 1 || max_lag < 1 || max_lag > S)
        return hipErrorInvalidValue;
    double* jc = scratch;
    double* part = scratch + 3 * S;
    const int G = gk_groups(S);
    k_gk_compact<<<(int)((S + kBlock - 1) / kBlock), kBlock, 0, s>>>(thermo, S, every, jc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 grid(G, (max_lag + kGkLags - 1) / kGkLags);
    k_gk_corr<<<grid, kBlock, 0, s>>>(jc, S, max_lag, part);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)max_lag * 3;
    k_gk_sum<<<(int)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(part, G * kGkWaves, S, max_lag,
                                                               hac);
    e = hipGetLastError();
    if (e != hipSuccess || !kappa) return e;
    k_gk_kappa<<<1, kBlock, 0, s>>>(hac, max_lag, scale, kappa);
    return hipGetLastError();
}

}  // namespace mbmd
