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
// The correlation is a lag x origin product: a block owns 64 consecutive
// lags and walks a strided set of 1024-origin tiles, staging the two sample
// windows it needs (J(t) and J(t + k0 ..)) in LDS, zero-padded past the end
// so no product needs a bounds test.  Each lag's sum is split over a fixed
// number of origin groups and over the four waves of the block in a fixed
// pattern, and the finishing pass adds the group partials in group order:
// the result is the same bits on every run, without atomics.
#include "mbmd_internal.h"

namespace mbmd {

constexpr int kGkLags = 64;          // lags per block (one per lane of a wave)
constexpr int kGkOrigins = 1024;     // origins per staged tile
constexpr int kGkWaves = kBlock / 64;

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

__global__ void __launch_bounds__(kBlock)
k_gk_corr(const double* __restrict__ jc, int64_t S, int max_lag, double* __restrict__ part)
{
    __shared__ double a_win[3][kGkOrigins];
    __shared__ double b_win[3][kGkOrigins + kGkLags];
    __shared__ double red[kGkWaves][kGkLags][3];
    const int g = blockIdx.x, G = gridDim.x;
    const int k0 = blockIdx.y * kGkLags;
    const int l = threadIdx.x & 63, q = threadIdx.x >> 6;
    double acc[3] = {0.0, 0.0, 0.0};
    // origins t with t + k0 < S can pair with a lag of this block
    const int64_t tend = S - k0;
    for (int64_t t0 = (int64_t)g * kGkOrigins; t0 < tend; t0 += (int64_t)G * kGkOrigins) {
        __syncthreads();   // the previous tile is consumed
        for (int x = threadIdx.x; x < kGkOrigins + kGkLags; x += kBlock) {
            const int64_t tb = t0 + k0 + x;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (x < kGkOrigins) {
                    const int64_t ta = t0 + x;
                    a_win[c][x] = ta < S ? jc[c * S + ta] : 0.0;
                }
                b_win[c][x] = tb < S ? jc[c * S + tb] : 0.0;
            }
        }
        __syncthreads();
        // lag k0 + l, origins t0 + i for i = q, q + 4, ...: J(t + k) sits at
        // b_win[i + l]; past the end of the series the window holds zeros
        for (int i = q; i < kGkOrigins; i += kGkWaves) {
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[c] = fma(a_win[c][i], b_win[c][i + l], acc[c]);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) red[q][l][c] = acc[c];
    __syncthreads();
    if (threadIdx.x < kGkLags) {
        const int k = k0 + threadIdx.x;
        if (k < max_lag) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double s = red[0][threadIdx.x][c];
#pragma unroll
                for (int w = 1; w < kGkWaves; ++w) s += red[w][threadIdx.x][c];
                part[((int64_t)g * max_lag + k) * 3 + c] = s;
            }
        }
    }
}

// One block: C(k) from the group partials (in group order), then the
// trapezoid running integral as a chunked scan (each thread a contiguous
// run of lags; the chunk totals are scanned in order by one thread).
__global__ void __launch_bounds__(kBlock)
k_gk_finish(const double* __restrict__ part, int G, int64_t S, int max_lag, double scale,
            double* __restrict__ hac, double* __restrict__ kappa)
{
    __shared__ double chunk_sum[kBlock][3];
    const int per = (max_lag + kBlock - 1) / kBlock;
    const int lo = threadIdx.x * per;
    const int hi = lo + per < max_lag ? lo + per : max_lag;
    for (int k = lo; k < hi; ++k) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int g = 0; g < G; ++g) s += part[((int64_t)g * max_lag + k) * 3 + c];
            hac[(int64_t)k * 3 + c] = s / (double)(S - k);
        }
    }
    __syncthreads();
    if (!kappa) return;
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
    return sizeof(double) * (3 * (size_t)S + (size_t)gk_groups(S) * max_lag * 3);
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
    k_gk_finish<<<1, kBlock, 0, s>>>(part, G, S, max_lag, scale, hac, kappa);
    return hipGetLastError();
}

}  // namespace mbmd
