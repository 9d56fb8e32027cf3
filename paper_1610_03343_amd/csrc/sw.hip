// Stillinger-Weber site-local pass: per-atom energy and partials.
//
// The paper evaluates SW with the same per-atom forms (Section 2.4) in a
// single kernel; it prints no SW formula.  The 1985 form is used, with the
// site energy of atom i taken as half of each two-body term plus every
// three-body term whose vertex is i:
//   U_i = 1/2 sum_c phi2(r_c) + sum_{c<e} h_ce,
//   phi2(r) = eps A (B (sigma/r)^p - (sigma/r)^q) exp(sigma / (r - a sigma)),
//   h_ce = eps lambda E_c E_e (cos_ce + 1/3)^2,  E_c = exp(gamma sigma / (r_c - a sigma)).
// The partials follow as
//   dU_i/dr_c = 1/2 phi2'(r_c) u_c
//             + sum_{e != c} [ -h_ce gamma sigma / (r_c - a sigma)^2 u_c
//                              + 2 eps lambda E_c E_e (cos_ce + 1/3) (u_e - cos_ce u_c) / r_c ].
#include "partials_common.h"

namespace mbmd {

template <class T>
struct SWK {
    T eps_A, B, p, q, sigma, asig, eps_lam, gsig;
};

template <class T>
SWK<T> sw_constants(const SWParams& p)
{
    SWK<T> k;
    k.eps_A = (T)(p.epsilon * p.A);
    k.B = (T)p.B;
    k.p = (T)p.p;
    k.q = (T)p.q;
    k.sigma = (T)p.sigma;
    k.asig = (T)(p.a * p.sigma);
    k.eps_lam = (T)(p.epsilon * p.lam);
    k.gsig = (T)(p.gamma * p.sigma);
    return k;
}

__device__ __forceinline__ double s_exp(double x) { return exp(x); }
__device__ __forceinline__ float s_exp(float x) { return expf(x); }
__device__ __forceinline__ double s_pow(double x, double y) { return pow(x, y); }
__device__ __forceinline__ float s_pow(float x, float y) { return powf(x, y); }
__device__ __forceinline__ double s_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float s_sqrt(float x) { return sqrtf(x); }

template <class T, int MAXC, bool FIXED>
__device__ __forceinline__ void sw_site(const SWK<T>& p, int64_t i, int64_t cap, const double4& xi,
                                        unsigned long long msk, int cnt,
                                        const int* __restrict__ nl,
                                        const double4* __restrict__ xw, const Box& box,
                                        double* __restrict__ U, T* __restrict__ dpart)
{
    T ux[MAXC], uy[MAXC], uz[MAXC], rr[MAXC], ex[MAXC], qg[MAXC], dph[MAXC];
    int slot[MAXC];
    unsigned long long rem = msk;
    double u_i = 0.0;
#pragma unroll
    for (int c = 0; c < (FIXED ? MAXC : cnt); ++c) {
        ux[c] = uy[c] = uz[c] = rr[c] = ex[c] = qg[c] = dph[c] = T(0);
        slot[c] = 0;
        if (c < cnt) {
            const int m = __builtin_ctzll(rem);
            slot[c] = m;
            rem &= rem - 1;
            const int j = nl[(int64_t)m * cap + i];
            const Disp d = cut_disp(xi, xw[j], box);
            const T dx = (T)d.x, dy = (T)d.y, dz = (T)d.z;
            const T r = s_sqrt(dx * dx + dy * dy + dz * dz);
            const T ir = T(1) / r;
            ux[c] = dx * ir;
            uy[c] = dy * ir;
            uz[c] = dz * ir;
            rr[c] = r;
            const T idr = T(1) / (r - p.asig);
            ex[c] = s_exp(p.gsig * idr);
            qg[c] = p.gsig * idr * idr;
            // two-body term and its radial derivative
            const T sr = p.sigma * ir;
            const T srp = s_pow(sr, p.p), srq = s_pow(sr, p.q);
            const T e2 = s_exp(p.sigma * idr);
            const T poly = p.B * srp - srq;
            const T dpoly = (-p.p * p.B * srp + p.q * srq) * ir;
            const T phi = p.eps_A * poly * e2;
            dph[c] = p.eps_A * dpoly * e2 - phi * p.sigma * idr * idr;
            u_i += 0.5 * (double)phi;
        }
    }
    // three-body energy over unordered pairs (vertex i)
#pragma unroll
    for (int c = 0; c < (FIXED ? MAXC : cnt); ++c) {
#pragma unroll
        for (int e = c + 1; e < (FIXED ? MAXC : cnt); ++e) {
            if (e < cnt) {
                const T cs = ux[c] * ux[e] + uy[c] * uy[e] + uz[c] * uz[e];
                const T ang = cs + T(1) / T(3);
                u_i += (double)(p.eps_lam * ex[c] * ex[e] * ang * ang);
            }
        }
    }
    U[i] = u_i;
#pragma unroll
    for (int c = 0; c < (FIXED ? MAXC : cnt); ++c) {
        if (c < cnt) {
            const T ir = T(1) / rr[c];
            T dx = T(0.5) * dph[c] * ux[c], dy = T(0.5) * dph[c] * uy[c], dz = T(0.5) * dph[c] * uz[c];
#pragma unroll
            for (int e = 0; e < (FIXED ? MAXC : cnt); ++e) {
                if (e != c && e < cnt) {
                    const T cs = ux[c] * ux[e] + uy[c] * uy[e] + uz[c] * uz[e];
                    const T ang = cs + T(1) / T(3);
                    const T ee = p.eps_lam * ex[c] * ex[e];
                    const T radial = -ee * ang * ang * qg[c];
                    const T angular = T(2) * ee * ang * ir;
                    dx += radial * ux[c] + angular * (ux[e] - cs * ux[c]);
                    dy += radial * uy[c] + angular * (uy[e] - cs * uy[c]);
                    dz += radial * uz[c] + angular * (uz[e] - cs * uz[c]);
                }
            }
            T* o = dpart + ((int64_t)slot[c] * cap + i) * 3;
            o[0] = dx;
            o[1] = dy;
            o[2] = dz;
        }
    }
}

template <class T, int MAXC>
__global__ void __launch_bounds__(kBlock)
k_sw_partials(SWK<T> p, double rc2, Segs S, int M, int64_t cap, const double4* __restrict__ xw,
              const int* __restrict__ nn, const int* __restrict__ nl,
              unsigned long long* __restrict__ mask, double* __restrict__ U,
              T* __restrict__ dpart, int* __restrict__ ovf_count, int* __restrict__ ovf_list)
{
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int sid = seg_of_block(S, lb, false);
    const Seg& g = S.seg[sid];
    if (S.phase_in[sid] > g.nsteps) return;   // finished segment, kept for retrieval
    const int local = (lb - g.blk) * kBlock + threadIdx.x;
    if (local >= g.n) return;
    const int64_t i = g.atom_off + local;
    const double4 xi = xw[i];
    const int nnb = min(nn[i], M);
    const unsigned long long msk = cutoff_mask(xi, i, cap, nnb, nl, xw, g.box, rc2);
    mask[i] = msk;
    const int cnt = __popcll(msk);
    if (cnt > MAXC) {
        ovf_list[atomicAdd(ovf_count, 1)] = (int)i;
        return;
    }
    sw_site<T, MAXC, true>(p, i, cap, xi, msk, cnt, nl, xw, g.box, U, dpart);
}

template <class T>
__global__ void __launch_bounds__(kBlock)
k_sw_partials_ovf(SWK<T> p, Segs S, int64_t cap, const double4* __restrict__ xw,
                  const int* __restrict__ nl, const unsigned long long* __restrict__ mask,
                  double* __restrict__ U, T* __restrict__ dpart,
                  const int* __restrict__ ovf_count, const int* __restrict__ ovf_list)
{
    const int total = *ovf_count;
    for (int k = blockIdx.x * kBlock + threadIdx.x; k < total; k += gridDim.x * kBlock) {
        const int64_t i = ovf_list[k];
        const double4 xi = xw[i];
        const unsigned long long msk = mask[i];
        sw_site<T, kMaxSlots, false>(p, i, cap, xi, msk, __popcll(msk), nl, xw,
                                     S.seg[seg_of_atom(S, i)].box, U, dpart);
    }
}

constexpr int kSWTile = kSiteFastBonds;
constexpr int kSWOvfGrid = 64;

template <class T>
hipError_t launch_sw_partials(const Buffers& b, const Segs& S, int cur, const SWParams& p,
                              bool overflow_pass, int max_nn, hipStream_t s)
{
    if (S.nblk <= 0) return hipSuccess;
    if (!segs_ready(S, b)) return hipErrorInvalidValue;
    const SWK<T> k = sw_constants<T>(p);
    const double rc = p.a * p.sigma;
    T* dp = static_cast<T*>(b.dpart);
    if (!overflow_pass) {
        k_sw_partials<T, kSWTile><<<S.nblk, kBlock, 0, s>>>(k, rc * rc, S, b.M, b.cap, b.xw[cur],
                                                            b.nn, b.nl, b.mask, b.U, dp,
                                                            b.ovf_count, b.ovf_list);
        return hipGetLastError();
    }
    if (b.M > kSiteFastBonds && max_nn > kSiteFastBonds)
        k_sw_partials_ovf<T><<<kSWOvfGrid, kBlock, 0, s>>>(k, S, b.cap, b.xw[cur], b.nl, b.mask,
                                                           b.U, dp, b.ovf_count, b.ovf_list);
    return hipGetLastError();
}

template hipError_t launch_sw_partials<double>(const Buffers&, const Segs&, int, const SWParams&,
                                               bool, int, hipStream_t);
template hipError_t launch_sw_partials<float>(const Buffers&, const Segs&, int, const SWParams&,
                                              bool, int, hipStream_t);

}  // namespace mbmd
