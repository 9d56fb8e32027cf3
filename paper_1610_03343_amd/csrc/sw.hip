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
    int ip, iq;   // p and q as small non-negative integers, or -1
};

inline int small_int_exponent(double e)
{
    return (e >= 0.0 && e <= 16.0 && e == (double)(int)e) ? (int)e : -1;
}

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
    k.ip = small_int_exponent(p.p);
    k.iq = small_int_exponent(p.q);
    return k;
}

__device__ __forceinline__ double s_exp(double x) { return fast_exp(x); }
__device__ __forceinline__ float s_exp(float x) { return expf(x); }
__device__ __forceinline__ double s_pow(double x, double y) { return pow(x, y); }
__device__ __forceinline__ float s_pow(float x, float y) { return powf(x, y); }

// x^e for the exponents p and q: repeated multiplication when e is a small
// non-negative integer (p = 4, q = 0 in the 1985 set), pow otherwise.
template <class T>
__device__ __forceinline__ T sw_power(T x, T e, int ie)
{
    if (ie < 0) return s_pow(x, e);
    T r = T(1);
    for (int k = 0; k < ie; ++k) r *= x;
    return r;
}

// Per-bond quantities at length r: E = exp(gamma sigma / (r - a sigma)),
// qg = -d ln E / dr = gamma sigma / (r - a sigma)^2, the two-body term phi2(r)
// and its derivative.  The bond is inside the cutoff by the FP64 test on r^2;
// r formed in the working precision can still round to a sigma or above, where
// every term and derivative takes its limit 0 (the exponent would overflow).
template <class T>
__device__ __forceinline__ void sw_bond(const SWK<T>& p, T r, T ir, T& E, T& qg, T& phi, T& dphi)
{
    if (!(r < p.asig)) {
        E = qg = phi = dphi = T(0);
        return;
    }
    const T idr = nr_rcp(r - p.asig);
    E = s_exp(p.gsig * idr);
    qg = p.gsig * idr * idr;
    const T sr = p.sigma * ir;
    const T srp = sw_power(sr, p.p, p.ip), srq = sw_power(sr, p.q, p.iq);
    const T e2 = s_exp(p.sigma * idr);
    const T poly = p.B * srp - srq;
    const T dpoly = (-p.p * p.B * srp + p.q * srq) * ir;
    phi = p.eps_A * poly * e2;
    dphi = p.eps_A * dpoly * e2 - phi * p.sigma * idr * idr;
}

// Unit vector, length and inverse length of bond d (r^2 > 0).
template <class T>
__device__ __forceinline__ void sw_geometry(const Disp& d, T& ux, T& uy, T& uz, T& r, T& ir)
{
    const T dx = (T)d.x, dy = (T)d.y, dz = (T)d.z;
    const T r2 = dx * dx + dy * dy + dz * dz;
    ir = nr_rsqrt(r2);
    r = r2 * ir;
    ux = dx * ir;
    uy = dy * ir;
    uz = dz * ir;
}

// Threads per block of the one-thread-per-atom overflow pass: its bond
// table (seven values and the list slot per bond, up to 64 bonds) lives in
// LDS, one column per thread, rather than in scratch memory (a launch with
// scratch took ~4.5 us longer on an empty list).
constexpr int kSWOvfThreads = 16;

// Site energy and partials of atom i, one thread, any number of in-cutoff
// bonds; tab and slot are the block's LDS bond table, col this thread's
// column.
template <class T>
__device__ __forceinline__ void sw_site(const SWK<T>& p, int64_t i, int64_t cap, const double4& xi,
                                        unsigned long long msk, int cnt,
                                        const int* __restrict__ nl,
                                        const double4* __restrict__ xw, const Box& box,
                                        double* __restrict__ U, T* __restrict__ dpart,
                                        T (*tab)[kMaxSlots][kSWOvfThreads],
                                        int (*slot)[kSWOvfThreads], int col)
{
    // bond c's unit vector, length, E_c, qg_c and phi2'(r_c)
    auto ux = [&](int c) -> T& { return tab[0][c][col]; };
    auto uy = [&](int c) -> T& { return tab[1][c][col]; };
    auto uz = [&](int c) -> T& { return tab[2][c][col]; };
    auto rr = [&](int c) -> T& { return tab[3][c][col]; };
    auto ex = [&](int c) -> T& { return tab[4][c][col]; };
    auto qg = [&](int c) -> T& { return tab[5][c][col]; };
    auto dph = [&](int c) -> T& { return tab[6][c][col]; };
    unsigned long long rem = msk;
    double u_i = 0.0;
    for (int c = 0; c < cnt; ++c) {
        const int m = __builtin_ctzll(rem);
        slot[c][col] = m;
        rem &= rem - 1;
        const int j = nl[(int64_t)m * cap + i];
        T x, y, z, r, ir, e, g, phi, d;
        sw_geometry(cut_disp(xi, xw[j], box), x, y, z, r, ir);
        sw_bond(p, r, ir, e, g, phi, d);
        ux(c) = x;
        uy(c) = y;
        uz(c) = z;
        rr(c) = r;
        ex(c) = e;
        qg(c) = g;
        dph(c) = d;
        u_i += 0.5 * (double)phi;
    }
    // three-body energy over unordered pairs (vertex i)
    for (int c = 0; c < cnt; ++c) {
        for (int e = c + 1; e < cnt; ++e) {
            const T cs = ux(c) * ux(e) + uy(c) * uy(e) + uz(c) * uz(e);
            const T ang = cs + T(1) / T(3);
            u_i += (double)(p.eps_lam * ex(c) * ex(e) * ang * ang);
        }
    }
    U[i] = u_i;
    for (int c = 0; c < cnt; ++c) {
        const T uxc = ux(c), uyc = uy(c), uzc = uz(c), exc = ex(c), qgc = qg(c);
        const T ir = nr_rcp(rr(c));
        T dx = T(0.5) * dph(c) * uxc, dy = T(0.5) * dph(c) * uyc, dz = T(0.5) * dph(c) * uzc;
        for (int e = 0; e < cnt; ++e) {
            if (e != c) {
                const T uxe = ux(e), uye = uy(e), uze = uz(e);
                const T cs = uxc * uxe + uyc * uye + uzc * uze;
                const T ang = cs + T(1) / T(3);
                const T ee = p.eps_lam * exc * ex(e);
                const T radial = -ee * ang * ang * qgc;
                const T angular = T(2) * ee * ang * ir;
                dx += radial * uxc + angular * (uxe - cs * uxc);
                dy += radial * uyc + angular * (uye - cs * uyc);
                dz += radial * uzc + angular * (uze - cs * uzc);
            }
        }
        T* o = dpart + ((int64_t)slot[c][col] * cap + i) * 3;
        o[0] = dx;
        o[1] = dy;
        o[2] = dz;
    }
}

// Quad site pass: four lanes per atom, lane q owning bonds q, q + 4 and
// q + 8 (the layout of the Tersoff quad pass with one more slot: SW crystals
// near room temperature have 4 to 11 bonds inside the cutoff).  Each lane forms its bonds' E_c, qg_c
// and two-body terms, then, over the partner bonds e fetched from the other
// lanes, half of h_ce for U_i (each unordered pair is met from both ends)
// and the three-body part of dU_i/dr_c.  Atoms with more than kQuadBonds
// in-cutoff bonds go to the overflow list.
template <class T, int SLOTS>
__global__ void __launch_bounds__(kBlock)
k_sw_site_quad(SWK<T> p, double rc2, Segs S, int M, int64_t cap,
               const double4* __restrict__ xw, const int* __restrict__ nn,
               const int* __restrict__ nl, unsigned long long* __restrict__ mask,
               double* __restrict__ U, T* __restrict__ dpart, int* __restrict__ ovf_count,
               int* __restrict__ ovf_list)
{
    const int q = threadIdx.x & (kQuad - 1);
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int sid = seg_of_block(S, lb, true);
    const Seg& g = S.seg[sid];
    const int phase = S.phase_in[sid];
    const Box box = g.box;
    const int local = (lb - g.blk_quad) * kQuadAtoms + (threadIdx.x >> 2);
    const int64_t i = g.atom_off + local;
    const bool valid = local < g.n;
    const double4 xi = valid ? xw[i] : make_double4(0.0, 0.0, 0.0, 0.0);
    const int nnb = valid ? min(nn[i], M) : 0;
    // a finished segment (kept for retrieval) is left as it is; the test
    // follows the first loads (in bounds for it too) to share their wait
    if (phase > g.nsteps) return;
    Disp d_first;
    const unsigned long long msk = quad_cutoff_mask<true>(xi, i, cap, nnb, q, nl, xw, box, rc2, d_first);
    const int cnt = __popcll(msk);
    const bool ovf = cnt > kQuad * SLOTS;
    if (valid && q == 0) {
        mask[i] = msk;
        if (ovf) ovf_list[atomicAdd(ovf_count, 1)] = (int)i;
    }
    const int kc = (valid && !ovf) ? cnt : 0;   // bonds handled by this quad

    T ux[SLOTS], uy[SLOTS], uz[SLOTS], ir[SLOTS], ex[SLOTS],
        qg[SLOTS], gx[SLOTS], gy[SLOTS], gz[SLOTS];
    int slot[SLOTS];
    double u_i = 0.0;
    // bond slots any atom of the wave needs (wave-uniform): slots past it
    // are empty in every lane and not issued
    const int tmax = wave_partner_slots<SLOTS>(kc);
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int c = q + kQuad * s;
        ux[s] = uy[s] = uz[s] = ex[s] = qg[s] = gx[s] = gy[s] = gz[s] = T(0);
        ir[s] = T(1);
        slot[s] = 0;
        if (s < tmax && c < kc) {
            const int m = nth_set_bit(msk, c);
            slot[s] = m;
            T r, phi, dphi;
            const Disp d = (s == 0 && m == q) ? d_first : cut_disp(xi, xw[nl[(int64_t)m * cap + i]], box);
            sw_geometry(d, ux[s], uy[s], uz[s], r, ir[s]);
            sw_bond(p, r, ir[s], ex[s], qg[s], phi, dphi);
            u_i += 0.5 * (double)phi;
            gx[s] = T(0.5) * dphi * ux[s];
            gy[s] = T(0.5) * dphi * uy[s];
            gz[s] = T(0.5) * dphi * uz[s];
        }
    }
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) {
        if (t >= tmax) break;   // wave-uniform
#pragma unroll
        for (int k = 0; k < kQuad; ++k) {
            const T fx = k ? quad_xor(ux[t], k) : ux[t];
            const T fy = k ? quad_xor(uy[t], k) : uy[t];
            const T fz = k ? quad_xor(uz[t], k) : uz[t];
            const T fe = k ? quad_xor(ex[t], k) : ex[t];
            const int e = (q ^ k) + kQuad * t;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                if (s >= tmax) break;   // wave-uniform: own slots past it are empty
                const int c = q + kQuad * s;
                if (c < kc && e < kc && e != c) {
                    const T cs = ux[s] * fx + uy[s] * fy + uz[s] * fz;
                    const T ang = cs + T(1) / T(3);
                    const T ee = p.eps_lam * ex[s] * fe;
                    const T h = ee * ang * ang;
                    u_i += 0.5 * (double)h;
                    const T radial = -h * qg[s];
                    const T angular = T(2) * ee * ang * ir[s];
                    gx[s] += radial * ux[s] + angular * (fx - cs * ux[s]);
                    gy[s] += radial * uy[s] + angular * (fy - cs * uy[s]);
                    gz[s] += radial * uz[s] + angular * (fz - cs * uz[s]);
                }
            }
        }
    }
    u_i = quad_sum(u_i);
    if (q == 0 && valid && !ovf) U[i] = u_i;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int c = q + kQuad * s;
        if (c < kc) {
            T* o = dpart + ((int64_t)slot[s] * cap + i) * 3;
            o[0] = gx[s];
            o[1] = gy[s];
            o[2] = gz[s];
        }
    }
}

template <class T>
__global__ void __launch_bounds__(kSWOvfThreads)
k_sw_partials_ovf(SWK<T> p, Segs S, int64_t cap, const double4* __restrict__ xw,
                  const int* __restrict__ nl, const unsigned long long* __restrict__ mask,
                  double* __restrict__ U, T* __restrict__ dpart,
                  const int* __restrict__ ovf_count, const int* __restrict__ ovf_list)
{
    __shared__ T tab[7][kMaxSlots][kSWOvfThreads];
    __shared__ int slot[kMaxSlots][kSWOvfThreads];
    const int total = *ovf_count;
    for (int k = blockIdx.x * kSWOvfThreads + threadIdx.x; k < total;
         k += gridDim.x * kSWOvfThreads) {
        const int64_t i = ovf_list[k];
        const double4 xi = xw[i];
        const unsigned long long msk = mask[i];
        sw_site<T>(p, i, cap, xi, msk, __popcll(msk), nl, xw, S.seg[seg_of_atom(S, i)].box, U,
                   dpart, tab, slot, threadIdx.x);
    }
}

constexpr int kSWOvfGrid = 256;

template <class T>
hipError_t launch_sw_partials(const Buffers& b, const Segs& S, int cur, const SWParams& p,
                              bool overflow_pass, int max_nn, hipStream_t s)
{
    if (S.nblk_quad <= 0) return hipSuccess;
    if (!segs_ready(S, b)) return hipErrorInvalidValue;
    const SWK<T> k = sw_constants<T>(p);
    const double rc = p.a * p.sigma;
    T* dp = static_cast<T*>(b.dpart);
    if (!overflow_pass) {
        k_sw_site_quad<T, kSWSlots><<<S.nblk_quad, kBlock, 0, s>>>(k, rc * rc, S, b.M, b.cap, b.xw[cur],
                                                         b.nn, b.nl, b.mask, b.U, dp,
                                                         b.ovf_count, b.ovf_list);
        return hipGetLastError();
    }
    if (b.M > kQuad * kSWSlots && max_nn > kQuad * kSWSlots)
        k_sw_partials_ovf<T><<<kSWOvfGrid, kSWOvfThreads, 0, s>>>(
            k, S, b.cap, b.xw[cur], b.nl, b.mask, b.U, dp, b.ovf_count, b.ovf_list);
    return hipGetLastError();
}

template hipError_t launch_sw_partials<double>(const Buffers&, const Segs&, int, const SWParams&,
                                               bool, int, hipStream_t);
template hipError_t launch_sw_partials<float>(const Buffers&, const Segs&, int, const SWParams&,
                                              bool, int, hipStream_t);

}  // namespace mbmd
