// Tersoff site-local pass: bond order and per-atom partials.
//
// For atom i with in-cutoff neighbours c = 0..K-1 (unit vectors u_c, lengths
// r_c), the Tersoff site energy (Section 2.1) is
//   U_i = 1/2 sum_c f_C(r_c) [f_R(r_c) - b_c f_A(r_c)],
//   b_c = (1 + (beta zeta_c)^n)^(-1/(2n)),  zeta_c = sum_{e != c} f_C(r_e) g(cos_ce),
// with f_R = A exp(-lambda r), f_A = B exp(-mu r) and the 1989 cutoff f_C.
// Every term depends on atom i's neighbours only, so one thread computes
// all zeta_c and b_c (the bond-order pass of the paper's Section 2.3 two-kernel
// approach) and, in the same registers, the partials
//   dU_i/dr_c = 1/2 [f_C'(f_R - b f_A) + f_C (f_R' - b f_A')] u_c
//             - 1/2 sum_{e != c} (P_c f_C(r_e) + P_e f_C(r_c)) g'(cos_ce) (u_e - cos_ce u_c) / r_c
//             - 1/2 sum_{e != c} P_e f_C'(r_c) g(cos_ce) u_c,
//   P_c = f_C(r_c) f_A(r_c) db_c/dzeta_c,
// i.e. the derivative of U_i through r_c's own bond and through the bond
// orders of all other bonds of atom i.  The partials are stored at the list
// slot of the neighbour for the pairwise-force pass.
//
// g is evaluated as 1 + c^2 t^2 / (d^2 (d^2 + t^2)), t = h - cos (identical to
// the printed 1 + c^2/d^2 - c^2/(d^2 + t^2) without its large cancellation);
// db/dzeta is 0 at zeta = 0, where it multiplies an empty sum.
//
// Several atom types (the generality the paper claims for its method in
// Section 2.1, with Tersoff's 1989 multicomponent form): the bond terms of
// bond c use the parameters of the type pair (i, c) (A, B, lambda, mu, R, S
// mixed from the two elements), g, beta and n those of atom i, and b_c is
// multiplied by chi of the pair.  The formulas above hold unchanged with
// f_R, f_A, f_C and their derivatives per bond.  The single-type kernels
// read every constant from the kernel arguments (uniform registers); the
// multi-type ones copy the table to LDS and index it by type.
#include <cmath>

#include "partials_common.h"

namespace mbmd {

// Constants of a centre atom's element: the angular term and the bond order.
template <class T>
struct TCenter {
    T beta, n, inv2n, c2, c2_d2, d2, h;
    // b = (1 + u)^a, a = -1/(2n): binomial series coefficients a_k = C(a, k),
    // used below u_series = 2^-9 where the first omitted term, |a_6| u^6, is
    // below 2e-17 relative
    T u_series, a1, a2, a3, a4, a5;
};
// Constants of a bond's type pair: f_R, f_A, f_C and the bond-order factor.
template <class T>
struct TPair {
    T A, B, lam, mu, R, S, pi_sr, chi;
};
// Kernel arguments: one element (MULTI = false), or the table indexed
// [ti] and [ti * kMaxTypes + tj].  S2 is the FP64 cutoff squared of a pair
// (the in-cutoff test on r^2, the same for (i, j) and (j, i)).  The
// single-type argument stays small: the table would be fetched with every
// launch.
template <class T, bool MULTI>
struct TersoffArg;
// b = (1 + u)^a, a = -1/(2n), as a polynomial in w = u - u0 on
// [kBPolyLo, kBPolyHi] (the range of u in a silicon crystal near room
// temperature, u ~ 0.07): its Taylor series about u0 = 7/64, the coefficients
// d_k = C(a, k) (1 + u0)^(a - k) formed on the host in extended precision.
// With |w| <= 5/64 the first omitted term is ~2e-17 of b.  FP64
// single-element kernels only (the one-thread overflow routine, the mixed
// and the multi-element kernels keep the logarithm and exponential).
constexpr int kBPolyTerms = 14;
constexpr double kBPolyLo = 0x1p-5, kBPolyHi = 0x3p-4, kBPolyU0 = 0x7p-6;

template <class T>
struct TersoffArg<T, false> {   // the centre and pair constants of one element, flat
    T A, B, lam, mu, beta, n, inv2n, c2, c2_d2, d2, h, R, pi_sr;
    T u_series, a1, a2, a3, a4, a5;
    T S;
    double bpoly[kBPolyTerms];   // d_0 .. d_13 (used when T is double)
};
template <class T>
struct TersoffArg<T, true> {
    TCenter<T> c[kMaxTypes];
    TPair<T> p[kMaxTypes * kMaxTypes];
    double S2[kMaxTypes * kMaxTypes];
};

template <class T>
TCenter<T> center_constants(const TersoffParams& e)
{
    TCenter<T> k;
    k.beta = (T)e.beta;
    k.n = (T)e.n;
    k.inv2n = (T)(1.0 / (2.0 * e.n));
    k.c2 = (T)(e.c * e.c);
    k.c2_d2 = (T)(e.c * e.c / (e.d * e.d));
    k.d2 = (T)(e.d * e.d);
    k.h = (T)e.h;
    const double a = -1.0 / (2.0 * e.n);
    double ak[6] = {1.0, 0, 0, 0, 0, 0};
    for (int j = 1; j < 6; ++j) ak[j] = ak[j - 1] * (a - (j - 1)) / j;
    k.a1 = (T)ak[1];
    k.a2 = (T)ak[2];
    k.a3 = (T)ak[3];
    k.a4 = (T)ak[4];
    k.a5 = (T)ak[5];
    k.u_series = (T)0x1p-9;
    return k;
}

// The constants of type pair (a, b): Tersoff's 1989 mixing rules (geometric
// means for A, B, R, S; arithmetic means for lambda, mu), which give the
// element's own values, exactly, for a == b (sqrt(x * x) = |x| in IEEE
// arithmetic).
template <class T>
TPair<T> pair_constants(const TersoffTable& tab, int a, int b, double* S_out)
{
    const TersoffParams& x = tab.elem[a];
    const TersoffParams& y = tab.elem[b];
    const double R = std::sqrt(x.R * y.R);
    const double S = std::sqrt(x.S * y.S);
    TPair<T> k;
    k.A = (T)std::sqrt(x.A * y.A);
    k.B = (T)std::sqrt(x.B * y.B);
    k.lam = (T)(0.5 * (x.lam + y.lam));
    k.mu = (T)(0.5 * (x.mu + y.mu));
    k.R = (T)R;
    k.S = (T)S;
    k.pi_sr = (T)(3.14159265358979323846 / (S - R));
    k.chi = (T)tab.chi[a * kMaxTypes + b];
    *S_out = S;
    return k;
}

template <class T>
TersoffArg<T, true> tersoff_table(const TersoffTable& tab)
{
    TersoffArg<T, true> k{};
    for (int a = 0; a < tab.nt; ++a) {
        k.c[a] = center_constants<T>(tab.elem[a]);
        for (int b = 0; b < tab.nt; ++b) {
            double S;
            k.p[a * kMaxTypes + b] = pair_constants<T>(tab, a, b, &S);
            k.S2[a * kMaxTypes + b] = S * S;
        }
    }
    return k;
}

template <class T>
TersoffArg<T, false> tersoff_single(const TersoffTable& tab, double* S2)
{
    double S;
    const TCenter<T> c = center_constants<T>(tab.elem[0]);
    const TPair<T> p = pair_constants<T>(tab, 0, 0, &S);
    TersoffArg<T, false> k;
    k.A = p.A;
    k.B = p.B;
    k.lam = p.lam;
    k.mu = p.mu;
    k.beta = c.beta;
    k.n = c.n;
    k.inv2n = c.inv2n;
    k.c2 = c.c2;
    k.c2_d2 = c.c2_d2;
    k.d2 = c.d2;
    k.h = c.h;
    k.R = p.R;
    k.pi_sr = p.pi_sr;
    k.u_series = c.u_series;
    k.a1 = c.a1;
    k.a2 = c.a2;
    k.a3 = c.a3;
    k.a4 = c.a4;
    k.a5 = c.a5;
    k.S = p.S;
    {
        const long double a = -1.0L / (2.0L * (long double)tab.elem[0].n);
        const long double v0 = 1.0L + (long double)kBPolyU0;
        long double binom = 1.0L;   // C(a, j)
        for (int j = 0; j < kBPolyTerms; ++j) {
            k.bpoly[j] = (double)(binom * powl(v0, a - (long double)j));
            binom *= (a - (long double)j) / (long double)(j + 1);
        }
    }
    *S2 = S * S;
    return k;
}

// Multi-type kernels: the table in LDS, filled by the whole block.
template <class T>
struct TersoffLds {
    TCenter<T> c[kMaxTypes];
    TPair<T> p[kMaxTypes * kMaxTypes];
    double S2[kMaxTypes * kMaxTypes];
};

template <class T>
__device__ __forceinline__ void fill_lds_table(const TersoffArg<T, true>& K, TersoffLds<T>& L)
{
    if (threadIdx.x < kMaxTypes) L.c[threadIdx.x] = K.c[threadIdx.x];
    if (threadIdx.x < kMaxTypes * kMaxTypes) {
        L.p[threadIdx.x] = K.p[threadIdx.x];
        L.S2[threadIdx.x] = K.S2[threadIdx.x];
    }
    __syncthreads();
}

__device__ __forceinline__ double t_exp(double x) { return fast_exp(x); }
__device__ __forceinline__ float t_exp(float x) { return expf(x); }
// Natural logarithm of a positive normal double for the bond order, from
// ln x = e ln 2 + ln m with x = m 2^e, m in [sqrt(1/2), sqrt(2)), and the
// series ln m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...), s = (m - 1)/(m + 1),
// |s| < 0.172, summed to s^21 (first omitted term below 1e-17 relative).
// A few ulp, against the correctly rounded library log at about half the
// arithmetic; (beta zeta)^n needs far less.  SCONST false writes the
// constants as literals: the bond order's second logarithm takes them so,
// since a second set held in scalar registers overflowed them.
template <bool SCONST = true>
__device__ __forceinline__ double t_log(double x)
{
    // (the constants go through scalar registers unless SCONST is false:
    // see sgpr_const)
    auto K = [](double c) { return SCONST ? sgpr_const(c) : c; };
    int e;
    double m = frexp(x, &e);               // x = m 2^e, m in [0.5, 1)
    if (m < K(0.70710678118654752440)) {
        m *= 2.0;
        e -= 1;
    }
    const double s = (m - 1.0) * nr_rcp(m + 1.0);
    const double s2 = s * s;
    double p = fma(K(1.0 / 21.0), s2, K(1.0 / 19.0));
    p = fma(p, s2, K(1.0 / 17.0));
    p = fma(p, s2, K(1.0 / 15.0));
    p = fma(p, s2, K(1.0 / 13.0));
    p = fma(p, s2, K(1.0 / 11.0));
    p = fma(p, s2, K(1.0 / 9.0));
    p = fma(p, s2, K(1.0 / 7.0));
    p = fma(p, s2, K(1.0 / 5.0));
    p = fma(p, s2, K(1.0 / 3.0));
    const double lnm = 2.0 * s + 2.0 * s * s2 * p;
    // ln 2 = ln2_hi + ln2_lo, ln2_hi with 32 significant bits (e * ln2_hi is
    // exact for |e| < 2^21), ln2_lo the rounded remainder
    const double ln2_hi = K(0x1.62e42fee00000p-1), ln2_lo = K(0x1.a39ef35793c76p-33);
    const double de = (double)e;
    return fma(de, ln2_hi, fma(de, ln2_lo, lnm));
}
template <bool SCONST = true>
__device__ __forceinline__ float t_log(float x) { return logf(x); }
__device__ __forceinline__ void t_sincos(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ void t_sincos(float x, float* s, float* c) { sincosf(x, s, c); }

// f_C and f_C' (the caller only passes bonds inside the cutoff by the FP64
// test on r^2; r formed in the working precision that rounds to S or above
// takes the limit 0).
template <class P, class T>
__device__ __forceinline__ void cutoff_fc(const P& p, T r, T& fc, T& dfc)
{
    if (r < p.R) {
        fc = T(1);
        dfc = T(0);
    } else if (!(r < p.S)) {
        fc = T(0);
        dfc = T(0);
    } else {
        T s, c;
        t_sincos(p.pi_sr * (r - p.R), &s, &c);
        fc = T(0.5) + T(0.5) * c;
        dfc = T(-0.5) * p.pi_sr * s;
    }
}

template <class P, class T>
__device__ __forceinline__ void angular_g(const P& p, T cs, T& g, T& dg)
{
    const T t = p.h - cs;
    const T iq = nr_rcp(p.d2 + t * t);
    g = T(1) + p.c2_d2 * t * t * iq;
    dg = T(-2) * p.c2 * t * iq * iq;
}

// b(zeta) and db/dzeta; b(0) = 1, db/dzeta(0) = 0.  With u = (beta zeta)^n,
// b = (1 + u)^(-1/(2n)) is summed as its binomial series when u < 2^-9 (few
// bonds or wide angles), else as exp(-ln(1 + u) / (2n)).  In the Si crystal
// u ~ 0.07 (each tetrahedral angle gives g ~ 1.0e4, c^2/d^2 being ~4e7), so
// the second form is the common one; ln(1 + u) is taken of the rounded sum,
// whose absolute error (half an ulp of 1 + u) becomes a relative error of
// about 1e-16 / (2n) in b for any u, so no log1p is needed.
// bp: the polynomial's coefficients (d_0 .. d_13, then u0, lo, hi) in LDS,
// or null: between lo and hi it replaces the logarithm and exponential.
template <class P, class T>
__device__ __forceinline__ void bond_order(const P& p, T zeta, T& b, T& db,
                                           const double* bp = nullptr)
{
    b = T(1);
    db = T(0);
    if (zeta > T(0)) {
        const T u = t_exp(p.n * t_log(p.beta * zeta));
        if (u < p.u_series) {
            b = T(1) + u * (p.a1 + u * (p.a2 + u * (p.a3 + u * (p.a4 + u * p.a5))));
        } else {
            bool done = false;
            if constexpr (sizeof(T) == 8) {
                if (bp && u >= bp[kBPolyTerms + 1] && u <= bp[kBPolyTerms + 2]) {
                    const double w = u - bp[kBPolyTerms];
                    double acc = bp[kBPolyTerms - 1];
#pragma unroll
                    for (int j = kBPolyTerms - 2; j >= 0; --j) acc = fma(acc, w, bp[j]);
                    b = acc;
                    done = true;
                }
            }
            if (!done) b = t_exp(-t_log<false>(T(1) + u) * p.inv2n);
        }
        db = -b * u * nr_rcp(T(2) * zeta * (T(1) + u));
    }
}

// Unit vector, length and inverse length of bond d (r^2 > 0).
template <class T>
__device__ __forceinline__ void bond_geometry(const Disp& d, T& ux, T& uy, T& uz, T& r, T& ir)
{
    const T dx = (T)d.x, dy = (T)d.y, dz = (T)d.z;
    const T r2 = dx * dx + dy * dy + dz * dz;
    ir = nr_rsqrt(r2);
    r = r2 * ir;
    ux = dx * ir;
    uy = dy * ir;
    uz = dz * ir;
}

// Per-bond and per-centre constants: the LDS table entries of type pair tp
// and of type ti, or the single element's flat argument (which carries both
// sets of fields).
template <class T, bool MULTI>
__device__ __forceinline__ const auto& pair_of(const TersoffArg<T, MULTI>& K,
                                               const TersoffLds<T>& L, int tp)
{
    if constexpr (MULTI) return L.p[tp];
    else return K;
}
template <class T, bool MULTI>
__device__ __forceinline__ const auto& center_of(const TersoffArg<T, MULTI>& K,
                                                 const TersoffLds<T>& L, int ti)
{
    if constexpr (MULTI) return L.c[ti];
    else return K;
}

// One thread, any number of bonds (the overflow pass).  tp of bond c is the
// table index ti * kMaxTypes + tj.
template <class T, int MAXC, bool MULTI>
__device__ __forceinline__ void tersoff_site(const TersoffArg<T, MULTI>& K, const TersoffLds<T>& L,
                                             int64_t i, int64_t cap, const double4& xi,
                                             unsigned long long msk, int cnt,
                                             const int* __restrict__ nl,
                                             const double4* __restrict__ xw, const Box& box,
                                             double* __restrict__ U, T* __restrict__ dpart)
{
    T ux[MAXC], uy[MAXC], uz[MAXC], rr[MAXC], fc[MAXC], dfc[MAXC], zp[MAXC], pd[MAXC];
    int slot[MAXC], tp[MAXC];
    const int ti = MULTI ? (int)xi.w : 0;
    const auto& pc = center_of<T, MULTI>(K, L, ti);
    unsigned long long rem = msk;
    for (int c = 0; c < cnt; ++c) {
        ux[c] = uy[c] = uz[c] = rr[c] = fc[c] = dfc[c] = zp[c] = pd[c] = T(0);
        slot[c] = 0;
        tp[c] = 0;
        if (c < cnt) {
            const int m = __builtin_ctzll(rem);
            slot[c] = m;
            rem &= rem - 1;
            const double4 xj = xw[nl[(int64_t)m * cap + i]];
            if (MULTI) tp[c] = ti * kMaxTypes + (int)xj.w;
            T ir;
            bond_geometry(cut_disp(xi, xj, box), ux[c], uy[c], uz[c], rr[c], ir);
            cutoff_fc(pair_of<T, MULTI>(K, L, tp[c]), rr[c], fc[c], dfc[c]);
        }
    }
    // zeta_c over unordered pairs: g(cos_ce) is shared by zeta_c and zeta_e.
    for (int c = 0; c < cnt; ++c) {
        for (int e = c + 1; e < cnt; ++e) {
            if (e < cnt) {
                const T cs = ux[c] * ux[e] + uy[c] * uy[e] + uz[c] * uz[e];
                T g, dg;
                angular_g(pc, cs, g, dg);
                zp[c] += fc[e] * g;
                zp[e] += fc[c] * g;
            }
        }
    }
    // bond orders, site energy (accumulated in FP64), pair-derivative factor
    // pd_c and P_c
    double u_i = 0.0;
    for (int c = 0; c < cnt; ++c) {
        if (c < cnt) {
            const auto& pp = pair_of<T, MULTI>(K, L, tp[c]);
            T b, db;
            bond_order(pc, zp[c], b, db);
            if constexpr (MULTI) {
                b *= pp.chi;
                db *= pp.chi;
            }
            const T fr = pp.A * t_exp(-pp.lam * rr[c]);
            const T fa = pp.B * t_exp(-pp.mu * rr[c]);
            u_i += (double)(fc[c] * (fr - b * fa));
            pd[c] = dfc[c] * (fr - b * fa) + fc[c] * (-pp.lam * fr + b * pp.mu * fa);
            zp[c] = fc[c] * fa * db;
        }
    }
    U[i] = 0.5 * u_i;
    // partials dU_i/dr_c
    for (int c = 0; c < cnt; ++c) {
        if (c < cnt) {
            const T ir = nr_rcp(rr[c]);
            T dx = T(0.5) * pd[c] * ux[c], dy = T(0.5) * pd[c] * uy[c], dz = T(0.5) * pd[c] * uz[c];
            for (int e = 0; e < cnt; ++e) {
                if (e != c && e < cnt) {
                    const T cs = ux[c] * ux[e] + uy[c] * uy[e] + uz[c] * uz[e];
                    T g, dg;
                    angular_g(pc, cs, g, dg);
                    const T a = T(-0.5) * (zp[c] * fc[e] + zp[e] * fc[c]) * dg * ir;
                    const T bb = T(-0.5) * zp[e] * dfc[c] * g;
                    dx += a * (ux[e] - cs * ux[c]) + bb * ux[c];
                    dy += a * (uy[e] - cs * uy[c]) + bb * uy[c];
                    dz += a * (uz[e] - cs * uz[c]) + bb * uz[c];
                }
            }
            T* o = dpart + ((int64_t)slot[c] * cap + i) * 3;
            o[0] = dx;
            o[1] = dy;
            o[2] = dz;
        }
    }
}

// Cutoff mask of atom i with a cutoff per type pair (the multi-type form of
// quad_cutoff_mask); also returns the type of the lane's first-slot
// neighbour.
__device__ __forceinline__ unsigned long long quad_cutoff_mask_typed(
    const double4& xi, int ti, int64_t i, int64_t cap, int nnb, int q, const int* __restrict__ nl,
    const double4* __restrict__ xw, const Box& box, const double* S2, Disp& d_first, int& t_first)
{
    unsigned long long msk = 0;
    d_first = Disp{0.0, 0.0, 0.0, 0.0};
    t_first = 0;
    int m = q;
    // two entries per iteration, both loads issued before either test
    for (; m + kQuad < nnb; m += 2 * kQuad) {
        const int j0 = nl[(int64_t)m * cap + i];
        const int j1 = nl[(int64_t)(m + kQuad) * cap + i];
        const double4 x0 = xw[j0], x1 = xw[j1];
        const int t0 = (int)x0.w, t1 = (int)x1.w;
        const Disp d0 = cut_disp(xi, x0, box), d1 = cut_disp(xi, x1, box);
        if (m == q) {
            d_first = d0;
            t_first = t0;
        }
        if (d0.r2 < S2[ti * kMaxTypes + t0]) msk |= 1ull << m;
        if (d1.r2 < S2[ti * kMaxTypes + t1]) msk |= 1ull << (m + kQuad);
    }
    if (m < nnb) {
        const double4 xj = xw[nl[(int64_t)m * cap + i]];
        const int tj = (int)xj.w;
        const Disp d = cut_disp(xi, xj, box);
        if (m == q) {
            d_first = d;
            t_first = tj;
        }
        if (d.r2 < S2[ti * kMaxTypes + tj]) msk |= 1ull << m;
    }
    return quad_or(msk);
}

// Partner terms of the partials of the quad site pass: for each own bond c
// and partner bond e of the same atom (fetched from the other lanes),
//   dU_i/dr_c += -1/2 (P_c f_C(r_e) + P_e f_C(r_c)) g'(cos_ce) (u_e - cos_ce u_c) / r_c
//               - 1/2 P_e f_C'(r_c) g(cos_ce) u_c.
// FULL: every bond of the wave lies below R, where f_C = 1 and f_C' = 0, so
// the partners' f_C are not fetched and the last term vanishes (the same
// values: products by 1 and sums with 0 are exact).
template <class T, int SLOTS, bool FULL, class P>
__device__ __forceinline__ void tersoff_partner_terms(
    const P& pc, int q, int kc, int tmax, const T (&ux)[SLOTS], const T (&uy)[SLOTS],
    const T (&uz)[SLOTS], const T (&ir)[SLOTS], const T (&fc)[SLOTS], const T (&dfc)[SLOTS],
    const T (&zp)[SLOTS], const T (&g0)[kQuad], const T (&dg0)[kQuad], T (&gx)[SLOTS],
    T (&gy)[SLOTS], T (&gz)[SLOTS])
{
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) {
        if (t >= tmax) break;   // wave-uniform
#pragma unroll
        for (int k = 0; k < kQuad; ++k) {
            const T ex = k ? quad_xor(ux[t], k) : ux[t];
            const T ey = k ? quad_xor(uy[t], k) : uy[t];
            const T ez = k ? quad_xor(uz[t], k) : uz[t];
            const T ef = FULL ? T(1) : (k ? quad_xor(fc[t], k) : fc[t]);
            const T ep = k ? quad_xor(zp[t], k) : zp[t];
            const int e = (q ^ k) + kQuad * t;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                if (s >= tmax) break;   // wave-uniform: own slots past it are empty
                const int c = q + kQuad * s;
                if (c < kc && e < kc && e != c) {
                    const T cs = ux[s] * ex + uy[s] * ey + uz[s] * ez;
                    T g, dg;
                    if (s == 0 && t == 0) {
                        g = g0[k];
                        dg = dg0[k];
                    } else {
                        angular_g(pc, cs, g, dg);
                    }
                    if constexpr (FULL) {
                        const T a = T(-0.5) * (zp[s] + ep) * dg * ir[s];
                        gx[s] += a * (ex - cs * ux[s]);
                        gy[s] += a * (ey - cs * uy[s]);
                        gz[s] += a * (ez - cs * uz[s]);
                    } else {
                        const T a = T(-0.5) * (zp[s] * ef + ep * fc[s]) * dg * ir[s];
                        const T bb = T(-0.5) * ep * dfc[s] * g;
                        gx[s] += a * (ex - cs * ux[s]) + bb * ux[s];
                        gy[s] += a * (ey - cs * uy[s]) + bb * uy[s];
                        gz[s] += a * (ez - cs * uz[s]) + bb * uz[s];
                    }
                }
            }
        }
    }
}

// Quad site pass: four lanes per atom, lane q owning bonds q, q + 4, ....  The
// arithmetic is the one of tersoff_site, distributed over the quad: each lane
// forms zeta_c, b_c and dU_i/dr_c for its own bonds c, fetching the partner
// bonds' unit vectors, f_C and P from the other lanes.  Atoms with more than
// kQuad * SLOTS in-cutoff bonds go to the overflow list.
// The single-type FP64 pass is held to 96 VGPRs, five waves per SIMD (it
// needs 97 otherwise and spills a few values instead, measured faster); the
// others keep their natural allocation.
template <class T, int SLOTS, bool MULTI>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(MULTI || sizeof(T) == 4 ? 1 : 5, 8)))
k_tersoff_site_quad(TersoffArg<T, MULTI> K, double rc2, Segs S, int M, int64_t cap,
                    const double4* __restrict__ xw, const int* __restrict__ nn,
                    const int* __restrict__ nl, unsigned long long* __restrict__ mask,
                    double* __restrict__ U, T* __restrict__ dpart, int* __restrict__ ovf_count,
                    int* __restrict__ ovf_list)
{
    __shared__ TersoffLds<T> L;
    __shared__ int order[MULTI ? kQuadAtoms : 1];
    constexpr bool kPoly = !MULTI && sizeof(T) == 8;   // the bond-order polynomial
    __shared__ double bp[kPoly ? kBPolyTerms + 3 : 1];
    const int q = threadIdx.x & (kQuad - 1);
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int sid = seg_of_block(S, lb, true);
    const Seg& g = S.seg[sid];
    const int phase = S.phase_in[sid];
    if constexpr (kPoly) {
        if (threadIdx.x == 0) {
#pragma unroll
            for (int j = 0; j < kBPolyTerms; ++j) bp[j] = K.bpoly[j];
            bp[kBPolyTerms] = kBPolyU0;
            bp[kBPolyTerms + 1] = kBPolyLo;
            bp[kBPolyTerms + 2] = kBPolyHi;
        }
        // published by the barrier after the cutoff test
    }
    const int first = (lb - g.blk_quad) * kQuadAtoms;
    int a = threadIdx.x >> 2;
    if constexpr (MULTI) {
        // The block's atoms are taken in the order of a stable partition by
        // type, so that the waves of an element with few bonds (C in SiC)
        // do not run the partner-slot loops sized for one with many.  Wave
        // 0 (threads 0-63, one per atom) ranks the keys; atoms past the
        // segment's end sort last.
        if (threadIdx.x < kQuadAtoms) {
            const int loc = first + (int)threadIdx.x;
            const int key =
                loc < g.n ? min(max((int)xw[g.atom_off + loc].w, 0), kMaxTypes - 1) : kMaxTypes;
            const unsigned long long below = (1ull << threadIdx.x) - 1ull;
            int rank = 0;
#pragma unroll
            for (int t = 0; t <= kMaxTypes; ++t) {
                const unsigned long long m = __ballot(key == t);
                rank += t < key ? __popcll(m) : (t == key ? __popcll(m & below) : 0);
            }
            order[rank] = (int)threadIdx.x;
        }
        fill_lds_table(K, L);   // its barrier also publishes the order
        a = order[a];
    }
    const Box box = g.box;
    const int local = first + a;
    const int64_t i = g.atom_off + local;
    const bool valid = local < g.n;
    const double4 xi = valid ? xw[i] : make_double4(0.0, 0.0, 0.0, 0.0);
    const int ti = MULTI ? (int)xi.w : 0;
    const int nnb = valid ? min(nn[i], M) : 0;
    // A finished segment (kept for retrieval) is left as it is.  The test
    // follows the first loads, which are in bounds for it too, so that they
    // share one wait with it (block-uniform: before any barrier of the block
    // that the others would miss).
    if (phase > g.nsteps) return;
    Disp d_first;
    int t_first = 0;
    unsigned long long msk;
    if constexpr (MULTI)
        msk = quad_cutoff_mask_typed(xi, ti, i, cap, nnb, q, nl, xw, box, L.S2, d_first, t_first);
    else
        msk = quad_cutoff_mask<false>(xi, i, cap, nnb, q, nl, xw, box, rc2, d_first);
    if constexpr (kPoly) {
        // The coefficients are the only LDS data written so far (an LDS-only
        // fence); the wait sits behind the cutoff test's gathers.
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    }
    const int cnt = __popcll(msk);
    const bool ovf = cnt > kQuad * SLOTS;
    if (valid && q == 0) {
        mask[i] = msk;
        if (ovf) ovf_list[atomicAdd(ovf_count, 1)] = (int)i;
    }
    const int kc = (valid && !ovf) ? cnt : 0;   // bonds handled by this quad
    const auto& pc = center_of<T, MULTI>(K, L, ti);

    T ux[SLOTS], uy[SLOTS], uz[SLOTS], rr[SLOTS], ir[SLOTS],
        fc[SLOTS], dfc[SLOTS], zp[SLOTS], pd[SLOTS];
    int slot[SLOTS], tp[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int c = q + kQuad * s;
        ux[s] = uy[s] = uz[s] = fc[s] = dfc[s] = zp[s] = pd[s] = T(0);
        rr[s] = ir[s] = T(1);
        slot[s] = 0;
        tp[s] = 0;
        if (c < kc) {
            const int m = nth_set_bit(msk, c);
            slot[s] = m;
            Disp d;
            if (s == 0 && m == q) {
                d = d_first;
                if (MULTI) tp[s] = ti * kMaxTypes + t_first;
            } else {
                const double4 xj = xw[nl[(int64_t)m * cap + i]];
                d = cut_disp(xi, xj, box);
                if (MULTI) tp[s] = ti * kMaxTypes + (int)xj.w;
            }
            bond_geometry(d, ux[s], uy[s], uz[s], rr[s], ir[s]);
            cutoff_fc(pair_of<T, MULTI>(K, L, tp[s]), rr[s], fc[s], dfc[s]);
        }
    }
    const int tmax = wave_partner_slots<SLOTS>(kc);
    // every bond of the wave below R (f_C = 1, f_C' = 0): wave-uniform
    bool partial = false;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) partial = partial || (q + kQuad * s < kc && fc[s] != T(1));
    const bool full = !__any(partial);

    // zeta_c = sum over partner bonds e != c of f_C(r_e) g(cos_ce).  g and g'
    // of the angles between first-slot bonds (every angle of an atom with at
    // most kQuad bonds) are kept for the derivative phase.
    T g0[kQuad], dg0[kQuad];
#pragma unroll
    for (int k = 0; k < kQuad; ++k) g0[k] = dg0[k] = T(0);
    if (tmax == 1) {   // wave-uniform: every bond is its lane's first slot
        // The angle of bonds c and e is the same value for both lanes, so
        // the lanes evaluate different angles in one instruction: lane q
        // takes (q, q+1 mod 4) and (q, q xor 2), and receives (q-1 mod 4, q)
        // from lane q-1; the three give bond q's partners q xor 1, 2, 3.
        // Products and fused adds are symmetric in their factors, so every
        // value has the bits lane q would compute itself.
        const int qa = (q + 1) & 3, qb = q ^ 2;
        const T ax = quad_rot<1>(ux[0]), ay = quad_rot<1>(uy[0]), az = quad_rot<1>(uz[0]);
        const T bx = quad_xor_k<2>(ux[0]), by = quad_xor_k<2>(uy[0]), bz = quad_xor_k<2>(uz[0]);
        T gA = T(0), dgA = T(0), gB = T(0), dgB = T(0);
        if (q < kc && qa < kc) {
            const T cs = ux[0] * ax + uy[0] * ay + uz[0] * az;
            angular_g(pc, cs, gA, dgA);
        }
        if (q < kc && qb < kc) {
            const T cs = ux[0] * bx + uy[0] * by + uz[0] * bz;
            angular_g(pc, cs, gB, dgB);
        }
        const T gP = quad_rot<-1>(gA), dgP = quad_rot<-1>(dgA);
        const bool even = (q & 1) == 0;
        g0[1] = even ? gA : gP;
        dg0[1] = even ? dgA : dgP;
        g0[2] = gB;
        dg0[2] = dgB;
        g0[3] = even ? gP : gA;
        dg0[3] = even ? dgP : dgA;
        if (full) {   // wave-uniform: partners' f_C are 1
            if (q < kc) {
                if ((q ^ 1) < kc) zp[0] += g0[1];
                if ((q ^ 2) < kc) zp[0] += g0[2];
                if ((q ^ 3) < kc) zp[0] += g0[3];
            }
        } else {
            const T ef1 = quad_xor_k<1>(fc[0]), ef2 = quad_xor_k<2>(fc[0]),
                    ef3 = quad_xor_k<3>(fc[0]);
            if (q < kc) {
                if ((q ^ 1) < kc) zp[0] += ef1 * g0[1];
                if ((q ^ 2) < kc) zp[0] += ef2 * g0[2];
                if ((q ^ 3) < kc) zp[0] += ef3 * g0[3];
            }
        }
    }
#pragma unroll
    for (int t = 0; t < SLOTS; ++t) {
        if (tmax == 1 || t >= tmax) break;   // wave-uniform
#pragma unroll
        for (int k = 0; k < kQuad; ++k) {
            const T ex = k ? quad_xor(ux[t], k) : ux[t];
            const T ey = k ? quad_xor(uy[t], k) : uy[t];
            const T ez = k ? quad_xor(uz[t], k) : uz[t];
            const T ef = k ? quad_xor(fc[t], k) : fc[t];
            const int e = (q ^ k) + kQuad * t;
#pragma unroll
            for (int s = 0; s < SLOTS; ++s) {
                if (s >= tmax) break;   // wave-uniform: own slots past it are empty
                const int c = q + kQuad * s;
                if (c < kc && e < kc && e != c) {
                    const T cs = ux[s] * ex + uy[s] * ey + uz[s] * ez;
                    T g, dg;
                    angular_g(pc, cs, g, dg);
                    zp[s] += ef * g;
                    if (s == 0 && t == 0) {
                        g0[k] = g;
                        dg0[k] = dg;
                    }
                }
            }
        }
    }
    // bond orders, site energy, pd_c and P_c
    double u_i = 0.0;
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        const int c = q + kQuad * s;
        if (c < kc) {
            const auto& pp = pair_of<T, MULTI>(K, L, tp[s]);
            T b, db;
            bond_order(pc, zp[s], b, db, kPoly ? bp : nullptr);
            if constexpr (MULTI) {
                b *= pp.chi;
                db *= pp.chi;
            }
            const T fr = pp.A * t_exp(-pp.lam * rr[s]);
            const T fa = pp.B * t_exp(-pp.mu * rr[s]);
            u_i += (double)(fc[s] * (fr - b * fa));
            pd[s] = dfc[s] * (fr - b * fa) + fc[s] * (-pp.lam * fr + b * pp.mu * fa);
            zp[s] = fc[s] * fa * db;
        }
    }
    u_i = quad_sum(u_i);
    if (q == 0 && kc > 0) U[i] = 0.5 * u_i;
    if (q == 0 && valid && !ovf && kc == 0) U[i] = 0.0;

    // partials dU_i/dr_c.  A wave all of whose bonds lie below R takes the
    // body without f_C and f_C' (a uniform branch, so only one body is
    // issued).
    T gx[SLOTS], gy[SLOTS], gz[SLOTS];
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
        gx[s] = T(0.5) * pd[s] * ux[s];
        gy[s] = T(0.5) * pd[s] * uy[s];
        gz[s] = T(0.5) * pd[s] * uz[s];
    }
    if (full)
        tersoff_partner_terms<T, SLOTS, true>(pc, q, kc, tmax, ux, uy, uz, ir, fc, dfc, zp, g0, dg0,
                                              gx, gy, gz);
    else
        tersoff_partner_terms<T, SLOTS, false>(pc, q, kc, tmax, ux, uy, uz, ir, fc, dfc, zp, g0,
                                               dg0, gx, gy, gz);
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

// Atoms whose in-cutoff count exceeded the main tile; the tile here covers
// the whole list capacity.
template <class T, bool MULTI>
__global__ void __launch_bounds__(kBlock)
k_tersoff_partials_ovf(TersoffArg<T, MULTI> K, Segs S, int64_t cap, const double4* __restrict__ xw,
                       const int* __restrict__ nl, const unsigned long long* __restrict__ mask,
                       double* __restrict__ U, T* __restrict__ dpart,
                       const int* __restrict__ ovf_count, const int* __restrict__ ovf_list)
{
    __shared__ TersoffLds<T> L;
    if constexpr (MULTI) fill_lds_table(K, L);
    const int total = *ovf_count;
    for (int k = blockIdx.x * kBlock + threadIdx.x; k < total; k += gridDim.x * kBlock) {
        const int64_t i = ovf_list[k];
        const double4 xi = xw[i];
        const Box box = S.seg[seg_of_atom(S, i)].box;
        const unsigned long long msk = mask[i];
        tersoff_site<T, kMaxSlots, MULTI>(K, L, i, cap, xi, msk, __popcll(msk), nl, xw,
                                                 box, U, dpart);
    }
}

constexpr int kOvfGrid = 64;

// rc2: the single element's cutoff squared (the multi-type table holds its own).
template <class T, bool MULTI>
hipError_t launch_tersoff_kernels(const Buffers& b, const Segs& S, int cur,
                                  const TersoffArg<T, MULTI>& k, double rc2, bool overflow_pass,
                                  int max_nn, hipStream_t s)
{
    constexpr int kSlots = MULTI ? kTersoffMultiSlots : kTersoffSlots;
    T* dp = static_cast<T*>(b.dpart);
    if (!overflow_pass) {
        k_tersoff_site_quad<T, kSlots, MULTI><<<S.nblk_quad, kBlock, 0, s>>>(
            k, rc2, S, b.M, b.cap, b.xw[cur], b.nn, b.nl, b.mask, b.U, dp, b.ovf_count,
            b.ovf_list);
        return hipGetLastError();
    }
    if (b.M > kQuad * kSlots && max_nn > kQuad * kSlots)
        k_tersoff_partials_ovf<T, MULTI><<<kOvfGrid, kBlock, 0, s>>>(
            k, S, b.cap, b.xw[cur], b.nl, b.mask, b.U, dp, b.ovf_count, b.ovf_list);
    return hipGetLastError();
}

template <class T>
hipError_t launch_tersoff_partials(const Buffers& b, const Segs& S, int cur,
                                   const TersoffTable& tab, bool overflow_pass, int max_nn,
                                   hipStream_t s)
{
    if (S.nblk_quad <= 0) return hipSuccess;
    if (!segs_ready(S, b) || tab.nt < 1 || tab.nt > kMaxTypes) return hipErrorInvalidValue;
    if (tab.nt > 1)
        return launch_tersoff_kernels<T, true>(b, S, cur, tersoff_table<T>(tab), 0.0,
                                               overflow_pass, max_nn, s);
    double rc2;
    const TersoffArg<T, false> k = tersoff_single<T>(tab, &rc2);
    return launch_tersoff_kernels<T, false>(b, S, cur, k, rc2, overflow_pass, max_nn, s);
}

template hipError_t launch_tersoff_partials<double>(const Buffers&, const Segs&, int,
                                                    const TersoffTable&, bool, int, hipStream_t);
template hipError_t launch_tersoff_partials<float>(const Buffers&, const Segs&, int,
                                                   const TersoffTable&, bool, int, hipStream_t);

}  // namespace mbmd
