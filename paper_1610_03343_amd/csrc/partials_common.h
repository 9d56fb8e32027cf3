// Pieces shared by the per-atom partials kernels (Tersoff, Stillinger-Weber).
//
// A partials kernel owns atom i and computes, from atom i's own neighbour
// list only, its site energy U_i and the partial derivatives
// dU_i/dr_ij for every neighbour j inside the potential cutoff.  These are
// the two ingredients of the paper's explicit pairwise force
// F_ij = dU_i/dr_ij - dU_j/dr_ji (Section 2.3, generalised in Section 2.4).
// Nothing outside atom i's list is read and only atom i's slots are written.
#pragma once

#include "mbmd_internal.h"

namespace mbmd {

struct Disp {
    double x, y, z, r2;
};

// Minimum-image displacement r_ij = r_j - r_i and its square, in explicit
// operations: r_j - r_i, the product by 1/L and the rounding are exactly
// negated for the pair seen from j, and so are a fused multiply-add's
// operands and exact result, so the kernels for atom i and for atom j agree
// bit for bit on r_ij = -r_ji and r_ij^2 = r_ji^2, and the in-cutoff masks of
// the two atoms are mutually consistent.
__device__ __forceinline__ Disp cut_disp(const double4& a, const double4& b, const Box& box)
{
#pragma clang fp contract(off)
    Disp d;
    d.x = b.x - a.x;
    d.y = b.y - a.y;
    d.z = b.z - a.z;
    d.x = fma(-box.L[0], rint(d.x * box.inv[0]), d.x);
    d.y = fma(-box.L[1], rint(d.y * box.inv[1]), d.y);
    d.z = fma(-box.L[2], rint(d.z * box.inv[2]), d.z);
    d.r2 = fma(d.x, d.x, fma(d.y, d.y, d.z * d.z));
    return d;
}

// Reciprocal and reciprocal square root: the hardware estimate refined by
// Newton's method, y <- y (2 - x y) and y <- y (3 - x y^2) / 2, twice in
// double (each step squares the relative error) and once in float.  Inputs
// are positive normal numbers here (bond lengths, sums of squares).
__device__ __forceinline__ double nr_rcp(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = fma(fma(-x, y, 1.0), y, y);
    return fma(fma(-x, y, 1.0), y, y);
}
__device__ __forceinline__ float nr_rcp(float x)
{
    const float y = __builtin_amdgcn_rcpf(x);
    return fmaf(fmaf(-x, y, 1.0f), y, y);
}
__device__ __forceinline__ double nr_rsqrt(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
    return fma(0.5 * y, fma(-x * y, y, 1.0), y);
}
__device__ __forceinline__ float nr_rsqrt(float x)
{
    const float y = __builtin_amdgcn_rsqf(x);
    return fmaf(0.5f * y, fmaf(-x * y, y, 1.0f), y);
}

// A 64-bit constant placed in scalar registers where it is used: moved there
// by the scalar unit, then read as the scalar operand of a vector
// instruction.  Written as a plain literal, a coefficient can instead be
// moved into vector registers, two vector instructions per use, in kernels
// whose scalar registers are otherwise full.
__device__ __forceinline__ double sgpr_const(double c)
{
    asm volatile("" : "+s"(c));
    return c;
}

// e^x for |x| < 708 (the range of every exponential of the potentials
// here: bond terms of lengths inside the cutoff, the bond order's
// (beta zeta)^n): x = k ln 2 + r with k = rint(x / ln 2) and |r| <= ln 2 / 2
// by Cody and Waite's reduction (ln 2 as its double and the rounded
// remainder, each product exact in the fused multiply-add), e^r by its
// Taylor series to r^13 (truncation below 5e-18 relative), and 2^k applied
// exactly.  Within 1 ulp of the correctly rounded e^x.
__device__ __forceinline__ double fast_exp(double x)
{
    const double k = rint(x * sgpr_const(0x1.71547652b82fep+0));
    double r = fma(-k, sgpr_const(0x1.62e42fefa39efp-1), x);
    r = fma(-k, sgpr_const(0x1.abc9e3b39803fp-56), r);
    double p = fma(sgpr_const(0x1.6124613a86d09p-33), r, sgpr_const(0x1.1eed8eff8d898p-29));
    p = fma(p, r, sgpr_const(0x1.ae64567f544e4p-26));
    p = fma(p, r, sgpr_const(0x1.27e4fb7789f5cp-22));
    p = fma(p, r, sgpr_const(0x1.71de3a556c734p-19));
    p = fma(p, r, sgpr_const(0x1.a01a01a01a01ap-16));
    p = fma(p, r, sgpr_const(0x1.a01a01a01a01ap-13));
    p = fma(p, r, sgpr_const(0x1.6c16c16c16c17p-10));
    p = fma(p, r, sgpr_const(0x1.1111111111111p-7));
    p = fma(p, r, sgpr_const(0x1.5555555555555p-5));
    p = fma(p, r, sgpr_const(0x1.5555555555555p-3));
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)k);
}

// Bit m of the returned mask is set iff list slot m of atom i is inside the
// cutoff (r^2 < rc2).
__device__ __forceinline__ unsigned long long cutoff_mask(const double4& xi, int64_t i, int64_t cap,
                                                          int nnb, const int* __restrict__ nl,
                                                          const double4* __restrict__ xw,
                                                          const Box& box, double rc2)
{
    unsigned long long msk = 0;
    for (int m = 0; m < nnb; ++m) {
        const int j = nl[(int64_t)m * cap + i];
        const Disp d = cut_disp(xi, xw[j], box);
        if (d.r2 < rc2) msk |= 1ull << m;
    }
    return msk;
}

// ---- quad layout: four lanes per atom ------------------------------------
//
// The site passes run one atom per aligned group of four lanes.  Lane q owns
// the in-cutoff bonds c = q + 4 s (s = 0 .. SLOTS-1) of its atom, where bond
// c is the c-th set bit of the atom's cutoff mask (ascending list slot); the
// lanes exchange bond data with __shfl_xor inside the group.  Atoms with more
// than 4 SLOTS in-cutoff bonds go to the overflow pass.
static_assert(kQuadAtoms * kQuad == kBlock, "a quad block holds kQuadAtoms atoms");

// Number of partner bond slots a wave must visit: the largest in-cutoff
// count of its atoms, in slots (wave-uniform, so every lane joins the
// shuffles).
template <int SLOTS>
__device__ __forceinline__ int wave_partner_slots(int kc)
{
    int tmax = 1;
#pragma unroll
    for (int t = 1; t < SLOTS; ++t)
        if (__any(kc > kQuad * t)) tmax = t + 1;
    return tmax;
}

// Value of lane (q xor k) of the same quad, k = 1, 2, 3 a compile-time
// constant after unrolling: a DPP quad permutation (a register move inside
// the vector unit, no LDS round trip).  Every lane of the wave is active at
// each call site.
template <int K>
__device__ __forceinline__ int quad_xor_i32(int v)
{
    static_assert(K >= 1 && K <= 3, "quad partner");
    // quad_perm selectors: lane l of each quad reads lane l ^ K
    constexpr int ctrl = K == 1 ? 0xB1 : (K == 2 ? 0x4E : 0x1B);
    return __builtin_amdgcn_mov_dpp(v, ctrl, 0xF, 0xF, false);
}
template <int K>
__device__ __forceinline__ double quad_xor_k(double v)
{
    const int lo = quad_xor_i32<K>(__double2loint(v));
    const int hi = quad_xor_i32<K>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
template <int K>
__device__ __forceinline__ float quad_xor_k(float v)
{
    return __int_as_float(quad_xor_i32<K>(__float_as_int(v)));
}
template <class T>
__device__ __forceinline__ T quad_xor(T v, int k)
{
    return k == 0 ? v : (k == 1 ? quad_xor_k<1>(v) : (k == 2 ? quad_xor_k<2>(v) : quad_xor_k<3>(v)));
}

// Value of lane (q + D) mod 4 of the same quad, D = +1 or -1 (a DPP quad
// rotation).  Every lane of the wave is active at each call site.
template <int D>
__device__ __forceinline__ int quad_rot_i32(int v)
{
    static_assert(D == 1 || D == -1, "quad rotation");
    // quad_perm selectors: lane l reads lane (l + 1) & 3 (0x39) or (l + 3) & 3 (0x93)
    constexpr int ctrl = D == 1 ? 0x39 : 0x93;
    return __builtin_amdgcn_mov_dpp(v, ctrl, 0xF, 0xF, false);
}
template <int D>
__device__ __forceinline__ double quad_rot(double v)
{
    const int lo = quad_rot_i32<D>(__double2loint(v));
    const int hi = quad_rot_i32<D>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
template <int D>
__device__ __forceinline__ float quad_rot(float v)
{
    return __int_as_float(quad_rot_i32<D>(__float_as_int(v)));
}

__device__ __forceinline__ unsigned long long quad_or(unsigned long long v)
{
    int lo = (int)(unsigned)v, hi = (int)(unsigned)(v >> 32);
    lo |= quad_xor_i32<1>(lo);
    hi |= quad_xor_i32<1>(hi);
    lo |= quad_xor_i32<2>(lo);
    hi |= quad_xor_i32<2>(hi);
    return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

// Fixed-order sum over the quad: ((l0 + l1) + (l2 + l3)) on every lane.
__device__ __forceinline__ double quad_sum(double v)
{
    v += quad_xor_k<1>(v);
    v += quad_xor_k<2>(v);
    return v;
}

// Slot of the c-th set bit of msk (c < popcount(msk)).
__device__ __forceinline__ int nth_set_bit(unsigned long long msk, int c)
{
    for (int k = 0; k < c; ++k) msk &= msk - 1;
    return __builtin_ctzll(msk);
}

// Cutoff mask of atom i computed by its quad: lane q tests slots q, q+4, ...
// and keeps the displacement of its first slot in d_first (the bond that
// lane owns first whenever the atom's first slots are all in the cutoff).
// TWO: four, then two, entries per iteration with their loads issued first,
// for long lists (SW's ~16 entries: 11 % off its site pass); short Tersoff
// lists keep the plain loop.
template <bool TWO>
__device__ __forceinline__ unsigned long long quad_cutoff_mask(const double4& xi, int64_t i,
                                                               int64_t cap, int nnb, int q,
                                                               const int* __restrict__ nl,
                                                               const double4* __restrict__ xw,
                                                               const Box& box, double rc2,
                                                               Disp& d_first)
{
    unsigned long long msk = 0;
    d_first = Disp{0.0, 0.0, 0.0, 0.0};
    int m = q;
    for (; TWO && m + 3 * kQuad < nnb; m += 4 * kQuad) {
        int jv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) jv[u] = nl[(int64_t)(m + u * kQuad) * cap + i];
        double4 xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = xw[jv[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const Disp d = cut_disp(xi, xv[u], box);
            if (u == 0 && m == q) d_first = d;
            if (d.r2 < rc2) msk |= 1ull << (m + u * kQuad);
        }
    }
    for (; TWO && m + kQuad < nnb; m += 2 * kQuad) {
        const int j0 = nl[(int64_t)m * cap + i];
        const int j1 = nl[(int64_t)(m + kQuad) * cap + i];
        const double4 x0 = xw[j0], x1 = xw[j1];
        const Disp d0 = cut_disp(xi, x0, box), d1 = cut_disp(xi, x1, box);
        if (m == q) d_first = d0;
        if (d0.r2 < rc2) msk |= 1ull << m;
        if (d1.r2 < rc2) msk |= 1ull << (m + kQuad);
    }
    for (; m < nnb; m += kQuad) {
        const Disp d = cut_disp(xi, xw[nl[(int64_t)m * cap + i]], box);
        if (m == q) d_first = d;
        if (d.r2 < rc2) msk |= 1ull << m;
    }
    return quad_or(msk);
}

}  // namespace mbmd
