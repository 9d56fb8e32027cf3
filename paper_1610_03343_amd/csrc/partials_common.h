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

// Minimum-image displacement r_ij = r_j - r_i and its square, with no
// contraction to fused multiply-add: the kernels for atom i and for atom j
// then agree bit for bit on r_ij^2 = r_ji^2, so the in-cutoff masks of the
// two atoms are mutually consistent.
__device__ __forceinline__ Disp cut_disp(const double4& a, const double4& b, const Box& box)
{
#pragma clang fp contract(off)
    Disp d;
    d.x = b.x - a.x;
    d.y = b.y - a.y;
    d.z = b.z - a.z;
    d.x = d.x - box.L[0] * rint(d.x * box.inv[0]);
    d.y = d.y - box.L[1] * rint(d.y * box.inv[1]);
    d.z = d.z - box.L[2] * rint(d.z * box.inv[2]);
    d.r2 = d.x * d.x + d.y * d.y + d.z * d.z;
    return d;
}

// Bit m of the returned mask is set iff list slot m of atom i is inside the
// cutoff (r^2 < rc2).
__device__ __forceinline__ unsigned long long cutoff_mask(const double4& xi, int64_t i, int64_t n,
                                                          int nnb, const int* __restrict__ nl,
                                                          const double4* __restrict__ xw,
                                                          const Box& box, double rc2)
{
    unsigned long long msk = 0;
    for (int m = 0; m < nnb; ++m) {
        const int j = nl[(int64_t)m * n + i];
        const Disp d = cut_disp(xi, xw[j], box);
        if (d.r2 < rc2) msk |= 1ull << m;
    }
    return msk;
}

}  // namespace mbmd
