// Staging kernels of the serving batch: admission of a structure into its
// atom range of the batch arrays, and copy-out of a finished structure.
// Each is one launch over the structure's atoms, so admitting or retiring
// costs the host one kernel launch.
#include "../../include/mbmd.h"
#include "mbmd_internal.h"

namespace mbmd {

// Positions go to both position buffers: a structure waits for the batch's
// next list-rebuild step before it starts, and until then no step carries
// its positions from one buffer to the other.
__global__ void __launch_bounds__(kBlock)
k_batch_admit(const double* __restrict__ pos, const double* __restrict__ vel, int64_t n, Box box,
              int atom_off, double4* __restrict__ xw0, double4* __restrict__ xw1,
              double* __restrict__ vel_dst, int64_t stride, unsigned* __restrict__ status,
              unsigned* __restrict__ sst)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double x = pos[i], y = pos[n + i], z = pos[2 * n + i];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
        atomicOr(status, ST_NONFINITE);
        atomicOr(sst, ST_NONFINITE);
        x = y = z = 0.0;
    }
    const double4 p = make_double4(wrap_coord(x, box.L[0]), wrap_coord(y, box.L[1]),
                                   wrap_coord(z, box.L[2]), 0.0);
    xw0[atom_off + i] = p;
    xw1[atom_off + i] = p;
#pragma unroll
    for (int r = 0; r < 3; ++r) vel_dst[r * stride + atom_off + i] = vel[r * n + i];
}

hipError_t launch_batch_admit(const double* pos, const double* vel, int64_t n, Box box,
                              int atom_off, double4* xw0, double4* xw1, double* vel_dst,
                              int64_t stride, unsigned* status, unsigned* sst, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    // the structure's status word starts clear (ordered before the admission)
    hipError_t e = launch_fill_int((int*)sst, 1, 0, s);
    if (e != hipSuccess) return e;
    k_batch_admit<<<blocks_for(n), kBlock, 0, s>>>(pos, vel, n, box, atom_off, xw0, xw1, vel_dst,
                                                   stride, status, sst);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock)
k_batch_copy_out(const double4* __restrict__ xw, const double* __restrict__ vel,
                 const double* __restrict__ U, const double* __restrict__ F,
                 const double* __restrict__ W, const double* __restrict__ J, int64_t stride,
                 int atom_off, int64_t n, double* __restrict__ pos_o, double* __restrict__ vel_o,
                 double* __restrict__ U_o, double* __restrict__ F_o, double* __restrict__ W_o,
                 double* __restrict__ J_o, const unsigned* __restrict__ sst,
                 int32_t* __restrict__ status_o)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i == 0 && status_o) {
        // one code per structure, the most fundamental condition first
        const unsigned st = *sst;
        int32_t code = MBMD_OK;
        if (st & ST_NONFINITE) code = MBMD_ENONFINITE;
        else if (st & ST_NEIGH_OVERFLOW) code = MBMD_ENEIGH;
        else if (st & ST_SKIN) code = MBMD_ESKIN;
        *status_o = code;
    }
    if (i >= n) return;
    const int64_t g = atom_off + i;
    if (pos_o) {
        const double4 p = xw[g];
        pos_o[i] = p.x;
        pos_o[n + i] = p.y;
        pos_o[2 * n + i] = p.z;
    }
    if (U_o) U_o[i] = U[g];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        if (vel_o) vel_o[r * n + i] = vel[r * stride + g];
        if (F_o) F_o[r * n + i] = F[r * stride + g];
        if (J_o) J_o[r * n + i] = J[r * stride + g];
    }
    if (W_o) {
#pragma unroll
        for (int r = 0; r < 9; ++r) W_o[r * n + i] = W[r * stride + g];
    }
}

hipError_t launch_batch_copy_out(const double4* xw, const double* vel, const double* U,
                                 const double* F, const double* W, const double* J,
                                 int64_t stride, int atom_off, int64_t n, double* pos_o,
                                 double* vel_o, double* U_o, double* F_o, double* W_o,
                                 double* J_o, const unsigned* sst, int32_t* status_o,
                                 hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_batch_copy_out<<<blocks_for(n), kBlock, 0, s>>>(xw, vel, U, F, W, J, stride, atom_off, n,
                                                      pos_o, vel_o, U_o, F_o, W_o, J_o, sst,
                                                      status_o);
    return hipGetLastError();
}

}  // namespace mbmd
