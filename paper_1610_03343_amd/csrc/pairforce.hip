// Pairwise-force pass with the fused velocity-Verlet update.
//
// One thread owns atom i and, over the in-cutoff neighbours j of its list,
// forms the paper's explicit pairwise force (Sections 2.3 and 2.4)
//   F_ij = dU_i/dr_ij - dU_j/dr_ji
// from the partials the site-local pass stored for i (at slot m of i's list)
// and for j (at the slot of i in j's list), and accumulates in FP64 registers
//   F_i = sum_j F_ij,   W_i = -1/2 sum_j r_ij (x) F_ij,
//   M_i = sum_j r_ij (x) dU_j/dr_ji   so that   J_i = M_i v_i
//       = sum_j r_ij (dU_j/dr_ji . v_i).
// Every output of atom i is written once, by its own thread: no write
// conflict and no atomics on results, the property the paper builds its GPU
// algorithm on.  J_i is formed after the second half-kick, so it pairs r(t)
// with v(t).  Optionally the thread then performs the next step's first
// half-kick and drift into the other position buffer (the neighbours'
// positions in the current buffer are still being read by other threads).
//
// Slot m of atom i is inside the cutoff iff slot rev of atom j is: both
// masks come from the same unfused evaluation of r^2, and
// (x_i - x_j)^2 equals (x_j - x_i)^2 bit for bit.
//
// Per-step totals (U, E_kin, W, J) are reduced per block in a fixed tree into
// a ring of per-step rows; a separate fold kernel sums each row in block
// order (a grid-wide fence inside this kernel would have to write back the
// L2 of every XCD).
#include "mbmd_internal.h"

namespace mbmd {

// Value of another lane by a DPP move (a register move inside the vector
// unit): CTRL selects the pattern.  Every lane of the wave is active.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Largest value over the wave, the same value in every lane (fmax is exact,
// so the order does not matter).
__device__ __forceinline__ double wave_max(double v)
{
    v = fmax(v, dpp_move<0xB1>(v));
    v = fmax(v, dpp_move<0x4E>(v));
    v = fmax(v, dpp_move<0x124>(v));
    v = fmax(v, dpp_move<0x128>(v));
    return fmax(fmax(read_lane(v, 0), read_lane(v, 16)), fmax(read_lane(v, 32), read_lane(v, 48)));
}

// Sum over the wave, the same value in every lane: quads by DPP xor 1 and
// 2, rows of 16 lanes by DPP rotations by 4 and 8, then the four row totals
// (read from lanes 0, 16, 32, 48) added in a fixed order.
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_move<0xB1>(v);    // quad_perm 1,0,3,2: lane xor 1
    v += dpp_move<0x4E>(v);    // quad_perm 2,3,0,1: lane xor 2
    v += dpp_move<0x124>(v);   // row_ror:4
    v += dpp_move<0x128>(v);   // row_ror:8
    return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Value of lane u (0..3, a compile-time constant after unrolling) of the
// same quad: DPP quad_perm u,u,u,u.
__device__ __forceinline__ double quad_bcast(double v, int u)
{
    return u == 0 ? dpp_move<0x00>(v)
                  : (u == 1 ? dpp_move<0x55>(v) : (u == 2 ? dpp_move<0xAA>(v) : dpp_move<0xFF>(v)));
}

// Fixed-order sum over a block of NT threads of kPartialCols values per
// thread into lds_out (lds: one row per wave).
template <int NT>
__device__ __forceinline__ void block_sum_cols(double (&vals)[kPartialCols],
                                               double (*lds)[kPartialCols],
                                               double* lds_out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < kPartialCols; ++c) {
        const double s = wave_sum(vals[c]);
        if (lane == 0) lds[wave][c] = s;
    }
    __syncthreads();
    if (threadIdx.x < kPartialCols) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < NT / 64; ++k) s += lds[k][threadIdx.x];
        lds_out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Threads of the fold kernels (1024 threads, four times fewer rounds of
// loads, measured slower: the fold is bound by launch latency).
constexpr int kFoldThreads = kBlock;

// The pairwise pass comes in two forms with the same bits: one thread per
// atom (k_pair_gather) and, for launches of at most kQuadPairBlocks blocks of
// 256 atoms, where that form leaves the chip mostly idle and each thread's
// chain of dependent loads sets the time, four lanes per atom (k_pair_quad).
// Both add the bond terms in ascending slot order with the explicit
// operations below and integrate with the same unfused statements.  Their
// thermo partials differ only in where the last additions happen: each
// 64-atom group is summed by wave_sum with atom k in lane k; k_pair_gather
// adds a block's four group sums in order (block_sum_cols) and stores one
// row per 256-atom block, k_pair_quad stores the four group sums (rows 4b ..
// 4b + 3) and the fold adds them in the same order.  So a launch may take
// either form whatever structures it holds, and a structure gives the same
// results alone and in a batch.

struct Vec3 {
    double v[3];
};

// Minimum-image r_ij = x_j - x_i.
__device__ __forceinline__ Vec3 bond_vector(const double4& xi, const double4& xj, const Box& box)
{
#pragma clang fp contract(off)
    Vec3 r{{xj.x - xi.x, xj.y - xi.y, xj.z - xi.z}};
#pragma unroll
    for (int c = 0; c < 3; ++c) r.v[c] = fma(-box.L[c], rint(r.v[c] * box.inv[c]), r.v[c]);
    return r;
}

// F_i += F_ij, W_i -= 1/2 r_ij (x) F_ij, M_i += r_ij (x) p_ji.
__device__ __forceinline__ void add_bond_terms(const double (&fij)[3], const double (&dji)[3],
                                               const Vec3& r, double (&f)[3], double (&w)[9],
                                               double (&mm)[9])
{
#pragma clang fp contract(off)
#pragma unroll
    for (int k = 0; k < 3; ++k) f[k] = f[k] + fij[k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double hr = -0.5 * r.v[c];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            w[3 * c + k] = fma(hr, fij[k], w[3 * c + k]);
            mm[3 * c + k] = fma(r.v[c], dji[k], mm[3 * c + k]);
        }
    }
}

template <class T>
__global__ void __launch_bounds__(kBlock)
k_pair_gather(Segs S, int64_t cap, int64_t os, StepArgs a, const double4* __restrict__ xw,
              double4* __restrict__ xw_next, const double4* __restrict__ xbuild,
              const int* __restrict__ nl,
              const uint8_t* __restrict__ rev, const unsigned long long* __restrict__ mask,
              const T* __restrict__ dpart, const double* __restrict__ U,
              double* __restrict__ vel, double* __restrict__ F, double* __restrict__ W,
              double* __restrict__ J, int* __restrict__ ovf_count)
{
    __shared__ double lds[kBlock / 64][kPartialCols];
    __shared__ double lds_tot[kPartialCols];
    __shared__ double lds_max[kBlock / 64];
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int sid = seg_of_block(S, lb, false);
    const Seg& g = S.seg[sid];
    const int phase = S.phase_in[sid];
    if (lb == g.blk && threadIdx.x == 0)
        S.phase_out[sid] = phase > g.nsteps ? phase : phase + 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) *ovf_count = 0;   // consumed by the partials pass
    if (phase > g.nsteps) return;              // finished segment, kept for retrieval
    const bool kick_before = phase > 0, advance = !a.hold && phase < g.nsteps;
    const Box box = g.box;
    const int local = (lb - g.blk) * kBlock + threadIdx.x;
    const int64_t i = g.atom_off + local;

    double f[3] = {0, 0, 0}, w[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, mm[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double v[3] = {0, 0, 0}, jj[3] = {0, 0, 0}, ekin = 0.0, ui = 0.0, disp2 = 0.0;
    if (local < g.n) {
        const double4 xi = xw[i];
        const unsigned long long msk = mask[i];
        ui = U[i];
        // One bond (list slot m, neighbour j): F_ij, W_i and M_i terms, in
        // the explicit operations of add_bond_terms.
        auto bond = [&](const T* pij, const T* pji, const double4& xj) {
            const double dji0 = (double)pji[0], dji1 = (double)pji[1], dji2 = (double)pji[2];
            const double fij[3] = {(double)pij[0] - dji0, (double)pij[1] - dji1,
                                   (double)pij[2] - dji2};
            const double dji[3] = {dji0, dji1, dji2};
            add_bond_terms(fij, dji, bond_vector(xi, xj, box), f, w, mm);
        };
        // The in-cutoff slots in ascending order, four per iteration with
        // every load of them issued first; the sums take the bonds in the
        // same order as one at a time.
        unsigned long long rem = msk;
        while (rem) {
            int mk[4], nk = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                mk[u] = rem ? __builtin_ctzll(rem) : mk[0];
                if (rem) {
                    rem &= rem - 1;
                    ++nk;
                }
            }
            int64_t e[4];
            int jk[4], rk[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                e[u] = (int64_t)mk[u] * cap + i;
                jk[u] = nl[e[u]];
                rk[u] = rev[e[u]];
            }
            double4 xk[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) xk[u] = xw[jk[u]];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (u < nk) bond(dpart + e[u] * 3, dpart + ((int64_t)rk[u] * cap + jk[u]) * 3, xk[u]);
        }
        double hdt, kin;
        atom_mass_factors(g, xi.w, hdt, kin);
        // The integrator arithmetic is kept unfused so that it rounds exactly
        // like a plain IEEE evaluation of v += (dt/2) a and x += dt v.
        if (vel) {
#pragma clang fp contract(off)
            v[0] = vel[i];
            v[1] = vel[os + i];
            v[2] = vel[2 * os + i];
            if (kick_before) {
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c] += hdt * f[c];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c)
                jj[c] = mm[3 * c + 0] * v[0] + mm[3 * c + 1] * v[1] + mm[3 * c + 2] * v[2];
            ekin = kin * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        }
        // Outputs are not read again by the step loop: streaming stores keep
        // them from evicting the partials and positions that neighbours of
        // later atoms still gather from L2.
        __builtin_nontemporal_store(f[0], &F[i]);
        __builtin_nontemporal_store(f[1], &F[os + i]);
        __builtin_nontemporal_store(f[2], &F[2 * os + i]);
#pragma unroll
        for (int c = 0; c < 9; ++c) __builtin_nontemporal_store(w[c], &W[(int64_t)c * os + i]);
        __builtin_nontemporal_store(jj[0], &J[i]);
        __builtin_nontemporal_store(jj[1], &J[os + i]);
        __builtin_nontemporal_store(jj[2], &J[2 * os + i]);
        if (vel && advance) {
#pragma clang fp contract(off)
            double vn[3], x[3] = {xi.x, xi.y, xi.z};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                vn[c] = v[c] + hdt * f[c];
                x[c] = wrap_coord(x[c] + g.dt * vn[c], box.L[c]);
            }
            vel[i] = vn[0];
            vel[os + i] = vn[1];
            vel[2 * os + i] = vn[2];
            xw_next[i] = make_double4(x[0], x[1], x[2], xi.w);
            if (a.check_skin) {
                const double4 xb = xbuild[i];
                double d[3] = {x[0] - xb.x, x[1] - xb.y, x[2] - xb.z};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    d[c] -= box.L[c] * rint(d[c] * box.inv[c]);
                    disp2 += d[c] * d[c];
                }
            }
        } else {
            // last step of this segment: full-step velocity, positions carried
            // into the buffer the next launch reads
            if (vel && kick_before) {
                vel[i] = v[0];
                vel[os + i] = v[1];
                vel[2 * os + i] = v[2];
            }
            if (!a.hold) xw_next[i] = xi;
        }
    }

    // largest squared displacement since the list build: one atomic per
    // block into the run's slot, and (serving batch) the skin bit of the
    // block's structure
    if (a.check_skin) {
        const double m = wave_max(disp2);
        if ((threadIdx.x & 63) == 0) lds_max[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            double bm = lds_max[0];
#pragma unroll
            for (int k = 1; k < kBlock / 64; ++k) bm = fmax(bm, lds_max[k]);
            // non-negative doubles order like their bit patterns
            if (a.disp_slot) atomicMax(a.disp_slot, (unsigned long long)__double_as_longlong(bm));
            if (a.seg_status && bm > a.skin_half2) atomicOr(&a.seg_status[g.sidx], ST_SKIN);
        }
    }

    if (!a.part_row) return;
    // per-block partial sums (U, E_kin, W (9), J (3)) into this step's row of
    // the partials ring; the fold kernel sums a segment's blocks in order
    double vals[kPartialCols];
    vals[0] = ui;
    vals[1] = ekin;
#pragma unroll
    for (int c = 0; c < 9; ++c) vals[2 + c] = w[c];
#pragma unroll
    for (int c = 0; c < 3; ++c) vals[11 + c] = jj[c];
    block_sum_cols<kBlock>(vals, lds, lds_tot);
    if (threadIdx.x < kPartialCols) a.part_row[(int64_t)lb * kPartialCols + threadIdx.x] = lds_tot[threadIdx.x];
}

// Four lanes per atom, for launches of at most kQuadPairBlocks blocks of 256
// atoms: a block is one 64-atom group (the 64-atom blocks of the site pass).
// Lane q takes in-cutoff bonds q, q + 4, ...; in round t the quad's lanes
// hold bonds 4t .. 4t + 3 and every lane adds the four (broadcast within the
// quad) in slot order, so that each holds the atom's sums formed as one
// thread forms them.  Lane 0 finishes the atom with the statements of
// k_pair_gather; the thermo values pass through LDS so that wave 0 sums the
// group with atom k in lane k, into row 4b + k of 256-atom block b.
template <class T>
__global__ void __launch_bounds__(kBlock)
k_pair_quad(Segs S, int64_t cap, int64_t os, StepArgs a, const double4* __restrict__ xw,
            double4* __restrict__ xw_next, const double4* __restrict__ xbuild,
            const int* __restrict__ nl,
            const uint8_t* __restrict__ rev, const unsigned long long* __restrict__ mask,
            const T* __restrict__ dpart, const double* __restrict__ U,
            double* __restrict__ vel, double* __restrict__ F, double* __restrict__ W,
            double* __restrict__ J, int* __restrict__ ovf_count)
{
    __shared__ double lds_max[kBlock / 64];
    __shared__ double lds_vals[kPartialCols][kQuadAtoms];
    const int q = threadIdx.x & (kQuad - 1);
    const int atom = threadIdx.x >> 2;   // within the group
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int sid = seg_of_block(S, lb, true);
    const Seg& g = S.seg[sid];
    const int phase = S.phase_in[sid];
    if (lb == g.blk_quad && threadIdx.x == 0)
        S.phase_out[sid] = phase > g.nsteps ? phase : phase + 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) *ovf_count = 0;   // consumed by the partials pass
    if (phase > g.nsteps) return;              // finished segment, kept for retrieval
    const bool kick_before = phase > 0, advance = !a.hold && phase < g.nsteps;
    const Box box = g.box;
    const int group = lb - g.blk_quad;   // within the segment
    const int local = group * kQuadAtoms + atom;
    const int64_t i = g.atom_off + local;
    const bool valid = local < g.n;

    double f[3] = {0, 0, 0}, w[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, mm[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double v[3] = {0, 0, 0}, jj[3] = {0, 0, 0}, ekin = 0.0, ui = 0.0, disp2 = 0.0;
    const double4 xi = valid ? xw[i] : make_double4(0.0, 0.0, 0.0, 0.0);
    const unsigned long long msk = valid ? mask[i] : 0ull;
    if (valid) ui = U[i];
    const int nb = __popcll(msk);
    // rounds: as many as the wave's largest count needs (wave-uniform, so
    // every lane joins the broadcasts)
    const int rounds = (int)wave_max((double)((nb + kQuad - 1) / kQuad));
    unsigned long long rem = msk;
    for (int k = 0; k < q && rem; ++k) rem &= rem - 1;   // this lane's first bond: the q-th
    for (int t = 0; t < rounds; ++t) {
        double fij[3] = {0, 0, 0}, dji[3] = {0, 0, 0};
        Vec3 r{{0, 0, 0}};
        if (rem) {
            const int m = __builtin_ctzll(rem);
            const int64_t e = (int64_t)m * cap + i;
            const int j = nl[e];
            const int rv = rev[e];
            const T* pij = dpart + e * 3;
            const T* pji = dpart + ((int64_t)rv * cap + j) * 3;
            const double dji0 = (double)pji[0], dji1 = (double)pji[1], dji2 = (double)pji[2];
            fij[0] = (double)pij[0] - dji0;
            fij[1] = (double)pij[1] - dji1;
            fij[2] = (double)pij[2] - dji2;
            dji[0] = dji0;
            dji[1] = dji1;
            dji[2] = dji2;
            r = bond_vector(xi, xw[j], box);
        }
#pragma unroll
        for (int k = 0; k < kQuad; ++k)
            if (rem) rem &= rem - 1;   // next round: four bonds on
#pragma unroll
        for (int u = 0; u < kQuad; ++u) {
            double bf[3], bd[3];
            Vec3 br;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                bf[c] = quad_bcast(fij[c], u);
                bd[c] = quad_bcast(dji[c], u);
                br.v[c] = quad_bcast(r.v[c], u);
            }
            if (kQuad * t + u < nb) add_bond_terms(bf, bd, br, f, w, mm);
        }
    }
    if (valid) {
        double hdt, kin;
        atom_mass_factors(g, xi.w, hdt, kin);
        // the statements of k_pair_gather
        if (vel) {
#pragma clang fp contract(off)
            v[0] = vel[i];
            v[1] = vel[os + i];
            v[2] = vel[2 * os + i];
            if (kick_before) {
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c] += hdt * f[c];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c)
                jj[c] = mm[3 * c + 0] * v[0] + mm[3 * c + 1] * v[1] + mm[3 * c + 2] * v[2];
            ekin = kin * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        }
        if (q == 0) {
            __builtin_nontemporal_store(f[0], &F[i]);
            __builtin_nontemporal_store(f[1], &F[os + i]);
            __builtin_nontemporal_store(f[2], &F[2 * os + i]);
#pragma unroll
            for (int c = 0; c < 9; ++c) __builtin_nontemporal_store(w[c], &W[(int64_t)c * os + i]);
            __builtin_nontemporal_store(jj[0], &J[i]);
            __builtin_nontemporal_store(jj[1], &J[os + i]);
            __builtin_nontemporal_store(jj[2], &J[2 * os + i]);
            if (vel && advance) {
#pragma clang fp contract(off)
                double vn[3], x[3] = {xi.x, xi.y, xi.z};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    vn[c] = v[c] + hdt * f[c];
                    x[c] = wrap_coord(x[c] + g.dt * vn[c], box.L[c]);
                }
                vel[i] = vn[0];
                vel[os + i] = vn[1];
                vel[2 * os + i] = vn[2];
                xw_next[i] = make_double4(x[0], x[1], x[2], xi.w);
                if (a.check_skin) {
                    const double4 xb = xbuild[i];
                    double d[3] = {x[0] - xb.x, x[1] - xb.y, x[2] - xb.z};
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        d[c] -= box.L[c] * rint(d[c] * box.inv[c]);
                        disp2 += d[c] * d[c];
                    }
                }
            } else {
                if (vel && kick_before) {
                    vel[i] = v[0];
                    vel[os + i] = v[1];
                    vel[2 * os + i] = v[2];
                }
                if (!a.hold) xw_next[i] = xi;
            }
        }
    }
    if (a.check_skin) {
        const double m = wave_max(disp2);
        if ((threadIdx.x & 63) == 0) lds_max[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            double bm = lds_max[0];
#pragma unroll
            for (int k = 1; k < kBlock / 64; ++k) bm = fmax(bm, lds_max[k]);
            if (a.disp_slot) atomicMax(a.disp_slot, (unsigned long long)__double_as_longlong(bm));
            if (a.seg_status && bm > a.skin_half2) atomicOr(&a.seg_status[g.sidx], ST_SKIN);
        }
    }

    if (!a.part_row) return;
    if (q == 0) {
        lds_vals[0][atom] = ui;
        lds_vals[1][atom] = ekin;
#pragma unroll
        for (int c = 0; c < 9; ++c) lds_vals[2 + c][atom] = w[c];
#pragma unroll
        for (int c = 0; c < 3; ++c) lds_vals[11 + c][atom] = jj[c];
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int64_t row = 4 * (int64_t)(g.blk + group / 4) + group % 4;
#pragma unroll
        for (int c = 0; c < kPartialCols; ++c) {
            const double t = wave_sum(lds_vals[c][threadIdx.x]);
            if (threadIdx.x == 0) a.part_row[row * kPartialCols + c] = t;
        }
    }
}

// Sums one segment's block partials of one step (ring row rowp), in a fixed
// order, into its thermo row: 0 E_pot, 1 E_kin, 2..10 W, 11..13 J,
// 14 E_pot + E_kin, 15 kinetic temperature (k_B in eV/K, 3N - 3 degrees of
// freedom).  Called by every thread of a kFoldThreads block; thread 0 writes
// the row.
__device__ __forceinline__ void fold_segment_row(const double* __restrict__ rowp, const Segs& S,
                                                 const Seg& g, double (*lds)[kPartialCols],
                                                 double* lds_tot, double* __restrict__ row)
{
    // k_pair_quad's launches leave four group rows per block: their sum in
    // block_sum_cols' order (a group past the segment's end adds 0, as an
    // all-zero wave does there)
    const bool groups = S.nblk <= kQuadPairBlocks;
    const int b0 = g.blk, b1 = g.blk + blocks_for(g.n);
    double vals[kPartialCols];
#pragma unroll
    for (int c = 0; c < kPartialCols; ++c) vals[c] = 0.0;
    if (groups) {
        for (int b = b0 + threadIdx.x; b < b1; b += kFoldThreads) {
            const double* p = rowp + 4 * (int64_t)b * kPartialCols;
            const int a0 = (b - g.blk) * kBlock;
#pragma unroll
            for (int c = 0; c < kPartialCols; ++c) {
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < 4; ++k) t += a0 + 64 * k < g.n ? p[k * kPartialCols + c] : 0.0;
                vals[c] += t;
            }
        }
    } else {
        // block rows b, b + kFoldThreads, ... in order; the next row's loads
        // are issued before the current row is added (one wait per row
        // instead of a load-then-add chain)
        double cur[kPartialCols], nxt[kPartialCols];
        int b = b0 + threadIdx.x;
        if (b < b1) {
            const double* p = rowp + (int64_t)b * kPartialCols;
#pragma unroll
            for (int c = 0; c < kPartialCols; ++c) cur[c] = p[c];
        }
        for (; b < b1; b += kFoldThreads) {
            const int bn = b + kFoldThreads;
            if (bn < b1) {
                const double* p = rowp + (int64_t)bn * kPartialCols;
#pragma unroll
                for (int c = 0; c < kPartialCols; ++c) nxt[c] = p[c];
            }
#pragma unroll
            for (int c = 0; c < kPartialCols; ++c) {
                vals[c] += cur[c];
                cur[c] = nxt[c];
            }
        }
    }
    block_sum_cols<kFoldThreads>(vals, lds, lds_tot);
    if (threadIdx.x == 0) {
        const double n = (double)g.n;
#pragma unroll
        for (int c = 0; c < kPartialCols; ++c) row[c] = lds_tot[c];
        row[14] = lds_tot[0] + lds_tot[1];
        row[15] = g.n > 1 ? 2.0 * lds_tot[1] / ((3.0 * n - 3.0) * 8.617333262e-5) : 0.0;
    }
}

// One block per step of one segment: row k = first + blockIdx.x.
__global__ void __launch_bounds__(kFoldThreads)
k_thermo_fold(const double* __restrict__ part_b, int64_t blk_cap, Segs S, int sid, int first,
              int ring0, double* __restrict__ thermo)
{
    __shared__ double lds[kFoldThreads / 64][kPartialCols];
    __shared__ double lds_tot[kPartialCols];
    const int k = first + blockIdx.x;
    const double* rowp = part_b + (int64_t)((ring0 + k) % kThermoRing) * blk_cap * kPartialCols;
    fold_segment_row(rowp, S, S.seg[sid], lds, lds_tot, thermo + (int64_t)k * kThermoCols);
}

hipError_t launch_thermo_fold(const Buffers& b, const Segs& S, int sid, int first, int count,
                              int ring0, double* thermo, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (!S.seg || sid < 0 || sid >= S.nseg || !thermo) return hipErrorInvalidValue;
    k_thermo_fold<<<count, kFoldThreads, 0, s>>>(b.part_b, b.blk_cap, S, sid, first, ring0, thermo);
    return hipGetLastError();
}

// End of a one-structure run in one launch: blocks 0 .. count - 1 fold
// thermo rows first .. first + count - 1 from the ring (as k_thermo_fold with
// ring0 = 0), blocks count .. count + nblk - 1 copy the final positions xw
// back to the caller's pos[3][n] (as the store kernel does).
__global__ void __launch_bounds__(kFoldThreads)
k_end_single(const double* __restrict__ part_b, int64_t blk_cap, Segs S, int first,
             double* __restrict__ thermo, const double4* __restrict__ xw,
             double* __restrict__ pos)
{
    __shared__ double lds[kFoldThreads / 64][kPartialCols];
    __shared__ double lds_tot[kPartialCols];
    const Seg& g = S.seg[0];
    const int count = (int)gridDim.x - S.nblk;
    if ((int)blockIdx.x < count) {   // the folds' serial loops start first
        const int k = first + (int)blockIdx.x;
        const double* rowp = part_b + (int64_t)(k % kThermoRing) * blk_cap * kPartialCols;
        fold_segment_row(rowp, S, g, lds, lds_tot, thermo + (int64_t)k * kThermoCols);
        return;
    }
    const int64_t i =
        (int64_t)xcd_block((int)blockIdx.x - count, S.nblk) * kBlock + threadIdx.x;
    if (i >= g.n) return;
    const double4 p = xw[i];
    pos[i] = p.x;
    pos[g.n + i] = p.y;
    pos[2 * g.n + i] = p.z;
}

hipError_t launch_end_single(const Buffers& b, const Segs& S, int first, int count,
                             double* thermo, int cur, double* pos, hipStream_t s)
{
    if (!segs_ready(S, b) || S.nseg != 1 || !pos || count < 0 || (count > 0 && !thermo))
        return hipErrorInvalidValue;
    const int grid = S.nblk + count;
    if (grid <= 0) return hipSuccess;
    k_end_single<<<grid, kFoldThreads, 0, s>>>(b.part_b, b.blk_cap, S, first, thermo, b.xw[cur],
                                               pos);
    return hipGetLastError();
}

// One block per segment: its row of the step just taken (phase_in) from ring
// row `ring_row`, for segments that took part and have a thermo pointer.
__global__ void __launch_bounds__(kFoldThreads)
k_thermo_fold_segments(const double* __restrict__ part_b, int64_t blk_cap, Segs S, int ring_row)
{
    __shared__ double lds[kFoldThreads / 64][kPartialCols];
    __shared__ double lds_tot[kPartialCols];
    const int sid = blockIdx.x;
    const Seg& g = S.seg[sid];
    const int k = S.phase_in[sid];
    if (!g.thermo || k > g.nsteps) return;
    const double* rowp = part_b + (int64_t)ring_row * blk_cap * kPartialCols;
    fold_segment_row(rowp, S, g, lds, lds_tot, g.thermo + (int64_t)k * kThermoCols);
}

hipError_t launch_thermo_fold_segments(const Buffers& b, const Segs& S, int ring_row,
                                       hipStream_t s)
{
    if (S.nseg <= 0) return hipSuccess;
    if (!segs_ready(S, b)) return hipErrorInvalidValue;
    k_thermo_fold_segments<<<S.nseg, kFoldThreads, 0, s>>>(b.part_b, b.blk_cap, S,
                                                      ring_row % kThermoRing);
    return hipGetLastError();
}

// ---- Berendsen weak coupling ---------------------------------------------
//
// After the second half-kick of step s the thermo row gives the kinetic
// temperature T and the pressure P = (2 E_kin + tr W) / (3 V) (the virial
// theorem with the per-atom virials W_i of Section 2.3).  Velocities are then
// scaled by lambda = sqrt(1 + dt/tau_T (T0/T - 1)) and positions and box
// edges by mu = (1 - beta dt/tau_P (P0 - P))^(1/3) before the first
// half-kick of step s + 1.  The fold forms both factors in one thread and
// scales the segment's box in device memory, so the step loop never waits
// for the host.  The arithmetic is kept unfused, as a plain IEEE evaluation
// of these expressions in this order.
__global__ void __launch_bounds__(kFoldThreads)
k_npt_fold(const double* __restrict__ rowp, Segs S, Seg* __restrict__ seg_rw, NptArgs a,
           int step, int last, double* __restrict__ coupling, double* __restrict__ thermo,
           double* __restrict__ box_traj, unsigned* __restrict__ status)
{
#pragma clang fp contract(off)
    __shared__ double lds[kFoldThreads / 64][kPartialCols];
    __shared__ double lds_tot[kPartialCols];
    double* row = thermo + (int64_t)step * kThermoCols;
    fold_segment_row(rowp, S, S.seg[0], lds, lds_tot, row);
    if (threadIdx.x != 0) return;
    const Box box = S.seg[0].box;
    if (box_traj)
        for (int c = 0; c < 3; ++c) box_traj[(int64_t)step * 3 + c] = box.L[c];
    if (last) return;
    const double T = row[15];
    double lambda = 1.0, mu = 1.0;
    if (a.tau_T > 0.0 && T > 0.0) lambda = sqrt(1.0 + a.dt / a.tau_T * (a.T0 / T - 1.0));
    if (a.tau_P > 0.0) {
        const double volume = box.L[0] * box.L[1] * box.L[2];
        const double P = (2.0 * row[1] + row[2] + row[6] + row[10]) / (3.0 * volume);
        const double mu3 = 1.0 - a.beta * a.dt / a.tau_P * (a.P0 - P);
        if (mu3 > 0.0) {
            mu = cbrt(mu3);
        } else {
            atomicOr(status, ST_BAROSTAT);
        }
    }
    coupling[0] = lambda;
    coupling[1] = mu;
    Box nb;
    for (int c = 0; c < 3; ++c) {
        nb.L[c] = box.L[c] * mu;
        nb.inv[c] = 1.0 / nb.L[c];
    }
    seg_rw[0].box = nb;
}

hipError_t launch_npt_fold(const Buffers& b, const Segs& S, int ring_row, int step, bool last,
                           const NptArgs& a, double* thermo, double* box_traj, hipStream_t s)
{
    if (!segs_ready(S, b) || S.nseg != 1 || !thermo || !b.coupling) return hipErrorInvalidValue;
    const double* rowp = b.part_b + (int64_t)(ring_row % kThermoRing) * b.blk_cap * kPartialCols;
    k_npt_fold<<<1, kFoldThreads, 0, s>>>(rowp, S, b.seg, a, step, last ? 1 : 0, b.coupling, thermo,
                                    box_traj, b.status);
    return hipGetLastError();
}

// Scaling by the factors of the previous step, then that step's first
// half-kick and drift, with the forces it left in F; the positions are
// wrapped into the scaled box.  No neighbour is read, so the update is in
// place.
__global__ void __launch_bounds__(kBlock)
k_npt_drift(Segs S, int64_t os, const double* __restrict__ coupling, double4* __restrict__ xw,
            double* __restrict__ vel, const double* __restrict__ F)
{
#pragma clang fp contract(off)
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    const int sid = seg_of_block(S, lb, false);
    const Seg& g = S.seg[sid];
    const int local = (lb - g.blk) * kBlock + threadIdx.x;
    if (local >= g.n) return;
    const int64_t i = g.atom_off + local;
    const double lambda = coupling[2 * sid], mu = coupling[2 * sid + 1];
    const double4 xi = xw[i];
    double hdt, kin;
    atom_mass_factors(g, xi.w, hdt, kin);
    double x[3] = {xi.x, xi.y, xi.z};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double v = vel[c * os + i] * lambda;
        v = v + hdt * F[c * os + i];
        vel[c * os + i] = v;
        x[c] = x[c] * mu;
        x[c] = wrap_coord(x[c] + g.dt * v, g.box.L[c]);
    }
    xw[i] = make_double4(x[0], x[1], x[2], xi.w);
}

hipError_t launch_npt_drift(const Buffers& b, const Segs& S, int cur, hipStream_t s)
{
    if (S.nblk <= 0) return hipSuccess;
    if (!segs_ready(S, b) || !b.vel || !b.F || !b.coupling) return hipErrorInvalidValue;
    k_npt_drift<<<S.nblk, kBlock, 0, s>>>(S, b.ostride, b.coupling, b.xw[cur], b.vel, b.F);
    return hipGetLastError();
}

// Continuation of a run: the first half-kick and drift that the pairwise
// pass of the previous run's last step left out, from its full-step
// velocities and forces, v <- v + (dt/2) kappa F / m and x_next <- wrap(x +
// dt v), with the pairwise pass's unfused arithmetic in the same order, so a
// continued run takes the same steps, bit for bit, as one that never
// stopped.  Returns the squared displacement of x_next from the list-build
// position when `track` (formed as in the pairwise pass), else 0.
__device__ __forceinline__ double kick_drift_atom(const Seg& g, int64_t os, int64_t i,
                                                  const double4& xi,
                                                  double4* __restrict__ xw_next,
                                                  const double4* __restrict__ xbuild,
                                                  double* __restrict__ vel,
                                                  const double* __restrict__ F, bool track)
{
#pragma clang fp contract(off)
    const Box& box = g.box;
    double hdt, kin;
    atom_mass_factors(g, xi.w, hdt, kin);
    double vn[3], x[3] = {xi.x, xi.y, xi.z};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        vn[c] = vel[c * os + i] + hdt * F[c * os + i];
        x[c] = wrap_coord(x[c] + g.dt * vn[c], box.L[c]);
    }
    vel[i] = vn[0];
    vel[os + i] = vn[1];
    vel[2 * os + i] = vn[2];
    xw_next[i] = make_double4(x[0], x[1], x[2], xi.w);
    double disp2 = 0.0;
    if (track) {
        const double4 xb = xbuild[i];
        double d[3] = {x[0] - xb.x, x[1] - xb.y, x[2] - xb.z};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            d[c] -= box.L[c] * rint(d[c] * box.inv[c]);
            disp2 += d[c] * d[c];
        }
    }
    return disp2;
}

// Largest value of v over the block into *slot (one atomic per block;
// non-negative doubles order like their bit patterns).  Every thread calls it.
__device__ __forceinline__ void block_max_to_slot(double v, double* lds_max,
                                                  unsigned long long* __restrict__ slot)
{
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0) lds_max[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double bm = lds_max[0];
#pragma unroll
        for (int k = 1; k < kBlock / 64; ++k) bm = fmax(bm, lds_max[k]);
        atomicMax(slot, (unsigned long long)__double_as_longlong(bm));
    }
}

// Prologue of a continued one-structure run in one launch: block 0, when
// `thermo` is set, folds the previous run's last step (ring row `ring_row`)
// into thermo row 0 (first, so that its serial loop overlaps the rest); the
// nblk atom blocks after it stage the caller's positions (as the staging
// kernel does) and apply the half-kick and drift into x_next
// (kick_drift_atom); the first atom block sets the phase word to `phase`.
__global__ void __launch_bounds__(kBlock)
k_resume_prologue(Segs S, int64_t os, const double* __restrict__ pos,
                  const int32_t* __restrict__ types, int ntypes, double4* __restrict__ xw_next,
                  const double4* __restrict__ xbuild, double* __restrict__ vel,
                  const double* __restrict__ F, unsigned* __restrict__ status,
                  unsigned long long* __restrict__ slot, const double* __restrict__ part_b,
                  int64_t blk_cap, int ring_row, double* __restrict__ thermo,
                  int* __restrict__ phase_word, int phase)
{
    __shared__ double lds[kFoldThreads / 64][kPartialCols];
    __shared__ double lds_tot[kPartialCols];
    const Seg& g = S.seg[0];
    const int nfold = (int)gridDim.x - S.nblk;   // 0 or 1, dispatched first
    if ((int)blockIdx.x < nfold) {
        const double* rowp = part_b + (int64_t)ring_row * blk_cap * kPartialCols;
        fold_segment_row(rowp, S, g, lds, lds_tot, thermo);
        return;
    }
    const int lb = xcd_block((int)blockIdx.x - nfold, S.nblk);
    if (lb == 0 && threadIdx.x == 0) *phase_word = phase;
    const int64_t i = (int64_t)lb * kBlock + threadIdx.x;
    double disp2 = 0.0;
    if (i < g.n) {
        const double4 xi = staged_position(pos, types, ntypes, g.n, i, g.box, status);
        disp2 = kick_drift_atom(g, os, i, xi, xw_next, xbuild, vel, F, slot);
    }
    if (slot) block_max_to_slot(disp2, lds[0], slot);
}

hipError_t launch_resume_prologue(const Buffers& b, const Segs& S, const double* pos,
                                  const int32_t* types, int ntypes, int cur,
                                  unsigned long long* slot, int ring_row, double* thermo,
                                  int* phase_word, int phase, hipStream_t s)
{
    if (S.nblk <= 0) return hipSuccess;
    if (!segs_ready(S, b) || S.nseg != 1 || !pos || !b.vel || !b.F || !phase_word ||
        ring_row < 0 || ring_row >= kThermoRing)
        return hipErrorInvalidValue;
    k_resume_prologue<<<S.nblk + (thermo ? 1 : 0), kBlock, 0, s>>>(
        S, b.ostride, pos, types, ntypes, b.xw[cur ^ 1], b.xbuild, b.vel, b.F, b.status, slot,
        b.part_b, b.blk_cap, ring_row, thermo, phase_word, phase);
    return hipGetLastError();
}

template <class T>
hipError_t launch_pair_gather(const Buffers& b, const Segs& S, const StepArgs& a, hipStream_t s)
{
    if (S.nblk <= 0) return hipSuccess;
    if (!segs_ready(S, b) || !b.F || !b.W || !b.J || !b.U) return hipErrorInvalidValue;
    if (S.nblk <= kQuadPairBlocks)
        k_pair_quad<T><<<S.nblk_quad, kBlock, 0, s>>>(
            S, b.cap, b.ostride, a, b.xw[a.cur], b.xw[a.cur ^ 1], b.xbuild, b.nl, b.rev,
            b.mask, static_cast<const T*>(b.dpart), b.U, b.vel, b.F, b.W, b.J, b.ovf_count);
    else
        k_pair_gather<T><<<S.nblk, kBlock, 0, s>>>(
            S, b.cap, b.ostride, a, b.xw[a.cur], b.xw[a.cur ^ 1], b.xbuild, b.nl, b.rev,
            b.mask, static_cast<const T*>(b.dpart), b.U, b.vel, b.F, b.W, b.J, b.ovf_count);
    return hipGetLastError();
}

template hipError_t launch_pair_gather<double>(const Buffers&, const Segs&, const StepArgs&,
                                               hipStream_t);
template hipError_t launch_pair_gather<float>(const Buffers&, const Segs&, const StepArgs&,
                                              hipStream_t);

}  // namespace mbmd
