// Position staging and the cell-list neighbour build.
//
// The neighbour list of atom i holds every j != i whose minimum-image squared
// distance is below r_list^2 = (cutoff + skin)^2 (the Verlet list over a cell
// list that the paper uses because f_C vanishes beyond the cutoff; Section
// 2.1).  Entries are ordered by a key of their own (inside the potential
// cutoff at build time first, then by ascending index), so the list - and
// every sum that runs over it - does not depend on the order in which atoms
// were binned, which is the only place integer atomics appear.
//
// The inclusion test d = x_j - x_i, d <- d - L rint(d / L),
// r^2 = (dx*dx + dy*dy) + dz*dz < r_list^2 is evaluated in FP64 with no
// contraction to fused multiply-add, so the list is reproducible bit for bit
// by any IEEE evaluation of the same expression.
#include "mbmd_internal.h"

#include <type_traits>

namespace mbmd {

__device__ __forceinline__ double list_r2(const double4& a, const double4& b, const Box& box)
{
#pragma clang fp contract(off)
    double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
    dx = dx - box.L[0] * rint(dx / box.L[0]);
    dy = dy - box.L[1] * rint(dy / box.L[1]);
    dz = dz - box.L[2] * rint(dz / box.L[2]);
    return dx * dx + dy * dy + dz * dz;
}

__global__ void k_fill_int(int* __restrict__ p, int64_t count, int value)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = value;
}

hipError_t launch_fill_int(int* p, int64_t count, int value, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int64_t nb = (count + kBlock - 1) / kBlock;
    int grid = (int)(nb < 65536 ? nb : 65536);
    k_fill_int<<<grid, kBlock, 0, s>>>(p, count, value);
    return hipGetLastError();
}

__global__ void k_begin_single(Seg g, Seg* __restrict__ dst, unsigned* __restrict__ status,
                               int* __restrict__ ovf_count, int* __restrict__ phase0,
                               int* __restrict__ clear, int nclear)
{
    if (threadIdx.x == 0) {
        *dst = g;
        *status = 0u;
        *ovf_count = 0;
        *phase0 = 0;
    }
    for (int k = threadIdx.x; k < nclear; k += blockDim.x) clear[k] = 0;
}

hipError_t launch_begin_single(const Seg& g, Seg* dst, unsigned* status, int* ovf_count,
                               int* phase0, int* clear, int nclear, hipStream_t s)
{
    if (!dst || !status || !ovf_count || !phase0 || (nclear > 0 && !clear))
        return hipErrorInvalidValue;
    k_begin_single<<<1, 64, 0, s>>>(g, dst, status, ovf_count, phase0, clear, nclear);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock)
k_load_positions(const double* __restrict__ pos, const int32_t* __restrict__ types, int ntypes,
                 int64_t n, Box box, int atom_off, double4* __restrict__ xw,
                 unsigned* __restrict__ status)
{
    const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    xw[atom_off + i] = staged_position(pos, types, ntypes, n, i, box, status);
}

hipError_t launch_load_positions(const double* pos_soa, const int32_t* types, int ntypes,
                                 int64_t n, Box box, int atom_off, double4* xw,
                                 unsigned* status, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_load_positions<<<blocks_for(n), kBlock, 0, s>>>(pos_soa, types, ntypes, n, box, atom_off,
                                                      xw, status);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kBlock)
k_store_positions(const double4* __restrict__ xw, int atom_off, int64_t n,
                  double* __restrict__ pos)
{
    const int64_t i = (int64_t)xcd_block(blockIdx.x, gridDim.x) * kBlock + threadIdx.x;
    if (i >= n) return;
    const double4 p = xw[atom_off + i];
    pos[i] = p.x;
    pos[n + i] = p.y;
    pos[2 * n + i] = p.z;
}

hipError_t launch_store_positions(const double4* xw, int atom_off, int64_t n, double* pos_soa,
                                  hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_store_positions<<<blocks_for(n), kBlock, 0, s>>>(xw, atom_off, n, pos_soa);
    return hipGetLastError();
}

// ---- cell binning ---------------------------------------------------------

__device__ __forceinline__ int cell_coord(double x, double inv_lc, int nc)
{
    int c = (int)(x * inv_lc);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// Logical 256-atom block -> (segment, global atom index); false past the
// segment's last atom.
__device__ __forceinline__ bool block_atom(const Segs& S, int& sid, int64_t& i)
{
    const int lb = xcd_block(blockIdx.x, gridDim.x);
    sid = seg_of_block(S, lb, false);
    const Seg& g = S.seg[sid];
    const int local = (lb - g.blk) * kBlock + threadIdx.x;
    i = g.atom_off + local;
    return local < g.n;
}

// Cell (index into the cell arrays) of a wrapped position of segment g; the
// binning, the fill and the search each evaluate it from the same position
// and so agree on every atom's cell.
__device__ __forceinline__ int cell_index(const Seg& g, const double4& p)
{
    const int cx = cell_coord(p.x, g.inv_lc[0], g.nc[0]);
    const int cy = cell_coord(p.y, g.inv_lc[1], g.nc[1]);
    const int cz = cell_coord(p.z, g.inv_lc[2], g.nc[2]);
    return g.cell_off + (cz * g.nc[1] + cy) * g.nc[0] + cx;
}

__global__ void __launch_bounds__(kBlock)
k_cell_count(Segs S, const double4* __restrict__ xw, int* __restrict__ count,
             double4* __restrict__ xbuild)
{
    int sid;
    int64_t i;
    if (!block_atom(S, sid, i)) return;
    const Seg& g = S.seg[sid];
    const double4 p = xw[i];
    atomicAdd(&count[cell_index(g, p)], 1);
    if (g.build) xbuild[i] = p;
}

// Two-pass exclusive scan of the cell counts: per-tile sums, then the
// per-tile scan, each tile adding the sums of the tiles before it.
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ int block_exclusive_scan(int v, int* lds_waves, int& total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) lds_waves[wave] = inc;
    __syncthreads();
    int wave_off = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        const int t = lds_waves[w];
        if (w < wave) wave_off += t;
        total += t;
    }
    __syncthreads();
    return wave_off + inc - v;
}

__global__ void __launch_bounds__(kBlock)
k_scan_block_sums(const int* __restrict__ count, int ncell, int* __restrict__ bsum)
{
    __shared__ int lds[kBlock / 64];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < ncell) s += count[base + k];
    int total;
    block_exclusive_scan(s, lds, total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kBlock)
k_scan_write(const int* __restrict__ count, int ncell, const int* __restrict__ bsum,
             int* __restrict__ start, int* __restrict__ fill)
{
    __shared__ int lds[kBlock / 64];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int v[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < ncell ? count[base + k] : 0;
        s += v[k];
    }
    // the tile's offset: the totals of the tiles before it
    int before = 0;
    for (int t = threadIdx.x; t < (int)blockIdx.x; t += kBlock) before += bsum[t];
    int total;
    block_exclusive_scan(before, lds, total);
    int run = total + block_exclusive_scan(s, lds, total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < ncell) {
            start[base + k] = run;
            fill[base + k] = 0;
        }
        run += v[k];
    }
    if (base + kScanItems >= ncell && base < ncell) start[ncell] = run;
    if (ncell == 0 && blockIdx.x == 0 && threadIdx.x == 0) start[0] = 0;
}

// The whole scan in one block, tile after tile with a running carry (grids
// of at most kScanOneBlockTiles tiles: one launch instead of two).
constexpr int kScanOneBlockTiles = 16;

__global__ void __launch_bounds__(kBlock)
k_scan_one_block(const int* __restrict__ count, int ncell, int* __restrict__ start,
                 int* __restrict__ fill)
{
    __shared__ int lds[kBlock / 64];
    int carry = 0;
    for (int tile = 0; tile * kScanTile < ncell; ++tile) {
        const int base = tile * kScanTile + threadIdx.x * kScanItems;
        int v[kScanItems];
        int s = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            v[k] = base + k < ncell ? count[base + k] : 0;
            s += v[k];
        }
        int total;
        int run = carry + block_exclusive_scan(s, lds, total);
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) {
            if (base + k < ncell) {
                start[base + k] = run;
                fill[base + k] = 0;
            }
            run += v[k];
        }
        if (base + kScanItems >= ncell && base < ncell) start[ncell] = run;
        carry += total;
    }
    if (ncell == 0 && threadIdx.x == 0) start[0] = 0;
}

// Zeroes a[0 .. na) and b[0 .. nb) in one launch.
__global__ void k_fill_zero2(int* __restrict__ a, int64_t na, int* __restrict__ b, int64_t nb)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb; i += stride) {
        if (i < na) a[i] = 0;
        else b[i - na] = 0;
    }
}

// Atom i's position in cell order, its index and type packed into the w
// lane as two 32-bit integers (low word i, high word the type): the search
// reads a candidate's position, index and type in one 32-byte access.  The
// w lane is never used in arithmetic.
__global__ void __launch_bounds__(kBlock)
k_cell_fill(Segs S, const double4* __restrict__ xw, const int* __restrict__ start,
            int* __restrict__ fill, double4* __restrict__ xcell)
{
    int sid;
    int64_t i;
    if (!block_atom(S, sid, i)) return;
    const double4 x = xw[i];
    const int c = cell_index(S.seg[sid], x);
    const int p = start[c] + atomicAdd(&fill[c], 1);
    xcell[p] = make_double4(x.x, x.y, x.z, __hiloint2double((int)x.w, (int)i));
}

// ---- neighbour search -----------------------------------------------------

constexpr int kSearchBlock = kBlock / 2;
// Launches of at most this many 256-atom blocks search and fill the reverse
// slots with four lanes per atom (shorter serial walks when the chip would
// otherwise hold few waves); larger ones search with one lane per atom and
// fill the reverse slots with two (measured best at 512,000 and 1,000,000
// atoms).  The lists do not depend on the choice.
constexpr int kQuadBuildBlocks = 512;
constexpr int kSearchLanesLarge = 1;    // lanes per atom above that size
constexpr int kSearchCands = 2;         // candidates loaded together
constexpr int kReverseLanesLarge = 2;

// Value of lane (lane xor K) of the same quad (DPP quad permutation).
template <int K>
__device__ __forceinline__ int search_quad_xor(int v)
{
    constexpr int ctrl = K == 1 ? 0xB1 : (K == 2 ? 0x4E : 0x1B);
    return __builtin_amdgcn_mov_dpp(v, ctrl, 0xF, 0xF, false);
}

// A cheap test (multiply by 1/L, fused arithmetic allowed) settles every
// candidate whose squared distance is not within a relative 1e-10 of r_list^2;
// only those near the boundary take the exact unfused test above, whose
// rounding error is many orders of magnitude below that margin.
__device__ __forceinline__ bool in_list(const double4& a, const double4& b, const Box& box,
                                        double rl2, double rl2_lo, double rl2_hi, double& r2)
{
    double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
    dx -= box.L[0] * rint(dx * box.inv[0]);
    dy -= box.L[1] * rint(dy * box.inv[1]);
    dz -= box.L[2] * rint(dz * box.inv[2]);
    r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < rl2_lo) return true;
    if (r2 > rl2_hi) return false;
    return list_r2(a, b, box) < rl2;
}

// LANES (1, 2 or 4) lanes per atom of a segment being built: lane q walks the
// stencil rows q, q + LANES, ... into a list of its own, kept in LDS
// (column-major over the block so that neighbouring threads hit distinct
// banks); each lane then writes its entries at their ranks in the union of
// the lanes' lists, slot-major, each rank the count of smaller keys over
// every list of the atom.  The union's order does not depend
// on how the offsets were split, so the list is the one a single walk
// gives.  A search block covers kSearchBlock / LANES atoms; 256 LANES /
// kSearchBlock of them make one 256-atom block of the other per-atom kernels.
// The list is ordered by the key (r^2 >= rc2, j): the neighbours inside the
// potential cutoff at build time first, each group by ascending index, so
// the pairwise pass can stop at the last in-cutoff slot.  The grouping only
// steers work (every step recomputes which slots are in the cutoff); the
// order is a deterministic function of the positions.
// TYPED: the radii of each pair come from R (copied to LDS), indexed by the
// types in the w lanes, and the stencil is pruned with the largest radius of
// atom i's type.
// CW candidates of a cell are loaded together, so that a lane waits once
// per CW candidates (a cell holds a few atoms).
template <bool TYPED, int LANES, int CW>
__global__ void __launch_bounds__(kSearchBlock)
k_search(Segs S, const double4* __restrict__ xcell, double rl2, double rl2_lo, double rl2_hi,
         double rc2, ListRadii R, int M,
         int64_t cap, const int* __restrict__ start,
         int* __restrict__ nn, int* __restrict__ nl, int* __restrict__ maxnn,
         unsigned* __restrict__ status, unsigned* __restrict__ sstat)
{
    extern __shared__ int lbuf[];
    __shared__ int lds_max[kSearchBlock / 64];
    __shared__ double t_rl2[TYPED ? kMaxTypes * kMaxTypes : 1];
    __shared__ double t_rc2[TYPED ? kMaxTypes * kMaxTypes : 1];
    if constexpr (TYPED) {
        if (threadIdx.x < kMaxTypes * kMaxTypes) {
            t_rl2[threadIdx.x] = R.rl2[threadIdx.x];
            t_rc2[threadIdx.x] = R.rc2[threadIdx.x];
        }
        __syncthreads();
    }
    static_assert(LANES == 1 || LANES == 2 || LANES == 4, "one, two or four lanes per atom");
    constexpr int kAtoms = kSearchBlock / LANES;       // atoms per search block
    constexpr int kPerBlock = kBlock / kAtoms;         // search blocks per 256-atom block
    const int q = threadIdx.x & (LANES - 1);
    const int lb2 = xcd_block(blockIdx.x, gridDim.x);
    const int lb = lb2 / kPerBlock;
    const int sid = seg_of_block(S, lb, false);
    const Seg& g = S.seg[sid];
    // Quad k of the segment takes the k-th atom in cell order, so the
    // quads of a wave sit in a run of neighbouring cells along x and, at
    // each stencil offset, read candidates from one stretch of xcell.
    const int local = (lb - g.blk) * kBlock + (lb2 % kPerBlock) * kAtoms +
                      (int)(threadIdx.x / LANES);
    const bool active = local < g.n && g.build;
    int cnt = 0;               // entries this lane found
    int64_t i = 0;
    int* buf = lbuf + threadIdx.x;
    if (active) {
        const int p0 = start[g.cell_off] + local;
        const Box box = g.box;
        const double4 xi = xcell[p0];
        i = __double2loint(xi.w);
        const int ti = TYPED ? min(max(__double2hiint(xi.w), 0), R.nt - 1) : 0;
        double rl2_i = rl2;   // largest list radius squared of i's pairs
        if constexpr (TYPED) {
            rl2_i = t_rl2[ti * kMaxTypes];
            for (int b = 1; b < R.nt; ++b) rl2_i = fmax(rl2_i, t_rl2[ti * kMaxTypes + b]);
        }
        const int c = cell_index(g, xi) - g.cell_off;   // xi: the binned position
        const int cx = c % g.nc[0], cy = (c / g.nc[0]) % g.nc[1], cz = c / (g.nc[0] * g.nc[1]);
        // The stencil cells to visit, as bits k = 9 (oz + 1) + 3 (oy + 1) +
        // (ox + 1).  A cell at offset (ox, oy, oz) whose nearest point is
        // farther from x_i than r_list (with a relative margin of 1e-5 on r^2,
        // far above the float rounding of these sums) holds no list entry and
        // is left out, so the lists are exactly those of the full stencil.
        // Boxes with fewer than three cells along an axis visit each distinct
        // cell once and prune nothing.
        unsigned visit = 0;
        {
            float gap2[3][3];
            const int ci[3] = {cx, cy, cz};
            const double xa[3] = {xi.x, xi.y, xi.z};
            int lo[3], hi[3];
            bool prune = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                lo[a] = g.nc[a] >= 3 ? -1 : 0;
                hi[a] = g.nc[a] >= 2 ? 1 : 0;
                prune = prune && g.nc[a] >= 3;
                double f = xa[a] * g.inv_lc[a] - (double)ci[a];
                f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
                const double side = g.box.L[a] / (double)g.nc[a];
                gap2[a][0] = (float)(f * f * side * side);
                gap2[a][1] = 0.0f;
                gap2[a][2] = (float)((1.0 - f) * (1.0 - f) * side * side);
            }
            const float skip2 = prune ? (float)(rl2_i * (1.0 + 1e-5)) : 3.0e38f;
            for (int oz = lo[2]; oz <= hi[2]; ++oz)
                for (int oy = lo[1]; oy <= hi[1]; ++oy)
                    for (int ox = lo[0]; ox <= hi[0]; ++ox)
                        if (gap2[2][oz + 1] + gap2[1][oy + 1] + gap2[0][ox + 1] <= skip2)
                            visit |= 1u << (9 * (oz + 1) + 3 * (oy + 1) + (ox + 1));
        }
        // Candidate at cell-order slot p (atom i itself sits at p0) against
        // the list radius of the pair; an entry is appended to the lane's LDS
        // list (capacity M), ranked by key once the walk is done.
        // Past M entries (an overflow, which fails the call) an entry
        // replaces the largest key if it is smaller, so the list keeps the
        // M smallest keys.
        auto consider = [&](int p, const double4& xj) {
            if (p == p0) return;
            const int j = __double2loint(xj.w);
            double r2;
            double pl2 = rl2, pl2_lo = rl2_lo, pl2_hi = rl2_hi, pc2 = rc2;
            if constexpr (TYPED) {
                const int t = ti * kMaxTypes + min(max(__double2hiint(xj.w), 0), R.nt - 1);
                pl2 = t_rl2[t];
                pl2_lo = pl2 * (1.0 - 1e-10);
                pl2_hi = pl2 * (1.0 + 1e-10);
                pc2 = t_rc2[t];
            }
            if (in_list(xi, xj, box, pl2, pl2_lo, pl2_hi, r2)) {
                const unsigned key = (unsigned)j | (r2 < pc2 ? 0u : 0x80000000u);
                if (cnt < M) {
                    buf[cnt * kSearchBlock] = (int)key;
                } else if (M > 0) {
                    int top = 0;
                    for (int t = 1; t < M; ++t)
                        if ((unsigned)buf[t * kSearchBlock] > (unsigned)buf[top * kSearchBlock])
                            top = t;
                    if ((unsigned)buf[top * kSearchBlock] > key) buf[top * kSearchBlock] = (int)key;
                }
                ++cnt;
            }
        };
        // Stencil row rr = 3 (oz + 1) + (oy + 1): its visited cells, at x
        // offsets -1 (if visited), 0 and +1 (if visited), are neighbours in
        // cell order and so one run [b, e) of xcell, except where the row
        // crosses the periodic boundary in x, whose far cell is a second run
        // [b2, e2).  A row whose middle cell is left out is empty (the middle
        // cell is the row's nearest, so its outer cells are left out too).
        auto row_range = [&](int rr, int& b, int& e, int& b2, int& e2) {
            b = e = b2 = e2 = 0;
            const unsigned bits = rr < 9 ? (visit >> (3 * rr)) & 7u : 0u;
            if (bits & 2u) {
                const int oz = rr / 3 - 1, oy = rr % 3 - 1;
                // periodic wrap by one cell (no integer division per offset)
                auto wrap = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
                const int nx = g.nc[0];
                const int row =
                    g.cell_off + (wrap(cz + oz, g.nc[2]) * g.nc[1] + wrap(cy + oy, g.nc[1])) * nx;
                int xa = cx - (int)(bits & 1u), xb = cx + (int)(bits >> 2);
                if (xa < 0) {
                    b2 = start[row + nx - 1];
                    e2 = start[row + nx];
                    xa = 0;
                }
                if (xb >= nx) {
                    b2 = start[row];
                    e2 = start[row + 1];
                    xb = nx - 1;
                }
                b = start[row + xa];
                e = start[row + xb + 1];
            }
        };
        // The candidates of a row's runs [b, e) and [b2, e2) in one loop (so
        // that a wave whose lanes at the box's x faces have a second run
        // does not loop twice), CW loaded before any is tested.
        auto scan = [&](int b, int e, int b2, int e2) {
            const int n1 = e - b, n = n1 + (e2 - b2);
            auto slot = [&](int t) { return t < n1 ? b + t : b2 + (t - n1); };
            for (int t = 0; t < n; t += CW) {
                // positions past the row's end re-read its last atom (in
                // bounds, no branch around the loads) and are not tested
                double4 xv[CW];
#pragma unroll
                for (int u = 0; u < CW; ++u) xv[u] = xcell[slot(min(t + u, n - 1))];
                // every loaded word counts as used here: the loads are issued
                // back to back (none sunk into the tests, none waiting on the
                // reuse of an unused word's register) and waited on once
#pragma unroll
                for (int u = 0; u < CW; ++u)
                    asm volatile("" ::"v"(xv[u].x), "v"(xv[u].y), "v"(xv[u].z), "v"(xv[u].w));
#pragma unroll
                for (int u = 0; u < CW; ++u)
                    if (t + u < n) consider(slot(t + u), xv[u]);
            }
        };
        // Lane q of every quad walks the rows q, q + LANES, ... in the same
        // order (a row left out is an empty iteration), which keeps the
        // wave's reads together; the next row's runs are fetched before the
        // current row is scanned.
        int b, e, b2, e2;
        row_range(q, b, e, b2, e2);
        for (int rr = q; rr < 9; rr += LANES) {
            int nb, ne, nb2, ne2;
            row_range(rr + LANES, nb, ne, nb2, ne2);
            scan(b, e, b2, e2);
            b = nb;
            e = ne;
            b2 = nb2;
            e2 = ne2;
        }
    }
    // counts of the quad's other lanes (every lane of the wave takes part)
    int c1 = 0, c2 = 0, c3 = 0;
    if constexpr (LANES >= 2) c1 = search_quad_xor<1>(cnt);
    if constexpr (LANES == 4) {
        c2 = search_quad_xor<2>(cnt);
        c3 = search_quad_xor<3>(cnt);
    }
    if constexpr (LANES > 1) __syncthreads();   // the atom's lists are complete in LDS
    const int total = cnt + c1 + c2 + c3;
    if (active) {
        // On overflow the stored entries are the M smallest keys (each lane
        // kept its M smallest); the status bit turns the call into an error.
        if (q == 0) {
            if (total > M) {
                atomicOr(status, ST_NEIGH_OVERFLOW);
                atomicOr(&sstat[S.seg[sid].sidx], ST_NEIGH_OVERFLOW);
            }
            nn[i] = total;
        }
        const int w = cnt < M ? cnt : M;
        const int wr[3] = {min(c1, M), min(c2, M), min(c3, M)};
        for (int p = 0; p < w; ++p) {
            const unsigned key = (unsigned)buf[p * kSearchBlock];
            // rank in the union (keys are distinct): the count of smaller
            // keys over every lane's list of the atom, own included, read
            // without early exits so that the reads do not wait on one
            // another (no list is sorted)
            int rank = 0;
#pragma unroll 4
            for (int t = 0; t < w; ++t) rank += (unsigned)buf[t * kSearchBlock] < key;
#pragma unroll
            for (int r = 1; r < LANES; ++r) {
                const int* col = lbuf + (threadIdx.x ^ r);
#pragma unroll 4
                for (int t = 0; t < wr[r - 1]; ++t) rank += (unsigned)col[t * kSearchBlock] < key;
            }
            // (k_reverse, which always follows, writes every reverse slot)
            if (rank < M) nl[(int64_t)rank * cap + i] = (int)(key & 0x7fffffffu);
        }
    }
    // largest count of the block, one atomic per block
    int mx = active ? total : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) lds_max[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        int bm = lds_max[0];
#pragma unroll
        for (int k = 1; k < kSearchBlock / 64; ++k) bm = max(bm, lds_max[k]);
        atomicMax(&maxnn[sid], bm);
    }
}

// LANES (1, 2 or 4) lanes per atom: lane q takes the list slots q, q + LANES,
// ... of its atom (kBlock / LANES atoms per block, LANES blocks per 256-atom
// block).
template <int LANES>
__global__ void __launch_bounds__(kBlock)
k_reverse(Segs S, const int* __restrict__ nn, const int* __restrict__ nl, int M, int64_t cap,
          uint8_t* __restrict__ rev, unsigned* __restrict__ status)
{
    const int lbl = xcd_block(blockIdx.x, gridDim.x);
    const int lb = lbl / LANES;
    const int sid = seg_of_block(S, lb, false);
    const Seg& g = S.seg[sid];
    const int local =
        (lb - g.blk) * kBlock + (lbl % LANES) * (kBlock / LANES) + (int)(threadIdx.x / LANES);
    if (local >= g.n || !g.build) return;
    const int64_t i = g.atom_off + local;
    const int cnt = min(nn[i], M);
    for (int m = (int)(threadIdx.x % LANES); m < cnt; m += LANES) {
        const int j = nl[(int64_t)m * cap + i];
        // Complete lists are symmetric (the inclusion test gives the same
        // bits for (i, j) and (j, i)), so such a pair is settled once, by
        // its smaller index, which writes both reverse slots.  When either
        // list overflowed (the call then fails) each thread writes its own
        // entry.  Either way every entry below the count is written exactly
        // once, so the pairwise pass never reads a stale slot.
        const bool both_complete = nn[i] <= M && nn[j] <= M;
        if (both_complete && j < (int)i) continue;
        const int cj = min(nn[j], M);
        int s = -1;
        // find i in j's list, eight independent loads at a time
        for (int q0 = 0; q0 < cj && s < 0; q0 += 8) {
            int v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = q0 + u < cj ? nl[(int64_t)(q0 + u) * cap + j] : -1;
#pragma unroll
            for (int u = 7; u >= 0; --u)
                if (v[u] == (int)i) s = q0 + u;
        }
        if (s < 0) {
            atomicOr(status, ST_ASYMMETRIC);
            rev[(int64_t)m * cap + i] = 0;
            continue;
        }
        rev[(int64_t)m * cap + i] = (uint8_t)s;
        if (both_complete) rev[(int64_t)s * cap + j] = (uint8_t)m;
    }
}

hipError_t launch_build_neighbors(const Buffers& b, const Segs& S, int total_cells, int cur,
                                  double rlist, double rcut, const ListRadii* typed,
                                  hipStream_t s)
{
    if (S.nblk <= 0) return hipSuccess;
    if (!S.seg || S.nseg > b.seg_cap || total_cells > b.cell_cap) return hipErrorInvalidValue;
    {
        const int64_t nz = (int64_t)total_cells + S.nseg;
        int64_t nb = (nz + kBlock - 1) / kBlock;
        if (nb > 65536) nb = 65536;
        k_fill_zero2<<<(int)nb, kBlock, 0, s>>>(b.cell_count, total_cells, b.maxnn, S.nseg);
    }
    k_cell_count<<<S.nblk, kBlock, 0, s>>>(S, b.xw[cur], b.cell_count, b.xbuild);
    const int nscan = (total_cells + kScanTile - 1) / kScanTile;
    if (nscan <= kScanOneBlockTiles) {
        k_scan_one_block<<<1, kBlock, 0, s>>>(b.cell_count, total_cells, b.cell_start,
                                              b.cell_fill);
    } else {
        // The block sums live in the fill array's tail: cell_fill has room
        // for cell capacity + 1 + scan blocks ints.
        int* bsum = b.cell_fill + total_cells + 1;
        k_scan_block_sums<<<nscan, kBlock, 0, s>>>(b.cell_count, total_cells, bsum);
        k_scan_write<<<nscan, kBlock, 0, s>>>(b.cell_count, total_cells, bsum, b.cell_start,
                                              b.cell_fill);
    }
    k_cell_fill<<<S.nblk, kBlock, 0, s>>>(S, b.xw[cur], b.cell_start, b.cell_fill,
                                          b.xcell);
    const size_t lds = sizeof(int) * (size_t)kSearchBlock * b.M;
    const double rl2 = rlist * rlist;
    if (typed && (typed->nt < 1 || typed->nt > kMaxTypes)) return hipErrorInvalidValue;
    const bool small = S.nblk <= kQuadBuildBlocks;
    const int sl = small ? 4 : kSearchLanesLarge, rl = small ? 4 : kReverseLanesLarge;
    const int nsb = sl * (kBlock / kSearchBlock) * S.nblk;   // search blocks
    const double lo = rl2 * (1.0 - 1e-10), hi = rl2 * (1.0 + 1e-10);
    const ListRadii R = typed ? *typed : ListRadii{};
    auto search = [&](auto typed_tag, auto lanes_tag) {
        constexpr bool TY = decltype(typed_tag)::value;
        constexpr int LN = decltype(lanes_tag)::value;
        k_search<TY, LN, kSearchCands><<<nsb, kSearchBlock, lds, s>>>(
            S, b.xcell, rl2, lo, hi, rcut * rcut, R, b.M, b.cap, b.cell_start,
            b.nn, b.nl, b.maxnn, b.status, b.sstat);
    };
    using T1 = std::integral_constant<int, 1>;
    using T2 = std::integral_constant<int, 2>;
    using T4 = std::integral_constant<int, 4>;
    const bool ty = typed && typed->nt > 1;
    if (ty) {
        if (sl == 4) search(std::true_type{}, T4{});
        else if (sl == 2) search(std::true_type{}, T2{});
        else search(std::true_type{}, T1{});
    } else {
        if (sl == 4) search(std::false_type{}, T4{});
        else if (sl == 2) search(std::false_type{}, T2{});
        else search(std::false_type{}, T1{});
    }
    if (rl == 4)
        k_reverse<4><<<4 * S.nblk, kBlock, 0, s>>>(S, b.nn, b.nl, b.M, b.cap, b.rev, b.status);
    else if (rl == 2)
        k_reverse<2><<<2 * S.nblk, kBlock, 0, s>>>(S, b.nn, b.nl, b.M, b.cap, b.rev, b.status);
    else
        k_reverse<1><<<S.nblk, kBlock, 0, s>>>(S, b.nn, b.nl, b.M, b.cap, b.rev, b.status);
    return hipGetLastError();
}

}  // namespace mbmd
