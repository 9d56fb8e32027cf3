// Internal declarations shared by the HIP translation units of libmbmd.
//
// Every kernel works on a set of segments: independent periodic structures
// (one for a plain call, many for the serving batch) whose atoms occupy
// contiguous ranges of the same device arrays.  A block never straddles two
// segments: a segment owns a contiguous range of blocks, found from the block
// index by binary search over the segment table, so everything a block
// reduces belongs to one structure and is summed in the same order whatever
// else shares the launch.
//
// Data layout in device memory (N atom capacity, M list slots per atom):
//   xw[2][N]         double4 {x, y, z, type}: wrapped positions, atom-major
//                    so a neighbour gather is one 32-byte access; two buffers
//                    because the drift writes while neighbours are still read
//   xbuild[N]        double4 positions at the last list build
//   xcell[N]         double4 {x, y, z, (index, type)} in cell order at the
//                    last build (the w lane holds the atom's index and type
//                    as two 32-bit integers), so the search's lanes, which
//                    also take atoms in cell order, read neighbouring cells'
//                    atoms from neighbouring addresses, one access each
//   nn[N]            int32 list count (true count, may exceed M on overflow)
//   nl[M][N]         int32 neighbour index, slot-major (lane i reads nl[m*N+i]
//                    coalesced); neighbours inside the potential cutoff at
//                    build time first, each group by ascending index
//   rev[M][N]        uint8 slot of i inside the list of nl[m][i] (M <= 64)
//   mask[N]          uint64 bit m set iff slot m lies inside the potential cutoff
//   dpart[M][N][3]   T: dU_i/dr_ij for list slot m (written for in-cutoff slots only)
//   U[N], F[3][N], W[9][N] (component 3a+b), J[3][N], v[3][N]: FP64 SoA
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbmd {

// Device status bits (OR-ed by any thread; results never use atomics).
enum : unsigned {
    ST_NEIGH_OVERFLOW = 1u << 0,   // a neighbour list needed more than M slots
    ST_NONFINITE = 1u << 2,        // non-finite position
    ST_ASYMMETRIC = 1u << 3,       // list or cutoff mask not symmetric (internal)
    ST_TYPES = 1u << 4,            // an atom type other than 0
    ST_BAROSTAT = 1u << 5,         // Berendsen box factor mu^3 <= 0 (mu set to 1)
    ST_SKIN = 1u << 6,             // serving batch: an atom moved more than skin/2 from
                                   // its position at the last list build before the
                                   // next scheduled build (per-structure word only)
};

constexpr int kBlock = 256;          // threads per block of every per-atom kernel
constexpr int kQuadAtoms = 64;       // atoms per block of the four-lanes-per-atom kernels
constexpr int kMaxSlots = 64;        // list capacity limit (cutoff mask is 64-bit)
constexpr int kQuad = 4;             // lanes per atom in the site passes
constexpr int kTersoffSlots = 2;     // bonds per lane: Tersoff site pass (8 bonds per atom)
constexpr int kTersoffMultiSlots = 3;    // several types (12 bonds: the Si-Si second
                                         // neighbours of SiC sit at the Si-Si cutoff)
constexpr int kSWSlots = 3;          // bonds per lane: SW site pass (12 bonds per atom)
constexpr int kThermoCols = 16;      // per-step thermo row
constexpr int kPartialCols = 14;     // per-block partials: U, E_kin, W(9), J(3)
constexpr int kMaxChunk = 256;       // steps enqueued between two checks of the skin
constexpr int kThermoRing = 256;     // per-step rows of block partials kept before a fold
// Launches of at most this many 256-atom blocks take the pairwise pass with
// four lanes per atom, which leaves four thermo rows per block.
constexpr int kQuadPairBlocks = 64;
constexpr int kMaxTypes = 4;         // atom types of the multicomponent Tersoff form

struct Box {
    double L[3];
    double inv[3];
};

// One structure of a launch.
struct Seg {
    Box box;
    int nc[3];              // cell grid
    double inv_lc[3];
    int cell_off, ncell;    // cells [cell_off, cell_off + ncell) of the cell arrays
    int atom_off, n;        // atoms [atom_off, atom_off + n)
    int blk, blk_quad;      // first block for 256-atom and 64-atom blocks
    int nsteps;             // steps of its run (0: a single force evaluation)
    int build;              // nonzero: its list is (re)built by the next build launch
    int sidx;               // index of its per-structure status word (batch; 0 alone)
    double half_dt_acc;     // dt/2 kappa/m
    double dt;
    double kin_scale;       // m / (2 kappa)
    int typed_mass;         // nonzero: per-type masses below replace the two above
    double hdt_t[kMaxTypes];    // dt/2 kappa/m_t
    double kin_t[kMaxTypes];    // m_t / (2 kappa)
    double* thermo;         // batch: [nsteps + 1][16] thermo rows of this structure, or null
};

// Integrator factors of atom i of segment g (type from the position's w).
__device__ __forceinline__ void atom_mass_factors(const Seg& g, double w, double& hdt, double& kin)
{
    hdt = g.half_dt_acc;
    kin = g.kin_scale;
    if (g.typed_mass) {
        const int t = (int)w;
        hdt = g.hdt_t[t];
        kin = g.kin_t[t];
    }
}

// Device view of the segment table.
struct Segs {
    const Seg* seg;
    int nseg;
    int nblk, nblk_quad;    // total blocks of each kind
    const int* phase_in;    // per segment: index of the step being computed
    int* phase_out;         // receives phase_in + 1 (written by the pairwise pass)
};

// Segment owning logical block b (field blk or blk_quad), by binary search.
__device__ __forceinline__ int seg_of_block(const Segs& S, int b, bool quad)
{
    int lo = 0, hi = S.nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int start = quad ? S.seg[mid].blk_quad : S.seg[mid].blk;
        if (start <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Segment holding global atom i, by binary search over the atom offsets.
__device__ __forceinline__ int seg_of_atom(const Segs& S, int64_t i)
{
    int lo = 0, hi = S.nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (S.seg[mid].atom_off <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

struct TersoffParams {                // the 1989 single-element form
    double A, B, lam, mu, beta, n, c, d, h, R, S;
};
// Tersoff's multicomponent form: per-element parameters and the bond-order
// factor chi of each type pair (nt = 1, chi = 1: the single-element form).
struct TersoffTable {
    int nt;
    TersoffParams elem[kMaxTypes];
    double chi[kMaxTypes * kMaxTypes];
};
struct SWParams {                     // the 1985 form
    double epsilon, sigma, a, lam, gamma, A, B, p, q;
};

// Workspace view passed to the launchers.
struct Buffers {
    int64_t cap;             // atom capacity (array length N)
    int M;
    double4* xw[2];
    double4* xbuild;
    int* nn;
    int* nl;
    uint8_t* rev;
    unsigned long long* mask;
    void* dpart;
    int* cell_count;
    int* cell_start;
    int* cell_fill;
    double4* xcell;          // [N] positions, index and type in cell order
    int64_t cell_cap;
    double* part_b;          // [kThermoRing][block capacity][kPartialCols]
    int64_t blk_cap;         // 256-atom block capacity, plus the rows the four-lane
                             // pairwise pass needs (rows of part_b per step)
    int* ovf_count;          // atoms whose in-cutoff count exceeds the fast path
    int* ovf_list;           // [N]
    unsigned* status;
    unsigned* sstat;         // [segments] per-structure status (indexed by Seg::sidx)
    double4* xsnap;          // [N] positions at the start of a checked chunk
    double* vsnap;           // [3][N] velocities at the start of a checked chunk
    unsigned long long* step_disp2;  // [kMaxChunk] largest squared displacement per step
    int* maxnn;              // [segments] largest list count of the last build
    int* phase[2];           // per segment step index (double-buffered)
    double* coupling;        // [segments][2] Berendsen lambda, mu for the next drift
    Seg* seg;                // segment table
    int seg_cap;
    double* vel;             // velocities [3][ostride]
    double *U, *F, *W, *J;   // per-atom outputs: U[ostride], F[3][..], W[9][..], J[3][..]
    int64_t ostride;         // row stride of vel, F, W, J (cap for the batch state)
};

// Mapping of a hardware block index to a logical block so that each XCD
// (hardware blocks b with b % 8 == x) works on one contiguous range of atoms,
// which keeps shared neighbour data in one XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int x = b & 7, idx = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x < r ? x * (q + 1) + idx : r * (q + 1) + (x - r) * q + idx;
}

// Host-side check of a launch's segment view: every pointer a kernel
// dereferences unconditionally is set and the table fits the workspace.
inline bool segs_ready(const Segs& S, const Buffers& b)
{
    return S.seg && S.phase_in && S.phase_out && S.nseg >= 1 && S.nseg <= b.seg_cap &&
           S.nblk <= b.blk_cap;
}

// x folded into [0, L): x - L floor(x / L), unfused, with the rounding
// corner cases (a result of exactly L, or below 0) folded back.
__device__ __forceinline__ double wrap_coord(double x, double L)
{
#pragma clang fp contract(off)
    double r = x - L * floor(x / L);
    if (r < 0.0) r += L;
    if (r >= L) r -= L;
    if (r < 0.0 || r >= L) r = 0.0;
    return r;
}

// Atom i of a caller's positions pos[3][n] as the workspace holds it:
// wrapped into the box, type in w.  A non-finite coordinate raises
// ST_NONFINITE (the atom is placed at the origin) and a type outside
// [0, ntypes) raises ST_TYPES (stored as 0).
__device__ __forceinline__ double4 staged_position(const double* __restrict__ pos,
                                                   const int32_t* __restrict__ types, int ntypes,
                                                   int64_t n, int64_t i, const Box& box,
                                                   unsigned* __restrict__ status)
{
    double x = pos[i], y = pos[n + i], z = pos[2 * n + i];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) {
        atomicOr(status, ST_NONFINITE);
        x = y = z = 0.0;
    }
    int t = types ? types[i] : 0;
    if (t < 0 || t >= ntypes) {
        atomicOr(status, ST_TYPES);
        t = 0;
    }
    return make_double4(wrap_coord(x, box.L[0]), wrap_coord(y, box.L[1]), wrap_coord(z, box.L[2]),
                        (double)t);
}

__host__ __device__ inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }
__host__ __device__ inline int quad_blocks_for(int64_t n) { return (int)((n + kQuadAtoms - 1) / kQuadAtoms); }

// ---- launchers (host) -----------------------------------------------------
hipError_t launch_fill_int(int* p, int64_t count, int value, hipStream_t s);
// Start of a one-structure call in one launch: writes the segment table's
// single entry g (passed by value) to dst, clears the status word, the
// overflow count and the phase word, and zeroes clear[0 .. nclear).
hipError_t launch_begin_single(const Seg& g, Seg* dst, unsigned* status, int* ovf_count,
                               int* phase0, int* clear, int nclear, hipStream_t s);
// Wraps positions pos[3][n] into xw[atom_off ..).
// Types (null: all 0) go to the w component; a type outside [0, ntypes)
// raises ST_TYPES and is stored as 0.
hipError_t launch_load_positions(const double* pos_soa, const int32_t* types, int ntypes,
                                 int64_t n, Box box, int atom_off, double4* xw,
                                 unsigned* status, hipStream_t s);
// Serving batch: wraps positions pos[3][n] into xw0 and xw1 at atom_off and
// copies velocities vel[3][n] into vel_dst (row stride `stride`) at atom_off.
// A non-finite position raises ST_NONFINITE in the batch word and in the
// structure's own word *sst (which the launch first clears).
hipError_t launch_batch_admit(const double* pos, const double* vel, int64_t n, Box box,
                              int atom_off, double4* xw0, double4* xw1, double* vel_dst,
                              int64_t stride, unsigned* status, unsigned* sst, hipStream_t s);
// Serving batch: copies one structure's final positions (from xw), velocities
// and U, F, W, J (row stride `stride`, from atom_off) into caller arrays of n
// atoms; any output may be null.  status_o (or null) receives the status
// code (an mbmd_status value) of the structure's own status word *sst.
hipError_t launch_batch_copy_out(const double4* xw, const double* vel, const double* U,
                                 const double* F, const double* W, const double* J,
                                 int64_t stride, int atom_off, int64_t n, double* pos_o,
                                 double* vel_o, double* U_o, double* F_o, double* W_o,
                                 double* J_o, const unsigned* sst, int32_t* status_o,
                                 hipStream_t s);
// Copies xw[atom_off ..) back to pos[3][n].
hipError_t launch_store_positions(const double4* xw, int atom_off, int64_t n, double* pos_soa,
                                  hipStream_t s);
// Builds the lists and reverse slots of every segment with build != 0 and
// the largest count of each (maxnn).  Lists hold the neighbours inside rcut
// at build time first, each group by ascending index.
// Per-type-pair radii of a list build: pair (a, b) at index a * kMaxTypes + b
// lists atoms closer than sqrt(rl2) and orders those closer than sqrt(rc2)
// first.  The cell grid is sized for the largest radius.
struct ListRadii {
    int nt;
    double rl2[kMaxTypes * kMaxTypes];
    double rc2[kMaxTypes * kMaxTypes];
};

// rlist, rcut: the one radius and cutoff of every pair; `typed` (or null)
// replaces them by per-pair values read with the types in the positions' w
// lanes (rlist must then be the largest list radius).
hipError_t launch_build_neighbors(const Buffers& b, const Segs& S, int total_cells, int cur,
                                  double rlist, double rcut, const ListRadii* typed,
                                  hipStream_t s);

// overflow_pass = false: the fast four-lanes-per-atom pass over every atom;
// true: the pass over the atoms the first one left over.  max_nn bounds the
// in-cutoff count of every atom; the overflow pass is only launched when it
// can exceed the fast path.
template <class T>
hipError_t launch_tersoff_partials(const Buffers& b, const Segs& S, int cur,
                                   const TersoffTable& tab, bool overflow_pass, int max_nn,
                                   hipStream_t s);
template <class T>
hipError_t launch_sw_partials(const Buffers& b, const Segs& S, int cur, const SWParams& p,
                              bool overflow_pass, int max_nn, hipStream_t s);

struct StepArgs {
    int cur;                 // position buffer read this step
    bool check_skin;         // measure how far x_next moved since the list build
    double skin_half2;       // (skin/2)^2
    unsigned long long* disp_slot;  // receives (atomic max) the squared displacement, as bits
    double* part_row;        // this step's row of block partials (null: no thermo)
    bool hold;               // second half-kick only: no drift, positions stay in
                             // buffer cur (the weak-coupling loop drifts separately)
    unsigned* seg_status;    // with check_skin: ST_SKIN is OR-ed into seg_status[sidx]
                             // of a structure whose displacement exceeds skin/2
                             // (null: not reported per structure)
};

// Berendsen weak coupling in the library's units: T0 in K, P0 in eV/A^3,
// beta in A^3/eV, times in fs; tau <= 0 switches that coupling off.
struct NptArgs {
    double T0, tau_T, P0, tau_P, beta, dt;
};

// Per segment, from its phase p and nsteps: second half-kick iff p > 0;
// first half-kick and drift into the other buffer iff p < nsteps and not
// a.hold, else the positions are copied forward unchanged (not at all under
// a.hold); segments with p > nsteps are idle.
template <class T>
hipError_t launch_pair_gather(const Buffers& b, const Segs& S, const StepArgs& a, hipStream_t s);

// Thermo rows [first, first + count) of segment `sid` from the partials ring:
// row k is ring row (ring0 + k) % kThermoRing.
hipError_t launch_thermo_fold(const Buffers& b, const Segs& S, int sid, int first, int count,
                              int ring0, double* thermo, hipStream_t s);
// Batch: for every segment with a thermo pointer that took part in the
// pairwise launch reading S.phase_in, its row for that step from ring row
// `ring_row`.
hipError_t launch_thermo_fold_segments(const Buffers& b, const Segs& S, int ring_row,
                                       hipStream_t s);
// Weak coupling, segment 0: folds ring row `ring_row` into thermo row `step`
// and box_traj row `step` (if not null); unless `last`, forms the thermostat
// and barostat factors from that row, stores them in b.coupling and scales
// the segment's box (b.seg) by mu.
hipError_t launch_npt_fold(const Buffers& b, const Segs& S, int ring_row, int step, bool last,
                           const NptArgs& a, double* thermo, double* box_traj, hipStream_t s);
// Green-Kubo: heat-current autocorrelation hac[max_lag][3] and running
// conductivity kappa[max_lag][3] (null: not formed, scaled by `scale`) from
// S samples, thermo rows 0, every, 2 every, ... (columns 11..13).  scratch
// holds gk_scratch_bytes(S, max_lag) bytes of device memory.
size_t gk_scratch_bytes(int64_t S, int max_lag);
hipError_t launch_green_kubo(const double* thermo, int64_t S, int every, int max_lag,
                             double scale, double* scratch, double* hac, double* kappa,
                             hipStream_t s);
// End of a one-structure run (single segment at atom 0) in one launch:
// positions of buffer cur back to pos[3][n], and thermo rows first ..
// first + count - 1 folded from the ring (ring row = step % kThermoRing).
hipError_t launch_end_single(const Buffers& b, const Segs& S, int first, int count,
                             double* thermo, int cur, double* pos, hipStream_t s);
// Continued one-structure run (single segment at atom 0): stages the
// caller's positions pos[3][n] and applies v <- v + (dt/2) kappa F / m,
// x <- wrap(x + dt v) (the pairwise pass's arithmetic) into buffer cur ^ 1
// in one launch, with slot (or null) taking the largest squared
// displacement from the list-build positions; with thermo (or null) ring row
// ring_row is folded into thermo row 0 by one extra block; *phase_word
// receives phase.
hipError_t launch_resume_prologue(const Buffers& b, const Segs& S, const double* pos,
                                  const int32_t* types, int ntypes, int cur,
                                  unsigned long long* slot, int ring_row, double* thermo,
                                  int* phase_word, int phase, hipStream_t s);
// Weak coupling: v <- lambda v + (dt/2) kappa F / m, x <- wrap(mu x + dt v)
// in the (already scaled) box, in place in position buffer `cur`.
hipError_t launch_npt_drift(const Buffers& b, const Segs& S, int cur, hipStream_t s);

}  // namespace mbmd
