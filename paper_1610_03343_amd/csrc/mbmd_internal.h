// Internal declarations shared by the HIP translation units of libmbmd.
//
// Data layout in device memory (N atoms, M list slots per atom):
//   xw[N]            double4 {x, y, z, 0}: wrapped positions, atom-major so a
//                    neighbour gather is one 32-byte access
//   nn[N]            int32 list count (true count, may exceed M on overflow)
//   nl[M][N]         int32 neighbour index, slot-major (lane i reads nl[m*N+i]
//                    coalesced), ascending index within each atom
//   rev[M][N]        int32 slot of i inside the list of nl[m][i]
//   mask[N]          uint64 bit m set iff slot m lies inside the potential cutoff
//   dpart[M][N][3]   T: dU_i/dr_ij for list slot m (written for in-cutoff slots only)
//   outputs          FP64 SoA: U[N], F[3][N], W[9][N] (component 3a+b), J[3][N]
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
};

constexpr int kBlock = 256;          // threads per block of every per-atom kernel
constexpr int kMaxSlots = 64;        // list capacity limit (cutoff mask is 64-bit)
constexpr int kSiteFastBonds = 8;    // in-cutoff bonds a site pass handles without overflow
constexpr int kThermoCols = 16;      // per-step thermo row
constexpr int kPartialCols = 14;     // per-block partials: U, E_kin, W(9), J(3)
constexpr int kMaxChunk = 256;       // steps enqueued between two checks of the skin
constexpr int kThermoRing = 256;     // per-step rows of block partials kept before a fold

struct Box {
    double L[3];
    double inv[3];
};

// Fixed per-call geometry of the cell grid.
struct CellGrid {
    int nc[3];
    double inv_lc[3];
    int ncell;
};

struct TersoffParams {                // the 1989 single-element form
    double A, B, lam, mu, beta, n, c, d, h, R, S;
};
struct SWParams {                     // the 1985 form
    double epsilon, sigma, a, lam, gamma, A, B, p, q;
};

// Workspace view passed to the launchers.
struct Buffers {
    int64_t n;
    int M;
    double4* xw[2];
    double4* xbuild;
    int* nn;
    int* nl;
    int* rev;
    unsigned long long* mask;
    void* dpart;
    int* cell_of;
    int* cell_count;
    int* cell_start;
    int* cell_fill;
    int* cell_atoms;
    double* part_b;          // [kThermoRing][nblocks][kPartialCols]
    int* ovf_count;          // atoms whose in-cutoff count exceeds the register tile
    int* ovf_list;           // [N]
    unsigned* status;
    double* thermo_scratch;  // [kThermoCols]
    double4* xsnap;          // [N] positions at the start of a checked chunk
    double* vsnap;           // [3][N] velocities at the start of a checked chunk
    unsigned long long* step_disp2;  // [kMaxChunk] largest squared displacement per step
    int* maxnn;                      // largest list count of the last build
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

inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

// ---- launchers (host) -----------------------------------------------------
hipError_t launch_fill_int(int* p, int64_t count, int value, hipStream_t s);
hipError_t launch_load_positions(const double* pos_soa, const int32_t* types, int64_t n,
                                 Box box, double4* xw, unsigned* status, hipStream_t s);
hipError_t launch_store_positions(const double4* xw, int64_t n, double* pos_soa, hipStream_t s);
// Builds the sorted lists, their reverse slots and the largest count (maxnn).
hipError_t launch_build_neighbors(const Buffers& b, int cur, Box box, CellGrid grid,
                                  double rlist, hipStream_t s);

// overflow_pass = false launches the register-tile kernel over all atoms;
// true launches the kernel for the atoms the first pass left over.
// max_nn bounds the in-cutoff count of every atom; the overflow pass is only
// launched when it can exceed the register tile.
template <class T>
hipError_t launch_tersoff_partials(const Buffers& b, int cur, Box box, const TersoffParams& p,
                                   double* U, bool overflow_pass, int max_nn, hipStream_t s);
template <class T>
hipError_t launch_sw_partials(const Buffers& b, int cur, Box box, const SWParams& p,
                              double* U, bool overflow_pass, int max_nn, hipStream_t s);

struct StepArgs {
    int cur;                 // position buffer read this step
    bool kick_before;        // v += dt/2 a before forming J (second half-kick)
    bool advance;            // then v += dt/2 a, x_next = wrap(x + dt v)
    bool check_skin;         // measure how far x_next moved since the list build
    unsigned long long* disp_slot;  // receives (atomic max) the squared displacement, as bits
    double* part_row;        // this step's row of block partials (null: no thermo)
    double half_dt_acc;      // dt/2 * kappa / m
    double dt;
    double skin_half2;       // (skin/2)^2
    double kin_scale;        // m / (2 kappa): E_kin = kin_scale * v^2
};

template <class T>
hipError_t launch_pair_gather(const Buffers& b, Box box, const StepArgs& a, const double* U,
                              double* vel_soa, double* F, double* W, double* J, hipStream_t s);

// Thermo rows of steps [first_step, first_step + count) from the partials ring.
hipError_t launch_thermo_fold(const Buffers& b, int first_step, int count, double* thermo,
                              hipStream_t s);


}  // namespace mbmd
