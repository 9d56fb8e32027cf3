// C ABI of libmbmd (declared in include/mbmd.h): contexts, workspace, and the
// host-side loops that sequence the neighbour build, the site-local partials
// pass and the pairwise-force pass on one HIP stream, for one structure or
// for a batch of independent structures (segments) sharing each launch.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mbmd.h"
#include "mbmd_internal.h"

using namespace mbmd;

// Device scratch of mbmd_compute_noalloc: the whole workspace of one single
// point, so that entry point allocates nothing.  Each device holds its own
// copy while the process runs; host code reaches it only through the address
// hipGetSymbolAddress gives on that device (kept in scratch_ptr), never by
// its name.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex scratch_mu;
bool scratch_looked_up[kScratchDevices] = {};
hipError_t scratch_err[kScratchDevices] = {};
void* scratch_ptr[kScratchDevices] = {};

// Looks up the scratch's address on `device` once (that device current).
void lookup_scratch(int device)
{
    if (device < 0 || device >= kScratchDevices) return;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_looked_up[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    scratch_err[device] = e;
    scratch_ptr[device] = e == hipSuccess ? p : nullptr;
    scratch_looked_up[device] = true;
}
}  // namespace

namespace {
// Kernel classes timed by the optional HIP-event profile.
enum ProfKind {
    P_STAGE, P_BUILD, P_PARTIALS, P_PARTIALS_OVF, P_GATHER, P_THERMO, P_NPT_FOLD, P_NPT_DRIFT,
    P_KINDS
};
const char* const kProfNames[P_KINDS] = {"stage_positions", "neighbor_build", "site_partials",
                                         "site_partials_overflow", "pair_gather", "thermo_fold",
                                         "npt_fold", "npt_drift"};
struct ProfRec {
    int kind;
    hipEvent_t a, b;
};

constexpr double kKappa = 9.64853321567e-3;   // eV/(A amu) in A/fs^2
constexpr double kGPaPerEvA3 = 160.21766208;   // 1 eV/A^3 in GPa
constexpr double kBoltzmannEv = 8.617333262e-5;  // eV/K
constexpr double kWPerMKPerEvFsAK = 1.602176634e6;   // eV/(fs A K) in W/(m K)

// One structure admitted to the serving batch.
struct Slot {
    int handle = -1;
    int atom_off = 0, n = 0;
    Box box{};
    int nsteps = 0;
    int step = 0;            // index of its next step
    double mass = 0, dt = 0;
    double* thermo = nullptr;
    bool started = false;    // stepping (admitted structures wait for a rebuild step)
    int final_buf = 0;       // position buffer holding its final positions
    bool done = false;
    int sidx = 0;            // its per-structure status word
};

// What the last completed mbmd_nve_run left for mbmd_nve_continue: the
// call's arguments (the continuation must name the same state) and where
// its list schedule and thermo ring stand.
struct ResumeState {
    bool valid = false;
    int64_t n = 0;
    double L[3] = {0, 0, 0};
    double mass = 0, dt = 0;
    int every = 0, prec = 0, policy = 0;
    const void *pos = nullptr, *vel = nullptr, *types = nullptr, *F = nullptr;
    int since_build = 0;     // steps taken since the last list build
    int ring_row = 0;        // ring row holding the final state's block partials
    bool ring_valid = false; // ... if the run formed them (it had a thermo array)
};

struct Batch {
    int64_t max_atoms = 0;
    int max_structs = 0;
    int rebuild_every = 10;
    int next_handle = 1;
    int batch_step = 0;
    int phase0 = 0;          // batch step of a list rebuild; they recur every rebuild_every
    int cur = 0;             // position buffer the next launch reads
    bool changed = true;     // segment table must be rebuilt
    std::vector<Slot> slots; // ordered by atom offset
    std::vector<int> table;  // slots (indices) of the segment table, in order
    std::vector<char> sidx_used;   // per-structure status words in use
    // Pinned staging for table uploads, used alternately; an event marks when
    // the stream has consumed each, so uploads never stall the host on the
    // kernels queued ahead of them.
    void* stage[2] = {nullptr, nullptr};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    int stage_k = 0;
};
}  // namespace

struct mbmd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int potential = -1;          // 0 Tersoff, 1 SW
    TersoffTable ttab{};         // Tersoff elements and chi (nt = 1: single element)
    double tmass[kMaxTypes] = {};    // per-type masses (amu) for mass_amu == 0
    int n_tmass = 0;
    SWParams sp{};
    double skin = 0.5;
    int max_nb = 0;              // 0: potential default
    int policy = MBMD_REBUILD_ON_SKIN;
    mbmd_run_stats stats{};
    void* ws = nullptr;          // workspace base
    size_t ws_bytes = 0;
    bool ws_owned = false;
    Buffers buf{};               // layout of the workspace
    int64_t laid_cap = -1;       // layout parameters currently held by buf
    int laid_M = 0, laid_segs = 0;
    bool laid_state = false;
    int max_nn = kMaxSlots;      // largest list count over the segments of the next launch
    int* nn_host = nullptr;      // pinned: per-segment largest list count of the last build
    int nn_host_cap = 0;
    hipEvent_t nn_ev = nullptr;  // marks when nn_host is complete
    bool nn_pending = false;     // max_nn still to be formed from nn_host
    int pp = 0;                  // phase buffer read by the next pairwise launch
    int fold_from = 0;           // single-structure thermo rows pending a fold
    int fold_to = 0;
    std::vector<Seg> segs_host;  // segment table of the current launch set
    Segs segs{};
    Batch* batch = nullptr;
    ResumeState resume;          // the last completed NVE run, for a continuation
    void* gk_ws = nullptr;       // Green-Kubo scratch (own allocation)
    size_t gk_bytes = 0;
    std::string err;
    bool profiling = false;
    std::vector<ProfRec> prof_pending;
    double prof_ms[P_KINDS] = {};
    int64_t prof_launches[P_KINDS] = {};
};

namespace {

constexpr size_t kAlign = 256;

// Records a pair of HIP events on the context's stream around the launches
// made while it is alive (only when profiling is on).
struct ProfScope {
    mbmd_ctx* c;
    int kind;
    hipEvent_t a = nullptr;
    ProfScope(mbmd_ctx* ctx, int k) : c(ctx), kind(k)
    {
        if (c->profiling && hipEventCreate(&a) == hipSuccess) (void)hipEventRecord(a, c->stream);
    }
    ~ProfScope()
    {
        if (!a) return;
        hipEvent_t b = nullptr;
        if (hipEventCreate(&b) == hipSuccess) {
            (void)hipEventRecord(b, c->stream);
            c->prof_pending.push_back(ProfRec{kind, a, b});
        } else {
            (void)hipEventDestroy(a);
        }
    }
};

// Folds the completed event pairs into the per-kind totals (after a sync).
void collect_profile(mbmd_ctx* c)
{
    for (const ProfRec& r : c->prof_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            c->prof_ms[r.kind] += ms;
            c->prof_launches[r.kind] += 1;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    c->prof_pending.clear();
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int64_t cell_cap_for(int64_t cap, int segs) { return 4 * cap + 64 * (int64_t)segs; }

int resolved_M(const mbmd_ctx* c)
{
    if (c->max_nb > 0) return c->max_nb;
    return c->potential == 1 ? 32 : 16;
}

double cutoff_of(const mbmd_ctx* c)
{
    if (c->potential == 1) return c->sp.a * c->sp.sigma;
    double s = 0.0;   // sqrt(S_a S_b) never exceeds the larger S
    for (int a = 0; a < c->ttab.nt; ++a) s = std::max(s, c->ttab.elem[a].S);
    return s;
}

// Atom types the current potential knows (SW: one).
int ntypes_of(const mbmd_ctx* c) { return c->potential == 0 ? c->ttab.nt : 1; }

// Per-pair list radii of a multi-element Tersoff potential: pair (a, b)
// lists atoms within S_ab + skin, S_ab = sqrt(S_a S_b) the pair's cutoff
// (the mixing rule of the multicomponent form), and orders those within
// S_ab first.  False (one radius for every pair) for one element and SW.
bool list_radii(const mbmd_ctx* c, ListRadii& r)
{
    if (c->potential != 0 || c->ttab.nt < 2) return false;
    r = ListRadii{};
    r.nt = c->ttab.nt;
    for (int a = 0; a < r.nt; ++a)
        for (int b = 0; b < r.nt; ++b) {
            const double S = std::sqrt(c->ttab.elem[a].S * c->ttab.elem[b].S);
            const double rl = S + c->skin;
            r.rl2[a * kMaxTypes + b] = rl * rl;
            r.rc2[a * kMaxTypes + b] = S * S;
        }
    return true;
}

// Per-type integrator factors from the context's type masses.
void apply_type_masses(const mbmd_ctx* c, double dt, Seg& g)
{
    g.typed_mass = 1;
    for (int a = 0; a < c->n_tmass; ++a) {
        g.hdt_t[a] = 0.5 * dt * kKappa / c->tmass[a];
        g.kin_t[a] = 0.5 * c->tmass[a] / kKappa;
    }
}

// Lays out every device array for `cap` atoms, M slots and `segs` segments
// from `base` (or only sizes it when base is null); `state` adds the batch's
// own velocity and output arrays.  Returns the total byte count.
size_t layout(int64_t cap, int M, int segs, bool state, char* base, Buffers* b)
{
    const int64_t nn = cap > 0 ? cap : 1;
    const int64_t ccap = cell_cap_for(nn, segs);
    const int64_t nscan = (ccap + kBlock * 4 - 1) / (kBlock * 4);
    // 256-atom blocks, and room for the four rows per block of the four-lane
    // pairwise pass (at most kQuadPairBlocks blocks)
    const int64_t blk_cap = blocks_for(nn) + segs + 3 * kQuadPairBlocks;
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    Buffers t{};
    t.cap = nn;
    t.M = M;
    t.xw[0] = (double4*)take(sizeof(double4) * nn);
    t.xw[1] = (double4*)take(sizeof(double4) * nn);
    t.xbuild = (double4*)take(sizeof(double4) * nn);
    t.nn = (int*)take(sizeof(int) * nn);
    t.nl = (int*)take(sizeof(int) * nn * M);
    t.rev = (uint8_t*)take(sizeof(uint8_t) * nn * M);
    t.mask = (unsigned long long*)take(sizeof(unsigned long long) * nn);
    t.dpart = take(sizeof(double) * 3 * nn * M);
    t.cell_cap = ccap;
    t.cell_count = (int*)take(sizeof(int) * ccap);
    t.cell_start = (int*)take(sizeof(int) * (ccap + 1));
    t.cell_fill = (int*)take(sizeof(int) * (ccap + 1 + nscan));
    t.xcell = (double4*)take(sizeof(double4) * nn);
    t.blk_cap = blk_cap;
    t.part_b = (double*)take(sizeof(double) * kPartialCols * blk_cap * kThermoRing);
    t.ovf_count = (int*)take(sizeof(int));
    t.ovf_list = (int*)take(sizeof(int) * nn);
    t.status = (unsigned*)take(sizeof(unsigned));
    t.sstat = (unsigned*)take(sizeof(unsigned) * segs);
    t.xsnap = (double4*)take(sizeof(double4) * nn);
    t.vsnap = (double*)take(sizeof(double) * 3 * nn);
    t.step_disp2 = (unsigned long long*)take(sizeof(unsigned long long) * kMaxChunk);
    t.maxnn = (int*)take(sizeof(int) * segs);
    t.phase[0] = (int*)take(sizeof(int) * segs);
    t.phase[1] = (int*)take(sizeof(int) * segs);
    t.coupling = (double*)take(sizeof(double) * 2 * segs);
    t.seg = (Seg*)take(sizeof(Seg) * segs);
    t.seg_cap = segs;
    if (state) {
        t.vel = (double*)take(sizeof(double) * 3 * nn);
        t.U = (double*)take(sizeof(double) * nn);
        t.F = (double*)take(sizeof(double) * 3 * nn);
        t.W = (double*)take(sizeof(double) * 9 * nn);
        t.J = (double*)take(sizeof(double) * 3 * nn);
        t.ostride = nn;
    }
    if (b) *b = t;
    return off;
}

mbmd_status fail(mbmd_ctx* c, mbmd_status s, const char* fmt, const char* what = "")
{
    char msg[512];
    snprintf(msg, sizeof msg, fmt, what);
    c->err = msg;
    return s;
}

mbmd_status hip_fail(mbmd_ctx* c, hipError_t e, const char* where)
{
    char msg[512];
    snprintf(msg, sizeof msg, "%s: %s", where, hipGetErrorString(e));
    c->err = msg;
    return MBMD_EDEVICE;
}

// Makes the workspace hold a layout for `cap` atoms and `segs` segments.
mbmd_status ensure_workspace(mbmd_ctx* c, int64_t cap, int segs, bool state)
{
    const int M = resolved_M(c);
    const size_t need = layout(cap, M, segs, state, nullptr, nullptr);
    if (c->ws && !c->ws_owned) {
        if (c->ws_bytes < need)
            return fail(c, MBMD_ENOMEM, "bound workspace too small for this call%s");
    } else if (c->ws_bytes < need) {
        if (c->ws) (void)hipFree(c->ws);
        c->ws = nullptr;
        c->ws_bytes = 0;
        hipError_t e = hipMalloc(&c->ws, need);
        if (e != hipSuccess) {
            c->ws = nullptr;
            return fail(c, MBMD_ENOMEM, "hipMalloc of the workspace failed%s");
        }
        c->ws_bytes = need;
        c->ws_owned = true;
    }
    if (c->laid_cap != cap || c->laid_M != M || c->laid_segs != segs || c->laid_state != state) {
        layout(cap, M, segs, state, (char*)c->ws, &c->buf);
        c->laid_cap = cap;
        c->laid_M = M;
        c->laid_segs = segs;
        c->laid_state = state;
    }
    return MBMD_OK;
}

mbmd_status check_box(mbmd_ctx* c, const double* box, Box* out)
{
    if (!box) return fail(c, MBMD_EINVAL, "box is NULL%s");
    const double rl = cutoff_of(c) + c->skin;
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(box[a]) || !(box[a] >= 2.0 * rl))
            return fail(c, MBMD_EBOX, "box edge shorter than 2 (cutoff + skin)%s");
        out->L[a] = box[a];
        out->inv[a] = 1.0 / box[a];
    }
    return MBMD_OK;
}

// Segment record with its cell grid: cells of side >= r_list, at most
// 4 n + 64 of them (larger cells are always correct).
Seg make_seg(const Box& box, double rlist, int atom_off, int n, int nsteps, double mass,
             double dt, double* thermo)
{
    Seg g{};
    g.box = box;
    const int64_t cap = 4 * (int64_t)n + 64;
    for (int a = 0; a < 3; ++a) {
        const int k = (int)std::floor(box.L[a] / (rlist * (1.0 + 1e-9)));
        g.nc[a] = k < 1 ? 1 : k;
    }
    while ((int64_t)g.nc[0] * g.nc[1] * g.nc[2] > cap) {
        int a = 0;
        if (g.nc[1] > g.nc[a]) a = 1;
        if (g.nc[2] > g.nc[a]) a = 2;
        g.nc[a] = g.nc[a] / 2 > 0 ? g.nc[a] / 2 : 1;
    }
    for (int a = 0; a < 3; ++a) g.inv_lc[a] = g.nc[a] / box.L[a];
    g.ncell = g.nc[0] * g.nc[1] * g.nc[2];
    g.atom_off = atom_off;
    g.n = n;
    g.nsteps = nsteps;
    g.dt = dt;
    if (mass > 0.0) {
        g.half_dt_acc = 0.5 * dt * kKappa / mass;
        g.kin_scale = 0.5 * mass / kKappa;
    }
    g.thermo = thermo;
    return g;
}

// Assigns cell and block offsets in table order (host copy of the table).
void assign_offsets(mbmd_ctx* c, int* total_cells)
{
    int cell = 0, blk = 0, blkq = 0;
    for (Seg& g : c->segs_host) {
        g.cell_off = cell;
        g.blk = blk;
        g.blk_quad = blkq;
        cell += g.ncell;
        blk += blocks_for(g.n);
        blkq += quad_blocks_for(g.n);
    }
    if (total_cells) *total_cells = cell;
    c->segs.seg = c->buf.seg;
    c->segs.nseg = (int)c->segs_host.size();
    c->segs.nblk = blk;
    c->segs.nblk_quad = blkq;
}

// Assigns the offsets and uploads the table from the context's host copy
// (which stays unchanged until the next call drains the stream).
hipError_t upload_segs(mbmd_ctx* c, int* total_cells)
{
    assign_offsets(c, total_cells);
    if (c->segs_host.empty()) return hipSuccess;
    return hipMemcpyAsync(c->buf.seg, c->segs_host.data(), sizeof(Seg) * c->segs_host.size(),
                          hipMemcpyHostToDevice, c->stream);
}

void set_phase_pointers(mbmd_ctx* c)
{
    c->segs.phase_in = c->buf.phase[c->pp];
    c->segs.phase_out = c->buf.phase[c->pp ^ 1];
}

mbmd_status status_to_code(mbmd_ctx* c, unsigned st)
{
    if (st & ST_TYPES) return fail(c, MBMD_EINVAL, "atom type other than 0%s");
    if (st & ST_NONFINITE) return fail(c, MBMD_ENONFINITE, "non-finite position%s");
    if (st & ST_BAROSTAT)
        return fail(c, MBMD_EINVAL,
                    "barostat factor 1 - beta dt/tau_P (P0 - P) <= 0; lower beta dt/tau_P%s");
    if (st & ST_NEIGH_OVERFLOW)
        return fail(c, MBMD_ENEIGH, "neighbour list capacity exceeded; raise max_neighbors%s");
    if (st & ST_ASYMMETRIC) return fail(c, MBMD_EDEVICE, "internal: asymmetric neighbour data%s");
    return MBMD_OK;
}

// Reads (and clears) the status word after draining the stream.
mbmd_status finish(mbmd_ctx* c)
{
    unsigned st = 0;
    hipError_t e = hipMemcpyAsync(&st, c->buf.status, sizeof st, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "stream synchronize");
    collect_profile(c);
    if (st) {
        (void)launch_fill_int((int*)c->buf.status, 1, 0, c->stream);
        (void)hipStreamSynchronize(c->stream);
    }
    return status_to_code(c, st);
}

// Builds the lists of every segment flagged in the table.  With `readback`
// the largest count per segment is copied to pinned host memory behind an
// event, and c->max_nn, the largest over the built segments, is formed from
// it when the partials pass has to decide on its overflow pass: by then the
// fast site pass is already queued, so the GPU computes while the host waits
// for the copy.  Without `readback` the overflow pass is always enqueued (it
// exits at once when no atom overflowed).
hipError_t build(mbmd_ctx* c, int total_cells, int cur, bool readback = true)
{
    hipError_t e;
    {
        ProfScope ps(c, P_BUILD);
        ListRadii r;
        const bool typed = list_radii(c, r);
        e = launch_build_neighbors(c->buf, c->segs, total_cells, cur, cutoff_of(c) + c->skin,
                                   cutoff_of(c), typed ? &r : nullptr, c->stream);
    }
    c->max_nn = kMaxSlots;
    c->nn_pending = false;
    const int ns = c->segs.nseg;
    if (!readback || e != hipSuccess || ns <= 0) return e;
    if (c->nn_host_cap < ns) {
        if (c->nn_host) (void)hipHostFree(c->nn_host);
        c->nn_host = nullptr;
        c->nn_host_cap = 0;
        e = hipHostMalloc((void**)&c->nn_host, sizeof(int) * ns, hipHostMallocDefault);
        if (e != hipSuccess) {
            c->nn_host = nullptr;
            return e;
        }
        c->nn_host_cap = ns;
    }
    if (!c->nn_ev) {
        e = hipEventCreateWithFlags(&c->nn_ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            c->nn_ev = nullptr;
            return e;
        }
    }
    e = hipMemcpyAsync(c->nn_host, c->buf.maxnn, sizeof(int) * ns, hipMemcpyDeviceToHost,
                       c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->nn_ev, c->stream);
    c->nn_pending = e == hipSuccess;
    return e;
}

// Forms c->max_nn from the read-back counts of the last build (waits for
// the copy if it is still in flight).
hipError_t resolve_max_nn(mbmd_ctx* c)
{
    if (!c->nn_pending) return hipSuccess;
    c->nn_pending = false;
    hipError_t e = hipEventSynchronize(c->nn_ev);
    if (e != hipSuccess) return e;
    int mx = 0;
    for (int k = 0; k < c->segs.nseg; ++k)
        if (c->segs_host[k].build) mx = std::max(mx, c->nn_host[k]);
    c->max_nn = mx;
    return hipSuccess;
}

template <class T>
hipError_t partials(mbmd_ctx* c, int cur)
{
    hipError_t e;
    for (int pass = 0; pass < 2; ++pass) {
        // the overflow pass only exists when a site can exceed the fast path
        const int fast = kQuad * (c->potential == 1 ? kSWSlots
                                  : (c->ttab.nt > 1 ? kTersoffMultiSlots : kTersoffSlots));
        if (pass == 1) {
            if (!(c->buf.M > fast)) break;
            e = resolve_max_nn(c);
            if (e != hipSuccess) return e;
            if (!(c->max_nn > fast)) break;
        }
        ProfScope ps(c, pass ? P_PARTIALS_OVF : P_PARTIALS);
        if (c->potential == 1)
            e = launch_sw_partials<T>(c->buf, c->segs, cur, c->sp, pass == 1, c->max_nn,
                                      c->stream);
        else
            e = launch_tersoff_partials<T>(c->buf, c->segs, cur, c->ttab, pass == 1, c->max_nn,
                                           c->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Force evaluation at the positions of buffer `cur` and the pairwise pass
// (integrator per segment phase); flips the phase buffers.
template <class T>
hipError_t force_step(mbmd_ctx* c, int cur, bool check, unsigned long long* slot,
                      double* part_row, bool hold = false, unsigned* seg_status = nullptr)
{
    // the site pass reads the phases too: point both passes at this step's
    set_phase_pointers(c);
    hipError_t e = partials<T>(c, cur);
    StepArgs a{};
    a.cur = cur;
    a.check_skin = check;
    a.skin_half2 = 0.25 * c->skin * c->skin;
    a.disp_slot = slot;
    a.part_row = part_row;
    a.hold = hold;
    a.seg_status = seg_status;
    if (e == hipSuccess) {
        ProfScope ps(c, P_GATHER);
        e = launch_pair_gather<T>(c->buf, c->segs, a, c->stream);
    }
    c->pp ^= 1;
    return e;
}

double* ring_row(mbmd_ctx* c, int row)
{
    return c->buf.part_b + (size_t)(row % kThermoRing) * c->buf.blk_cap * kPartialCols;
}

// ---- one structure ----------------------------------------------------------

// Sets up a one-segment launch set over caller-owned arrays and (unless
// `stage` is false: the caller stages them with its first kernel) stages the
// positions into buffer 0.  The table entry goes to the device as a kernel
// argument of the launch that also clears the status, overflow and phase
// words (and, with clear_disp, the first step-displacement slot): two
// launches and no host-to-device copy.
mbmd_status begin_single(mbmd_ctx* c, int64_t n, const Box& box, const double* pos,
                         const int32_t* types, int nsteps, double mass, double dt, double* vel,
                         double* U, double* F, double* W, double* J, int* total_cells,
                         bool dt_run = false, char* scratch_base = nullptr, bool stage = true,
                         bool clear_disp = false)
{
    if (c->batch) return fail(c, MBMD_EINVAL, "a serving batch is open on this context%s");
    c->resume.valid = false;     // this call reuses the workspace
    if (scratch_base) {
        // the call's whole workspace is laid out over the device scratch; the
        // next ordinary call lays out the context's own workspace again
        layout(n, resolved_M(c), 1, false, scratch_base, &c->buf);
        c->laid_cap = -1;
    } else {
        mbmd_status s = ensure_workspace(c, n, 1, false);
        if (s != MBMD_OK) return s;
    }
    Buffers& b = c->buf;
    b.vel = vel;
    b.U = U;
    b.F = F;
    b.W = W;
    b.J = J;
    b.ostride = n;
    Seg g = make_seg(box, cutoff_of(c) + c->skin, 0, (int)n, nsteps, mass, dt, nullptr);
    // dynamics with mass 0: per-type masses (the entry points check that
    // every type has one)
    if (vel && dt_run && mass == 0.0) apply_type_masses(c, dt, g);
    g.build = 1;
    c->segs_host.assign(1, g);
    c->pp = 0;
    assign_offsets(c, total_cells);
    hipError_t e = launch_begin_single(c->segs_host[0], b.seg, b.status, b.ovf_count, b.phase[0],
                                       clear_disp ? (int*)b.step_disp2 : nullptr,
                                       clear_disp ? 2 : 0, c->stream);
    if (e == hipSuccess && stage) {
        ProfScope ps(c, P_STAGE);
        e = launch_load_positions(pos, types, ntypes_of(c), n, box, 0, b.xw[0], b.status,
                                  c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "staging positions");
    return MBMD_OK;
}

template <class T>
mbmd_status compute_impl(mbmd_ctx* c, int64_t n, const Box& box, const double* pos,
                         const double* vel, const int32_t* types, double* U, double* F,
                         double* W, double* J)
{
    int cells = 0;
    mbmd_status s = begin_single(c, n, box, pos, types, 0, 0.0, 0.0, const_cast<double*>(vel),
                                 U, F, W, J, &cells);
    if (s != MBMD_OK) return s;
    hipError_t e = build(c, cells, 0);
    if (e == hipSuccess) e = force_step<T>(c, 0, false, nullptr, nullptr);
    if (e != hipSuccess) return hip_fail(c, e, "compute launch");
    return finish(c);
}

// Folds the pending per-step partials of the single structure.
hipError_t flush_thermo(mbmd_ctx* c, double* thermo)
{
    if (!thermo || c->fold_to <= c->fold_from) return hipSuccess;
    ProfScope ps(c, P_THERMO);
    hipError_t e = launch_thermo_fold(c->buf, c->segs, 0, c->fold_from, c->fold_to - c->fold_from,
                                      0, thermo, c->stream);
    c->fold_from = c->fold_to;
    return e;
}

// End of a one-structure run: the pending thermo rows and the final
// positions (buffer cur) back to the caller, in one launch.
hipError_t end_single(mbmd_ctx* c, double* thermo, int cur, double* pos)
{
    const int count = thermo && c->fold_to > c->fold_from ? c->fold_to - c->fold_from : 0;
    ProfScope ps(c, P_THERMO);
    hipError_t e = launch_end_single(c->buf, c->segs, c->fold_from, count, thermo, cur, pos,
                                     c->stream);
    if (thermo) c->fold_from = c->fold_to;
    return e;
}

// One MD step of the single structure: force evaluation at the current
// positions, second half-kick, heat current and thermo partials, then
// (unless last) first half-kick and drift.
template <class T>
hipError_t md_step(mbmd_ctx* c, int step, int cur, bool check, unsigned long long* slot,
                   double* thermo)
{
    hipError_t e = force_step<T>(c, cur, check, slot, thermo ? ring_row(c, step) : nullptr);
    if (e == hipSuccess && thermo) {
        if (step < c->fold_from || step > c->fold_to) c->fold_from = step;   // replayed steps
        c->fold_to = step + 1;
        if (c->fold_to - c->fold_from == kThermoRing) e = flush_thermo(c, thermo);
    }
    return e;
}

// Records a completed NVE run for mbmd_nve_continue (prev: the state the
// run itself continued, if it did).
void keep_resume(mbmd_ctx* c, int prec, int64_t n, const Box& box, double mass, const double* pos,
                 const double* vel, const int32_t* types, double dt, int n_steps, int every,
                 const double* F, const double* thermo, int last_build, const ResumeState* prev)
{
    ResumeState r;
    r.valid = true;
    r.n = n;
    for (int a = 0; a < 3; ++a) r.L[a] = box.L[a];
    r.mass = mass;
    r.dt = dt;
    r.every = every;
    r.prec = prec;
    r.policy = c->policy;
    r.pos = pos;
    r.vel = vel;
    r.types = types;
    r.F = F;
    r.since_build = n_steps - last_build;
    if (n_steps > 0 || !prev) {
        r.ring_row = n_steps % kThermoRing;
        r.ring_valid = thermo != nullptr;
    } else {
        r.ring_row = prev->ring_row;
        r.ring_valid = prev->ring_valid;
    }
    c->resume = r;
}

template <class T>
mbmd_status nve_impl(mbmd_ctx* c, int64_t n, const Box& box, double mass, double* pos,
                     double* vel, const int32_t* types, double dt, int n_steps, int every,
                     double* U, double* F, double* W, double* J, double* thermo, bool resume)
{
    // a continuation keeps the lists, the build positions and the thermo
    // ring the previous run left in the workspace
    const ResumeState prev = c->resume;
    int cells = 0;
    // a continuation that takes steps stages the positions with its prologue
    // (whose displacement from the list-build positions is tracked under the
    // skin policy unless the schedule rebuilds at step 1 anyway)
    const bool fused = resume && n_steps > 0;
    const bool chk = fused && c->policy == MBMD_REBUILD_ON_SKIN && 1 + prev.since_build != every;
    mbmd_status s = begin_single(c, n, box, pos, types, n_steps, mass, dt, vel, U, F, W, J,
                                 &cells, true, nullptr, !fused, chk);
    if (s != MBMD_OK) return s;
    const Buffers& b = c->buf;
    mbmd_run_stats st{};
    st.steps = n_steps;
    const double skin_half2 = 0.25 * c->skin * c->skin;
    double committed_max2 = 0.0;
    int cur = 0, last_build = 0, step0 = 0;
    hipError_t e = hipSuccess;
    if (!resume) {
        c->fold_from = c->fold_to = 0;
        e = build(c, cells, cur);
        st.rebuilds = 1;
    } else {
        // Step 0 is the state the previous run ended in: its thermo row is
        // that run's last one, folded again from the ring, and the first
        // half-kick and drift its last step left out come first.
        last_build = -prev.since_build;
        c->fold_from = c->fold_to = 1;
        if (!fused && thermo)
            e = launch_thermo_fold(b, c->segs, 0, 0, 1, prev.ring_row, thermo, c->stream);
        if (e == hipSuccess && fused) {
            // one launch: staging, half-kick and drift into buffer 1, the
            // previous run's last thermo row, and the phase of step 1
            e = launch_resume_prologue(b, c->segs, pos, types, ntypes_of(c), cur,
                                       chk ? b.step_disp2 : nullptr, prev.ring_row, thermo,
                                       b.phase[c->pp], 1, c->stream);
            cur = 1;
            if (e == hipSuccess && chk) {
                unsigned long long bits = 0;
                e = hipMemcpyAsync(&bits, b.step_disp2, sizeof bits, hipMemcpyDeviceToHost,
                                   c->stream);
                if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
                double d2;
                std::memcpy(&d2, &bits, sizeof d2);
                if (e == hipSuccess && d2 > skin_half2) {
                    e = build(c, cells, cur);
                    last_build = 1;
                    ++st.rebuilds;
                } else if (d2 > committed_max2) {
                    committed_max2 = d2;
                }
            }
            if (e == hipSuccess && c->policy == MBMD_REBUILD_ON_SKIN && 1 - last_build == every) {
                e = build(c, cells, cur);
                last_build = 1;
                ++st.rebuilds;
            }
        }
        step0 = 1;
    }

    if (c->policy == MBMD_REBUILD_FIXED) {
        // The list is rebuilt every `every` steps whatever the atoms do; no
        // displacement is tracked (the statistics report -1).
        for (int step = step0; step <= n_steps && e == hipSuccess; ++step) {
            if (step - last_build == every) {
                e = build(c, cells, cur);
                last_build = step;
                ++st.rebuilds;
            }
            if (e == hipSuccess) e = md_step<T>(c, step, cur, false, nullptr, thermo);
            cur ^= 1;
        }
        if (e == hipSuccess) e = end_single(c, thermo, cur, pos);
        if (e != hipSuccess) return hip_fail(c, e, "nve launch");
        s = finish(c);
        st.max_displacement = -1.0;
        c->stats = st;
        if (s == MBMD_OK)
            keep_resume(c, sizeof(T) == 4 ? MBMD_MIXED : MBMD_FP64, n, box, mass, pos, vel, types,
                        dt, n_steps, every, F, thermo, last_build, resume ? &prev : nullptr);
        return s;
    }

    // Rebuild on skin: chunks of steps are enqueued from a snapshot of the
    // state; after each chunk the per-step largest displacement is read
    // back.  If the positions of some step moved more than skin/2 from the
    // last build, the chunk is replayed from the snapshot (bit-identically)
    // up to that step and the list is rebuilt there.
    int step = step0;
    int chunk = every < kMaxChunk ? every : kMaxChunk;
    std::vector<unsigned long long> disp(kMaxChunk);
    while (step <= n_steps && e == hipSuccess) {
        const int cs = step;
        int cend = last_build + every;
        if (cend > n_steps + 1) cend = n_steps + 1;
        if (cend > cs + chunk) cend = cs + chunk;
        const int len = cend - cs;
        const int cur_snap = cur;
        e = hipMemcpyAsync(b.xsnap, b.xw[cur], sizeof(double4) * n, hipMemcpyDeviceToDevice,
                           c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b.vsnap, vel, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice,
                               c->stream);
        if (e == hipSuccess) e = launch_fill_int((int*)b.step_disp2, 2 * len, 0, c->stream);
        for (int k = 0; k < len && e == hipSuccess; ++k) {
            const int sk = cs + k;
            const bool check = sk < n_steps && (sk + 1 - last_build) != every;
            e = md_step<T>(c, sk, cur, check, b.step_disp2 + k, thermo);
            cur ^= 1;
        }
        if (e == hipSuccess) e = flush_thermo(c, thermo);
        if (e == hipSuccess)
            e = hipMemcpyAsync(disp.data(), b.step_disp2, sizeof(unsigned long long) * len,
                               hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) break;
        int bad = -1;   // first step whose positions violate the skin
        for (int k = 0; k < len; ++k) {
            double d2;
            std::memcpy(&d2, &disp[k], sizeof d2);
            if (d2 > skin_half2) {
                bad = cs + k + 1;
                break;
            }
            if (d2 > committed_max2) committed_max2 = d2;
        }
        if (bad < 0) {
            step = cend;
            if (step <= n_steps && step - last_build == every) {
                e = build(c, cells, cur);
                last_build = step;
                ++st.rebuilds;
            }
            continue;
        }
        // replay [cs, bad) from the snapshot, then rebuild at `bad`
        cur = cur_snap;
        e = hipMemcpyAsync(b.xw[cur], b.xsnap, sizeof(double4) * n, hipMemcpyDeviceToDevice,
                           c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(vel, b.vsnap, sizeof(double) * 3 * n, hipMemcpyDeviceToDevice,
                               c->stream);
        if (e == hipSuccess) e = launch_fill_int(b.phase[c->pp], 1, cs, c->stream);
        for (int sk = cs; sk < bad && e == hipSuccess; ++sk) {
            e = md_step<T>(c, sk, cur, false, nullptr, thermo);
            cur ^= 1;
        }
        if (e == hipSuccess) e = build(c, cells, cur);
        last_build = bad;
        step = bad;
        ++st.rebuilds;
        ++st.rollbacks;
        chunk = bad - cs > 0 ? bad - cs : 1;
    }
    if (e == hipSuccess) e = end_single(c, thermo, cur, pos);
    if (e != hipSuccess) return hip_fail(c, e, "nve launch");
    s = finish(c);
    st.max_displacement = std::sqrt(committed_max2);
    c->stats = st;
    if (s == MBMD_OK)
        keep_resume(c, sizeof(T) == 4 ? MBMD_MIXED : MBMD_FP64, n, box, mass, pos, vel, types, dt,
                    n_steps, every, F, thermo, last_build, resume ? &prev : nullptr);
    return s;
}


// Velocity-Verlet with Berendsen weak coupling: per step, the scaling and
// first half-kick and drift (from step 1), a fixed-schedule rebuild on the
// box of that step (read back from the device, whose fold scales it), the
// force evaluation with the second half-kick, then the fold that forms the
// thermo row and the next step's factors.
template <class T>
mbmd_status npt_impl(mbmd_ctx* c, int64_t n, const Box& box, double mass, double* pos,
                     double* vel, const int32_t* types, double dt, int n_steps, int every,
                     const NptArgs& na, double* U, double* F, double* W, double* J,
                     double* thermo, double* box_traj, double* box_out)
{
    int cells = 0;
    mbmd_status s = begin_single(c, n, box, pos, types, n_steps, mass, dt, vel, U, F, W, J,
                                 &cells, true);
    if (s != MBMD_OK) return s;
    const Buffers& b = c->buf;
    const double rlist = cutoff_of(c) + c->skin;
    mbmd_run_stats st{};
    st.steps = n_steps;
    st.max_displacement = -1.0;
    int last_build = 0;
    hipError_t e = build(c, cells, 0);
    st.rebuilds = 1;
    Seg dev_seg{};
    for (int step = 0; step <= n_steps && e == hipSuccess; ++step) {
        if (step > 0) {
            ProfScope ps(c, P_NPT_DRIFT);
            e = launch_npt_drift(b, c->segs, 0, c->stream);
        }
        if (e == hipSuccess && step > 0 && step - last_build == every) {
            e = hipMemcpyAsync(&dev_seg, b.seg, sizeof(Seg), hipMemcpyDeviceToHost, c->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
            if (e != hipSuccess) break;
            for (int a = 0; a < 3; ++a)
                if (!std::isfinite(dev_seg.box.L[a]) || !(dev_seg.box.L[a] >= 2.0 * rlist))
                    return fail(c, MBMD_EBOX,
                                "barostat shrank a box edge below 2 (cutoff + skin)%s");
            Seg g = make_seg(dev_seg.box, rlist, 0, (int)n, n_steps, mass, dt, nullptr);
            if (mass == 0.0) apply_type_masses(c, dt, g);
            g.build = 1;
            c->segs_host.assign(1, g);
            e = upload_segs(c, &cells);
            if (e == hipSuccess) e = build(c, cells, 0);
            last_build = step;
            ++st.rebuilds;
        }
        if (e == hipSuccess) e = force_step<T>(c, 0, false, nullptr, ring_row(c, step), true);
        if (e == hipSuccess) {
            ProfScope ps(c, P_NPT_FOLD);
            e = launch_npt_fold(b, c->segs, step, step, step == n_steps, na, thermo, box_traj,
                                c->stream);
        }
    }
    if (e == hipSuccess) e = launch_store_positions(b.xw[0], 0, n, pos, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&dev_seg, b.seg, sizeof(Seg), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "npt launch");
    s = finish(c);
    for (int a = 0; a < 3; ++a) box_out[a] = dev_seg.box.L[a];
    c->stats = st;
    return s;
}

mbmd_status common_checks(mbmd_ctx* c, int64_t n, const double* box, Box* b)
{
    if (c->potential < 0) return fail(c, MBMD_ENOPOT, "no potential set%s");
    if (n < 0 || n > (int64_t)0x7fffffff) return fail(c, MBMD_EINVAL, "atom count out of range%s");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    return check_box(c, box, b);
}

// ---- serving batch -----------------------------------------------------------

// First free atom range of length n in [0, max_atoms), or -1.
int64_t find_range(const Batch& B, int64_t n)
{
    int64_t at = 0;
    for (const Slot& s : B.slots) {
        if (s.atom_off - at >= n) return at;
        at = s.atom_off + s.n;
    }
    return B.max_atoms - at >= n ? at : -1;
}

Slot* find_slot(Batch& B, int handle)
{
    for (Slot& s : B.slots)
        if (s.handle == handle) return &s;
    return nullptr;
}

// Segment table of the batch in atom order with this step's build flags; the
// phase of each segment (its slot's step counter, nsteps + 1 once finished)
// goes into the phase buffer the next launch reads.  Both are staged in
// pinned memory and copied asynchronously.
// Segment table of the started structures (build flag on every unfinished
// one when `rebuild`), uploaded through the pinned staging buffers.
hipError_t batch_table(mbmd_ctx* c, int* total_cells, bool rebuild)
{
    Batch& B = *c->batch;
    c->segs_host.clear();
    B.table.clear();
    const double rl = cutoff_of(c) + c->skin;
    for (size_t q = 0; q < B.slots.size(); ++q) {
        const Slot& s = B.slots[q];
        if (!s.started) continue;
        Seg g = make_seg(s.box, rl, s.atom_off, s.n, s.nsteps, s.mass, s.dt, s.thermo);
        g.build = rebuild && !s.done;
        g.sidx = s.sidx;
        c->segs_host.push_back(g);
        B.table.push_back((int)q);
    }
    assign_offsets(c, total_cells);
    const size_t ns = B.table.size();
    if (ns == 0) return hipSuccess;
    const int k = B.stage_k;
    B.stage_k ^= 1;
    // the copy issued from this staging buffer two uploads ago has completed
    hipError_t e = hipEventSynchronize(B.stage_ev[k]);
    if (e != hipSuccess) return e;
    Seg* hs = static_cast<Seg*>(B.stage[k]);
    int* hp = reinterpret_cast<int*>(hs + B.max_structs);
    for (size_t q = 0; q < ns; ++q) {
        hs[q] = c->segs_host[q];
        const Slot& s = B.slots[B.table[q]];
        hp[q] = s.done ? s.nsteps + 1 : s.step;
    }
    e = hipMemcpyAsync(c->buf.seg, hs, sizeof(Seg) * ns, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->buf.phase[c->pp], hp, sizeof(int) * ns, hipMemcpyHostToDevice,
                           c->stream);
    if (e == hipSuccess) e = hipEventRecord(B.stage_ev[k], c->stream);
    return e;
}

size_t batch_stage_bytes(int max_structs) { return (sizeof(Seg) + sizeof(int)) * max_structs; }

void free_batch(mbmd_ctx* c)
{
    Batch* B = c->batch;
    if (!B) return;
    (void)hipStreamSynchronize(c->stream);
    for (int k = 0; k < 2; ++k) {
        if (B->stage_ev[k]) (void)hipEventDestroy(B->stage_ev[k]);
        if (B->stage[k]) (void)hipHostFree(B->stage[k]);
    }
    delete B;
    c->batch = nullptr;
}

template <class T>
mbmd_status batch_step_impl(mbmd_ctx* c, int* n_active)
{
    Batch& B = *c->batch;
    int running = 0, waiting = 0;
    for (const Slot& s : B.slots) {
        if (s.done) continue;
        if (s.started) ++running;
        else ++waiting;
    }
    // Lists are rebuilt for every running structure at the batch steps
    // phase0 + k rebuild_every; an admitted structure starts at the next of
    // them, so its own rebuild steps are 0, rebuild_every, ... as when it
    // runs alone, and one build launch serves the whole batch.  An idle
    // batch starts a new phase at once.
    if (running == 0) B.phase0 = B.batch_step;
    const bool due = (B.batch_step - B.phase0) % B.rebuild_every == 0;
    if (due && waiting > 0) {
        for (Slot& s : B.slots)
            if (!s.done) s.started = true;
        running += waiting;
        B.changed = true;
    }
    if (n_active) *n_active = running;
    if (running == 0) return MBMD_OK;
    hipError_t e = hipSuccess;
    int cells = 0;
    if (B.changed || due) {
        e = batch_table(c, &cells, due);
        B.changed = false;
    }
    if (e == hipSuccess && due) {
        e = build(c, cells, B.cur, false);
        // the uploaded table carries build flags: the next step uploads one
        // without them
        B.changed = true;
    }
    // no list counts are read back in the batch: the overflow pass is always
    // enqueued
    c->max_nn = kMaxSlots;
    const int row = B.batch_step % kThermoRing;
    // Unless the next batch step rebuilds the lists, every atom's drift is
    // measured from its position at the last build: a structure whose atoms
    // moved more than skin/2 gets its skin bit, reported when it is retired
    // (its lists may then miss pairs; the step is not checked against the
    // positions the next build sees).
    const bool next_due = (B.batch_step + 1 - B.phase0) % B.rebuild_every == 0;
    if (e == hipSuccess)
        e = force_step<T>(c, B.cur, !next_due, nullptr, ring_row(c, row), false,
                          c->buf.sstat);
    if (e == hipSuccess) {
        // the fold reads the phase buffer the pairwise launch read
        ProfScope ps(c, P_THERMO);
        Segs S = c->segs;
        S.phase_in = c->buf.phase[c->pp ^ 1];
        e = launch_thermo_fold_segments(c->buf, S, row, c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "batch step");
    B.cur ^= 1;
    ++B.batch_step;
    for (Slot& s : B.slots) {
        if (s.done || !s.started) continue;
        if (s.step == s.nsteps) {
            s.done = true;
            s.final_buf = B.cur;
        }
        ++s.step;
    }
    return MBMD_OK;
}

}  // namespace

extern "C" {

mbmd_status mbmd_create(mbmd_ctx** out, int device, void* hip_stream)
{
    if (!out) return MBMD_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return MBMD_EDEVICE;
    if (hipSetDevice(device) != hipSuccess) return MBMD_EDEVICE;
    mbmd_ctx* c = new (std::nothrow) mbmd_ctx();
    if (!c) return MBMD_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    // the address of the no-allocation scratch on this device (once per
    // device; a failure is reported by mbmd_compute_noalloc)
    lookup_scratch(device);
    *out = c;
    return MBMD_OK;
}

void mbmd_destroy(mbmd_ctx* c)
{
    if (!c) return;
    for (const ProfRec& r : c->prof_pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    if (c->ws && c->ws_owned) {
        (void)hipSetDevice(c->device);
        (void)hipFree(c->ws);
    }
    if (c->gk_ws) {
        (void)hipSetDevice(c->device);
        (void)hipFree(c->gk_ws);
    }
    if (c->nn_host) (void)hipHostFree(c->nn_host);
    if (c->nn_ev) (void)hipEventDestroy(c->nn_ev);
    free_batch(c);
    delete c;
}

const char* mbmd_last_error(const mbmd_ctx* c) { return c ? c->err.c_str() : "null context"; }

bool tersoff_params_ok(const mbmd_tersoff_params* p)
{
    const double v[] = {p->A, p->B, p->lambda, p->mu, p->beta, p->n, p->c, p->d, p->h, p->R, p->S};
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return p->R > 0.0 && p->S > p->R && p->n > 0.0 && p->beta > 0.0 && p->d != 0.0;
}

mbmd_status mbmd_set_tersoff_multi(mbmd_ctx* c, int ntypes, const mbmd_tersoff_params* elem,
                                   const double* chi)
{
    if (!c || !elem) return MBMD_EINVAL;
    c->resume.valid = false;
    if (c->batch) return fail(c, MBMD_EINVAL, "a serving batch is open on this context%s");
    if (ntypes < 1 || ntypes > kMaxTypes)
        return fail(c, MBMD_EINVAL, "ntypes must be in 1..4%s");
    for (int a = 0; a < ntypes; ++a)
        if (!tersoff_params_ok(&elem[a]))
            return fail(c, MBMD_EINVAL,
                        "Tersoff parameters need finite values, 0 < R < S, n > 0, beta > 0, d != 0%s");
    if (chi)
        for (int a = 0; a < ntypes; ++a)
            for (int b = 0; b < ntypes; ++b) {
                const double x = chi[a * ntypes + b];
                if (!std::isfinite(x) || !(x > 0.0) || x != chi[b * ntypes + a])
                    return fail(c, MBMD_EINVAL, "chi must be finite, positive and symmetric%s");
            }
    TersoffTable t{};
    t.nt = ntypes;
    for (int a = 0; a < ntypes; ++a) {
        const mbmd_tersoff_params* p = &elem[a];
        t.elem[a] = TersoffParams{p->A, p->B, p->lambda, p->mu, p->beta, p->n, p->c, p->d, p->h,
                                  p->R, p->S};
        for (int b = 0; b < ntypes; ++b) t.chi[a * kMaxTypes + b] = chi ? chi[a * ntypes + b] : 1.0;
    }
    c->ttab = t;
    c->potential = 0;
    c->laid_cap = -1;
    return MBMD_OK;
}

mbmd_status mbmd_set_type_masses(mbmd_ctx* c, int ntypes, const double* mass_amu)
{
    if (!c) return MBMD_EINVAL;
    c->resume.valid = false;
    if (ntypes == 0) {
        c->n_tmass = 0;
        return MBMD_OK;
    }
    if (ntypes < 0 || ntypes > kMaxTypes || !mass_amu)
        return fail(c, MBMD_EINVAL, "ntypes must be in 0..4 with a mass array%s");
    for (int a = 0; a < ntypes; ++a)
        if (!std::isfinite(mass_amu[a]) || !(mass_amu[a] > 0.0))
            return fail(c, MBMD_EINVAL, "masses must be finite and positive%s");
    for (int a = 0; a < ntypes; ++a) c->tmass[a] = mass_amu[a];
    c->n_tmass = ntypes;
    return MBMD_OK;
}

mbmd_status mbmd_set_tersoff(mbmd_ctx* c, const mbmd_tersoff_params* p)
{
    if (!c || !p) return MBMD_EINVAL;
    c->resume.valid = false;
    if (c->batch) return fail(c, MBMD_EINVAL, "a serving batch is open on this context%s");
    if (!tersoff_params_ok(p))
        return fail(c, MBMD_EINVAL,
                    "Tersoff parameters need finite values, 0 < R < S, n > 0, beta > 0, d != 0%s");
    c->ttab = TersoffTable{};
    c->ttab.nt = 1;
    c->ttab.elem[0] =
        TersoffParams{p->A, p->B, p->lambda, p->mu, p->beta, p->n, p->c, p->d, p->h, p->R, p->S};
    c->ttab.chi[0] = 1.0;
    c->potential = 0;
    c->laid_cap = -1;
    return MBMD_OK;
}

mbmd_status mbmd_set_sw(mbmd_ctx* c, const mbmd_sw_params* p)
{
    if (!c || !p) return MBMD_EINVAL;
    c->resume.valid = false;
    if (c->batch) return fail(c, MBMD_EINVAL, "a serving batch is open on this context%s");
    const double v[] = {p->epsilon, p->sigma, p->a, p->lambda, p->gamma, p->A, p->B, p->p, p->q};
    for (double x : v)
        if (!std::isfinite(x)) return fail(c, MBMD_EINVAL, "non-finite SW parameter%s");
    if (!(p->sigma > 0.0) || !(p->a > 0.0))
        return fail(c, MBMD_EINVAL, "SW parameters need sigma > 0 and a > 0%s");
    c->sp = SWParams{p->epsilon, p->sigma, p->a, p->lambda, p->gamma, p->A, p->B, p->p, p->q};
    c->potential = 1;
    c->laid_cap = -1;
    return MBMD_OK;
}

mbmd_status mbmd_set_neighbor(mbmd_ctx* c, double skin, int max_neighbors)
{
    if (!c) return MBMD_EINVAL;
    c->resume.valid = false;
    if (c->batch) return fail(c, MBMD_EINVAL, "a serving batch is open on this context%s");
    if (!std::isfinite(skin) || skin < 0.0) return fail(c, MBMD_EINVAL, "skin must be >= 0%s");
    if (max_neighbors < 0 || max_neighbors > kMaxSlots)
        return fail(c, MBMD_EINVAL, "max_neighbors must be in 0..64%s");
    c->skin = skin;
    c->max_nb = max_neighbors;
    c->laid_cap = -1;
    return MBMD_OK;
}

mbmd_status mbmd_set_rebuild_policy(mbmd_ctx* c, mbmd_rebuild_policy policy)
{
    if (!c) return MBMD_EINVAL;
    c->resume.valid = false;
    if (policy != MBMD_REBUILD_FIXED && policy != MBMD_REBUILD_ON_SKIN)
        return fail(c, MBMD_EINVAL, "unknown rebuild policy%s");
    c->policy = policy;
    return MBMD_OK;
}

mbmd_status mbmd_get_run_stats(const mbmd_ctx* c, mbmd_run_stats* out)
{
    if (!c || !out) return MBMD_EINVAL;
    *out = c->stats;
    return MBMD_OK;
}

mbmd_status mbmd_set_profiling(mbmd_ctx* c, int enable)
{
    if (!c) return MBMD_EINVAL;
    c->profiling = enable != 0;
    return MBMD_OK;
}

mbmd_status mbmd_reset_profile(mbmd_ctx* c)
{
    if (!c) return MBMD_EINVAL;
    collect_profile(c);
    for (int k = 0; k < P_KINDS; ++k) {
        c->prof_ms[k] = 0.0;
        c->prof_launches[k] = 0;
    }
    return MBMD_OK;
}

mbmd_status mbmd_get_profile(const mbmd_ctx* c, mbmd_kernel_time* out, int capacity, int* count)
{
    if (!c || !count || capacity < 0 || (capacity > 0 && !out)) return MBMD_EINVAL;
    *count = P_KINDS;
    for (int k = 0; k < P_KINDS && k < capacity; ++k) {
        out[k].name = kProfNames[k];
        out[k].launches = c->prof_launches[k];
        out[k].total_ms = c->prof_ms[k];
    }
    return MBMD_OK;
}

mbmd_status mbmd_get_max_neighbors(const mbmd_ctx* c, int* out)
{
    if (!c || !out) return MBMD_EINVAL;
    *out = resolved_M(c);
    return MBMD_OK;
}

mbmd_status mbmd_workspace_size(const mbmd_ctx* c, int64_t n_atoms, size_t* bytes)
{
    if (!c || !bytes || n_atoms < 0) return MBMD_EINVAL;
    *bytes = layout(n_atoms, resolved_M(c), 1, false, nullptr, nullptr);
    return MBMD_OK;
}

mbmd_status mbmd_batch_workspace_size(const mbmd_ctx* c, int64_t max_atoms, int max_structures,
                                      size_t* bytes)
{
    if (!c || !bytes || max_atoms < 1 || max_structures < 1) return MBMD_EINVAL;
    *bytes = layout(max_atoms, resolved_M(c), max_structures, true, nullptr, nullptr);
    return MBMD_OK;
}

mbmd_status mbmd_bind_workspace(mbmd_ctx* c, void* dev_ptr, size_t bytes)
{
    if (!c) return MBMD_EINVAL;
    c->resume.valid = false;
    if (c->batch) return fail(c, MBMD_EINVAL, "a serving batch is open on this context%s");
    if (dev_ptr && ((uintptr_t)dev_ptr % kAlign) != 0)
        return fail(c, MBMD_EINVAL, "workspace must be 256-byte aligned%s");
    if (c->ws && c->ws_owned) {
        (void)hipSetDevice(c->device);
        (void)hipFree(c->ws);
    }
    c->ws = dev_ptr;
    c->ws_bytes = dev_ptr ? bytes : 0;
    c->ws_owned = false;
    c->laid_cap = -1;
    return MBMD_OK;
}

mbmd_status mbmd_neighbors(mbmd_ctx* c, int64_t n, const double box[3], const double* pos,
                           const int32_t* types, int32_t* nn, int32_t* nl)
{
    if (!c) return MBMD_EINVAL;
    Box b{};
    mbmd_status s = common_checks(c, n, box, &b);
    if (s != MBMD_OK) return s;
    if (n == 0) return MBMD_OK;
    if (!pos || !nn || !nl) return fail(c, MBMD_EINVAL, "null device pointer%s");
    int cells = 0;
    s = begin_single(c, n, b, pos, types, 0, 0.0, 0.0, nullptr, nullptr, nullptr, nullptr,
                     nullptr, &cells);
    if (s != MBMD_OK) return s;
    hipError_t e = build(c, cells, 0);
    const int M = c->buf.M;
    if (e == hipSuccess)
        e = hipMemcpyAsync(nn, c->buf.nn, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(nl, c->buf.nl, sizeof(int32_t) * n * M, hipMemcpyDeviceToDevice,
                           c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "neighbour build");
    return finish(c);
}

mbmd_status mbmd_compute(mbmd_ctx* c, mbmd_precision prec, int64_t n, const double box[3],
                         const double* pos, const double* vel, const int32_t* types, double* U,
                         double* F, double* W, double* J)
{
    if (!c) return MBMD_EINVAL;
    Box b{};
    mbmd_status s = common_checks(c, n, box, &b);
    if (s != MBMD_OK) return s;
    if (prec != MBMD_FP64 && prec != MBMD_MIXED) return fail(c, MBMD_EINVAL, "bad precision%s");
    if (n == 0) return MBMD_OK;
    if (!pos || !U || !F || !W || !J) return fail(c, MBMD_EINVAL, "null device pointer%s");
    if (prec == MBMD_MIXED) return compute_impl<float>(c, n, b, pos, vel, types, U, F, W, J);
    return compute_impl<double>(c, n, b, pos, vel, types, U, F, W, J);
}

mbmd_status mbmd_compute_noalloc(mbmd_ctx* c, mbmd_precision prec, int64_t n,
                                 const double box[3], const double* pos, const double* vel,
                                 const int32_t* types, double* U, double* F, double* W,
                                 double* J)
{
    if (!c) return MBMD_EINVAL;
    Box b{};
    mbmd_status s = common_checks(c, n, box, &b);
    if (s != MBMD_OK) return s;
    if (prec != MBMD_FP64 && prec != MBMD_MIXED) return fail(c, MBMD_EINVAL, "bad precision%s");
    if (n == 0) return MBMD_OK;
    if (!pos || !U || !F || !W || !J) return fail(c, MBMD_EINVAL, "null device pointer%s");
    if (c->device < 0 || c->device >= kScratchDevices || !scratch_ptr[c->device]) {
        char msg[256];
        snprintf(msg, sizeof msg, "no device scratch on device %d (%s)", c->device,
                 c->device >= 0 && c->device < kScratchDevices
                     ? hipGetErrorString(scratch_err[c->device]) : "device index too large");
        c->err = msg;
        return MBMD_EDEVICE;
    }
    const size_t need = layout(n, resolved_M(c), 1, false, nullptr, nullptr);
    if (need > kScratchBytes) {
        char msg[256];
        snprintf(msg, sizeof msg,
                 "%lld atoms need %zu bytes of workspace, more than the %zu-byte static "
                 "scratch of mbmd_compute_noalloc", (long long)n, need, kScratchBytes);
        c->err = msg;
        return MBMD_ENOMEM;
    }
    // no HIP events either: profiling is off for this call
    const bool prof = c->profiling;
    c->profiling = false;
    int cells = 0;
    s = begin_single(c, n, b, pos, types, 0, 0.0, 0.0, const_cast<double*>(vel), U, F, W, J,
                     &cells, false, static_cast<char*>(scratch_ptr[c->device]));
    hipError_t e = hipSuccess;
    if (s == MBMD_OK) {
        // no list counts are read back (that needs pinned host memory): the
        // overflow pass is enqueued and exits at once if no site overflowed
        e = build(c, cells, 0, false);
        c->max_nn = kMaxSlots;
        if (e == hipSuccess)
            e = prec == MBMD_MIXED ? force_step<float>(c, 0, false, nullptr, nullptr)
                                   : force_step<double>(c, 0, false, nullptr, nullptr);
        s = e != hipSuccess ? hip_fail(c, e, "compute launch") : finish(c);
    }
    c->profiling = prof;
    return s;
}

mbmd_status mbmd_nve_run(mbmd_ctx* c, mbmd_precision prec, int64_t n, const double box[3],
                         double mass_amu, double* pos, double* vel, const int32_t* types,
                         double dt_fs, int n_steps, int rebuild_every, double* U, double* F,
                         double* W, double* J, double* thermo)
{
    if (!c) return MBMD_EINVAL;
    Box b{};
    mbmd_status s = common_checks(c, n, box, &b);
    if (s != MBMD_OK) return s;
    if (prec != MBMD_FP64 && prec != MBMD_MIXED) return fail(c, MBMD_EINVAL, "bad precision%s");
    if (!std::isfinite(mass_amu) || mass_amu < 0.0 || !std::isfinite(dt_fs) || n_steps < 0 ||
        rebuild_every < 1)
        return fail(c, MBMD_EINVAL, "need mass >= 0, finite dt, n_steps >= 0, rebuild_every >= 1%s");
    if (mass_amu == 0.0 && c->n_tmass < ntypes_of(c))
        return fail(c, MBMD_EINVAL, "mass 0 needs a type mass for every atom type%s");
    if (n == 0) return MBMD_OK;
    if (!pos || !vel || !U || !F || !W || !J) return fail(c, MBMD_EINVAL, "null device pointer%s");
    if (prec == MBMD_MIXED)
        return nve_impl<float>(c, n, b, mass_amu, pos, vel, types, dt_fs, n_steps, rebuild_every,
                               U, F, W, J, thermo, false);
    return nve_impl<double>(c, n, b, mass_amu, pos, vel, types, dt_fs, n_steps, rebuild_every, U,
                            F, W, J, thermo, false);
}

mbmd_status mbmd_nve_continue(mbmd_ctx* c, mbmd_precision prec, int64_t n, const double box[3],
                              double mass_amu, double* pos, double* vel, const int32_t* types,
                              double dt_fs, int n_steps, int rebuild_every, double* U, double* F,
                              double* W, double* J, double* thermo)
{
    if (!c) return MBMD_EINVAL;
    Box b{};
    mbmd_status s = common_checks(c, n, box, &b);
    if (s != MBMD_OK) return s;
    if (n_steps < 0) return fail(c, MBMD_EINVAL, "need n_steps >= 0%s");
    if (!pos || !vel || !U || !F || !W || !J) return fail(c, MBMD_EINVAL, "null device pointer%s");
    const ResumeState& r = c->resume;
    if (!r.valid)
        return fail(c, MBMD_EINVAL,
                    "nothing to continue: the last call on this context was not a completed "
                    "mbmd_nve_run or mbmd_nve_continue%s");
    const bool same = r.n == n && r.L[0] == b.L[0] && r.L[1] == b.L[1] && r.L[2] == b.L[2] &&
                      r.mass == mass_amu && r.dt == dt_fs && r.every == rebuild_every &&
                      r.prec == (int)prec && r.policy == c->policy && r.pos == pos &&
                      r.vel == vel && r.types == types && r.F == F;
    if (!same)
        return fail(c, MBMD_EINVAL,
                    "a continuation takes the arguments of the run it continues (n, box, mass, "
                    "dt, rebuild_every, precision, policy and the pos, vel, types and F "
                    "buffers)%s");
    if (thermo && !r.ring_valid)
        return fail(c, MBMD_EINVAL,
                    "thermo rows of a continuation need a thermo array in the run it "
                    "continues%s");
    if (n == 0) return MBMD_OK;
    if (prec == MBMD_MIXED)
        return nve_impl<float>(c, n, b, mass_amu, pos, vel, types, dt_fs, n_steps, rebuild_every,
                               U, F, W, J, thermo, true);
    return nve_impl<double>(c, n, b, mass_amu, pos, vel, types, dt_fs, n_steps, rebuild_every, U,
                            F, W, J, thermo, true);
}

mbmd_status mbmd_npt_run(mbmd_ctx* c, mbmd_precision prec, int64_t n, double box[3],
                         double mass_amu, double* pos, double* vel, const int32_t* types,
                         double dt_fs, int n_steps, int rebuild_every,
                         const mbmd_berendsen* coupling, double* U, double* F, double* W,
                         double* J, double* thermo, double* box_traj)
{
    if (!c) return MBMD_EINVAL;
    Box b{};
    mbmd_status s = common_checks(c, n, box, &b);
    if (s != MBMD_OK) return s;
    if (prec != MBMD_FP64 && prec != MBMD_MIXED) return fail(c, MBMD_EINVAL, "bad precision%s");
    if (!std::isfinite(mass_amu) || mass_amu < 0.0 || !std::isfinite(dt_fs) ||
        !(dt_fs > 0.0) || n_steps < 0 || rebuild_every < 1)
        return fail(c, MBMD_EINVAL, "need mass >= 0, dt > 0, n_steps >= 0, rebuild_every >= 1%s");
    if (mass_amu == 0.0 && c->n_tmass < ntypes_of(c))
        return fail(c, MBMD_EINVAL, "mass 0 needs a type mass for every atom type%s");
    if (!coupling) return fail(c, MBMD_EINVAL, "coupling is NULL%s");
    const mbmd_berendsen& k = *coupling;
    if (!std::isfinite(k.T0_K) || k.T0_K < 0.0 || !std::isfinite(k.P0_GPa) ||
        !std::isfinite(k.beta_per_GPa) || k.beta_per_GPa < 0.0 || !std::isfinite(k.tau_T_fs) ||
        !std::isfinite(k.tau_P_fs) || (k.tau_T_fs > 0.0 && k.tau_T_fs < dt_fs))
        return fail(c, MBMD_EINVAL,
                    "need finite T0 >= 0, P0, beta >= 0, tau_T, tau_P; tau_T >= dt when on%s");
    if (n == 0) return MBMD_OK;
    if (!pos || !vel || !U || !F || !W || !J || !thermo)
        return fail(c, MBMD_EINVAL, "null device pointer%s");
    NptArgs na{};
    na.T0 = k.T0_K;
    na.tau_T = k.tau_T_fs;
    na.P0 = k.P0_GPa / kGPaPerEvA3;
    na.tau_P = k.tau_P_fs;
    na.beta = k.beta_per_GPa * kGPaPerEvA3;
    na.dt = dt_fs;
    if (prec == MBMD_MIXED)
        return npt_impl<float>(c, n, b, mass_amu, pos, vel, types, dt_fs, n_steps, rebuild_every,
                               na, U, F, W, J, thermo, box_traj, box);
    return npt_impl<double>(c, n, b, mass_amu, pos, vel, types, dt_fs, n_steps, rebuild_every,
                            na, U, F, W, J, thermo, box_traj, box);
}

mbmd_status mbmd_green_kubo(mbmd_ctx* c, const double* thermo, int64_t n_rows, int sample_every,
                            int max_lag, double dt_fs, double volume_A3, double T_K, double* hac,
                            double* kappa)
{
    if (!c) return MBMD_EINVAL;
    if (!thermo || !hac) return fail(c, MBMD_EINVAL, "null device pointer%s");
    if (n_rows < 1 || sample_every < 1 || max_lag < 1)
        return fail(c, MBMD_EINVAL, "need n_rows >= 1, sample_every >= 1, max_lag >= 1%s");
    const int64_t S = (n_rows - 1) / sample_every + 1;
    if (max_lag > S) return fail(c, MBMD_EINVAL, "max_lag exceeds the number of samples%s");
    if (!(dt_fs > 0.0) || !(volume_A3 > 0.0) || !(T_K > 0.0) || !std::isfinite(dt_fs) ||
        !std::isfinite(volume_A3) || !std::isfinite(T_K))
        return fail(c, MBMD_EINVAL, "need finite dt, volume and temperature > 0%s");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    const size_t need = gk_scratch_bytes(S, max_lag);
    if (c->gk_bytes < need) {
        if (c->gk_ws) (void)hipFree(c->gk_ws);
        c->gk_ws = nullptr;
        c->gk_bytes = 0;
        if (hipMalloc(&c->gk_ws, need) != hipSuccess) {
            c->gk_ws = nullptr;
            return fail(c, MBMD_ENOMEM, "hipMalloc of the correlation scratch failed%s");
        }
        c->gk_bytes = need;
    }
    const double dtau = dt_fs * sample_every;
    const double scale = dtau / (kBoltzmannEv * T_K * T_K * volume_A3) * kWPerMKPerEvFsAK;
    e = launch_green_kubo(thermo, S, sample_every, max_lag, scale, (double*)c->gk_ws, hac, kappa,
                          c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "green-kubo launch");
    return MBMD_OK;
}

// ---- serving batch ----------------------------------------------------------

mbmd_status mbmd_batch_open(mbmd_ctx* c, int64_t max_atoms, int max_structures,
                            int rebuild_every)
{
    if (!c) return MBMD_EINVAL;
    c->resume.valid = false;
    if (c->potential < 0) return fail(c, MBMD_ENOPOT, "no potential set%s");
    if (c->batch) return fail(c, MBMD_EINVAL, "a serving batch is already open%s");
    if (max_atoms < 1 || max_atoms > (int64_t)0x3fffffff || max_structures < 1 ||
        max_structures > (1 << 20) || rebuild_every < 1)
        return fail(c, MBMD_EINVAL,
                    "need max_atoms >= 1, max_structures >= 1, rebuild_every >= 1%s");
    hipError_t he = hipSetDevice(c->device);
    if (he != hipSuccess) return hip_fail(c, he, "hipSetDevice");
    mbmd_status s = ensure_workspace(c, max_atoms, max_structures, true);
    if (s != MBMD_OK) return s;
    Batch* B = new (std::nothrow) Batch();
    if (!B) return MBMD_ENOMEM;
    B->max_atoms = max_atoms;
    B->max_structs = max_structures;
    B->sidx_used.assign(max_structures, 0);
    B->rebuild_every = rebuild_every;
    c->batch = B;
    for (int k = 0; k < 2; ++k) {
        if (hipHostMalloc(&B->stage[k], batch_stage_bytes(max_structures)) != hipSuccess) {
            B->stage[k] = nullptr;
            free_batch(c);
            return fail(c, MBMD_ENOMEM, "pinned staging for the batch table%s");
        }
        if (hipEventCreateWithFlags(&B->stage_ev[k], hipEventDisableTiming) != hipSuccess) {
            B->stage_ev[k] = nullptr;
            free_batch(c);
            return fail(c, MBMD_EDEVICE, "event for the batch table%s");
        }
    }
    c->pp = 0;
    hipError_t e = launch_fill_int((int*)c->buf.status, 1, 0, c->stream);
    if (e == hipSuccess) e = launch_fill_int(c->buf.ovf_count, 1, 0, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "batch open");
    return MBMD_OK;
}

mbmd_status mbmd_batch_close(mbmd_ctx* c)
{
    if (!c) return MBMD_EINVAL;
    free_batch(c);
    return MBMD_OK;
}

mbmd_status mbmd_batch_capacity(const mbmd_ctx* c, int64_t* free_atoms, int* free_slots,
                                int64_t* largest_range)
{
    if (!c || !c->batch) return MBMD_EINVAL;
    const Batch& B = *c->batch;
    int64_t used = 0, largest = 0, at = 0;
    for (const Slot& s : B.slots) {
        used += s.n;
        largest = std::max<int64_t>(largest, s.atom_off - at);
        at = s.atom_off + s.n;
    }
    largest = std::max<int64_t>(largest, B.max_atoms - at);
    if (free_atoms) *free_atoms = B.max_atoms - used;
    if (free_slots) *free_slots = B.max_structs - (int)B.slots.size();
    if (largest_range) *largest_range = largest;
    return MBMD_OK;
}

mbmd_status mbmd_batch_add(mbmd_ctx* c, int64_t n, const double box[3], const double* pos,
                           const double* vel, double mass_amu, double dt_fs, int n_steps,
                           double* thermo, int* handle)
{
    if (!c || !handle) return MBMD_EINVAL;
    if (!c->batch) return fail(c, MBMD_EINVAL, "no serving batch is open%s");
    Batch& B = *c->batch;
    Box b{};
    mbmd_status s = common_checks(c, n, box, &b);
    if (s != MBMD_OK) return s;
    if (n < 1 || !pos || !vel) return fail(c, MBMD_EINVAL, "need n >= 1 and device pos, vel%s");
    if (!std::isfinite(mass_amu) || !(mass_amu > 0.0) || !std::isfinite(dt_fs) || n_steps < 0)
        return fail(c, MBMD_EINVAL, "need mass > 0, finite dt, n_steps >= 0%s");
    if ((int)B.slots.size() >= B.max_structs) return fail(c, MBMD_EBUSY, "no free structure slot%s");
    const int64_t at = find_range(B, n);
    if (at < 0) return fail(c, MBMD_EBUSY, "no free atom range of this size%s");
    Slot sl;
    // the lowest free status word (one exists: slots and words are as many)
    while (sl.sidx < B.max_structs && B.sidx_used[sl.sidx]) ++sl.sidx;
    if (sl.sidx >= B.max_structs) return fail(c, MBMD_EDEVICE, "no free status word%s");
    sl.handle = B.next_handle++;
    sl.atom_off = (int)at;
    sl.n = (int)n;
    sl.box = b;
    sl.nsteps = n_steps;
    sl.mass = mass_amu;
    sl.dt = dt_fs;
    sl.thermo = thermo;
    // positions into the buffer the next launch reads, velocities into the
    // batch state
    hipError_t e = launch_batch_admit(pos, vel, n, b, (int)at, c->buf.xw[0], c->buf.xw[1],
                                      c->buf.vel, c->buf.ostride, c->buf.status,
                                      c->buf.sstat + sl.sidx, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "batch add");
    B.sidx_used[sl.sidx] = 1;
    auto it = std::lower_bound(B.slots.begin(), B.slots.end(), (int)at,
                               [](const Slot& x, int off) { return x.atom_off < off; });
    B.slots.insert(it, sl);
    B.changed = true;
    *handle = sl.handle;
    return MBMD_OK;
}

mbmd_status mbmd_batch_step(mbmd_ctx* c, mbmd_precision prec, int* n_active)
{
    if (!c) return MBMD_EINVAL;
    if (!c->batch) return fail(c, MBMD_EINVAL, "no serving batch is open%s");
    if (prec != MBMD_FP64 && prec != MBMD_MIXED) return fail(c, MBMD_EINVAL, "bad precision%s");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    if (prec == MBMD_MIXED) return batch_step_impl<float>(c, n_active);
    return batch_step_impl<double>(c, n_active);
}

mbmd_status mbmd_batch_finished(const mbmd_ctx* c, int* handles, int capacity, int* count)
{
    if (!c || !c->batch || !count || capacity < 0 || (capacity > 0 && !handles))
        return MBMD_EINVAL;
    int k = 0;
    for (const Slot& s : c->batch->slots) {
        if (!s.done) continue;
        if (k < capacity) handles[k] = s.handle;
        ++k;
    }
    *count = k;
    return MBMD_OK;
}

mbmd_status mbmd_batch_retire(mbmd_ctx* c, int handle, double* pos, double* vel, double* U,
                              double* F, double* W, double* J, int32_t* status)
{
    if (!c) return MBMD_EINVAL;
    if (!c->batch) return fail(c, MBMD_EINVAL, "no serving batch is open%s");
    Batch& B = *c->batch;
    Slot* sl = find_slot(B, handle);
    if (!sl) return fail(c, MBMD_EINVAL, "unknown structure handle%s");
    if (!sl->done) return fail(c, MBMD_EBUSY, "structure has not finished%s");
    const Buffers& b = c->buf;
    hipError_t e = hipSetDevice(c->device);
    if (e == hipSuccess)
        e = launch_batch_copy_out(b.xw[sl->final_buf], b.vel, b.U, b.F, b.W, b.J, b.ostride,
                                  sl->atom_off, sl->n, pos, vel, U, F, W, J,
                                  b.sstat + sl->sidx, status, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "batch retire");
    // the status word can be reused at once too: a later admission clears it
    // on the stream after this copy-out has read it
    B.sidx_used[sl->sidx] = 0;
    // the range can be handed out at once: a later admission's copy-in is
    // ordered after this copy-out on the stream
    B.slots.erase(B.slots.begin() + (sl - B.slots.data()));
    B.changed = true;
    return MBMD_OK;
}

mbmd_status mbmd_sync(mbmd_ctx* c)
{
    if (!c) return MBMD_EINVAL;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    if (!c->ws) return MBMD_OK;   // nothing was ever enqueued
    return finish(c);
}

mbmd_status mbmd_batch_sync(mbmd_ctx* c)
{
    if (!c) return MBMD_EINVAL;
    if (!c->batch) return fail(c, MBMD_EINVAL, "no serving batch is open%s");
    return mbmd_sync(c);
}

}  // extern "C"
