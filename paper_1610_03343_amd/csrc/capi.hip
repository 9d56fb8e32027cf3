// C ABI of libmbmd (declared in include/mbmd.h): contexts, workspace, and the
// host-side step loop that sequences the neighbour build, the site-local
// partials pass and the pairwise-force pass on one HIP stream.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mbmd.h"
#include "mbmd_internal.h"

using namespace mbmd;

namespace {
// Kernel classes timed by the optional HIP-event profile.
enum ProfKind { P_STAGE, P_BUILD, P_PARTIALS, P_PARTIALS_OVF, P_GATHER, P_THERMO, P_KINDS };
const char* const kProfNames[P_KINDS] = {"stage_positions", "neighbor_build", "site_partials",
                                         "site_partials_overflow", "pair_gather", "thermo_fold"};
struct ProfRec {
    int kind;
    hipEvent_t a, b;
};
}  // namespace

struct mbmd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int potential = -1;          // 0 Tersoff, 1 SW
    TersoffParams tp{};
    SWParams sp{};
    double skin = 0.5;
    int max_nb = 0;              // 0: potential default
    int policy = MBMD_REBUILD_ON_SKIN;
    mbmd_run_stats stats{};
    void* ws = nullptr;          // workspace base
    size_t ws_bytes = 0;
    bool ws_owned = false;
    Buffers buf{};
    int max_nn = kMaxSlots;      // largest list count of the last build
    int fold_from = 0;           // first step whose thermo row is not folded yet
    int fold_to = 0;             // one past the last step with pending partials
    int64_t laid_n = -1;         // layout currently held by buf
    int laid_M = 0;
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
        if (c->profiling && hipEventCreate(&a) == hipSuccess) hipEventRecord(a, c->stream);
    }
    ~ProfScope()
    {
        if (!a) return;
        hipEvent_t b = nullptr;
        if (hipEventCreate(&b) == hipSuccess) {
            hipEventRecord(b, c->stream);
            c->prof_pending.push_back(ProfRec{kind, a, b});
        } else {
            hipEventDestroy(a);
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
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    c->prof_pending.clear();
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int64_t cell_cap(int64_t n) { return n * 4 > 64 ? n * 4 : 64; }

int resolved_M(const mbmd_ctx* c)
{
    if (c->max_nb > 0) return c->max_nb;
    return c->potential == 1 ? 32 : 16;
}

double cutoff_of(const mbmd_ctx* c)
{
    return c->potential == 1 ? c->sp.a * c->sp.sigma : c->tp.S;
}

// Lays out every device array for n atoms and M slots from `base` (or only
// sizes it when base is null); returns the total byte count.
size_t layout(int64_t n, int M, char* base, Buffers* b)
{
    const int64_t nn = n > 0 ? n : 1;
    const int64_t ncap = cell_cap(nn);
    const int64_t nscan = (ncap + kBlock * 4 - 1) / (kBlock * 4);
    const int64_t nblk = blocks_for(nn);
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off = align_up(off + bytes);
        return p;
    };
    Buffers t{};
    t.n = n;
    t.M = M;
    t.xw[0] = (double4*)take(sizeof(double4) * nn);
    t.xw[1] = (double4*)take(sizeof(double4) * nn);
    t.xbuild = (double4*)take(sizeof(double4) * nn);
    t.nn = (int*)take(sizeof(int) * nn);
    t.nl = (int*)take(sizeof(int) * nn * M);
    t.rev = (int*)take(sizeof(int) * nn * M);
    t.mask = (unsigned long long*)take(sizeof(unsigned long long) * nn);
    t.dpart = take(sizeof(double) * 3 * nn * M);
    t.cell_of = (int*)take(sizeof(int) * nn);
    t.cell_count = (int*)take(sizeof(int) * ncap);
    t.cell_start = (int*)take(sizeof(int) * (ncap + 1));
    t.cell_fill = (int*)take(sizeof(int) * (ncap + 1 + nscan));
    t.cell_atoms = (int*)take(sizeof(int) * nn);
    t.part_b = (double*)take(sizeof(double) * kPartialCols * nblk * kThermoRing);
    t.ovf_count = (int*)take(sizeof(int));
    t.ovf_list = (int*)take(sizeof(int) * nn);
    t.status = (unsigned*)take(sizeof(unsigned));
    t.thermo_scratch = (double*)take(sizeof(double) * kThermoCols);
    t.xsnap = (double4*)take(sizeof(double4) * nn);
    t.vsnap = (double*)take(sizeof(double) * 3 * nn);
    t.step_disp2 = (unsigned long long*)take(sizeof(unsigned long long) * kMaxChunk);
    t.maxnn = (int*)take(sizeof(int));
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

// Makes the workspace hold a layout for n atoms.
mbmd_status ensure_workspace(mbmd_ctx* c, int64_t n)
{
    const int M = resolved_M(c);
    const size_t need = layout(n, M, nullptr, nullptr);
    if (c->ws && !c->ws_owned) {
        if (c->ws_bytes < need)
            return fail(c, MBMD_ENOMEM, "bound workspace too small for this call%s");
    } else if (c->ws_bytes < need) {
        if (c->ws) hipFree(c->ws);
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
    if (c->laid_n != n || c->laid_M != M) {
        layout(n, M, (char*)c->ws, &c->buf);
        c->laid_n = n;
        c->laid_M = M;
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

CellGrid make_grid(const Box& box, double rlist, int64_t n)
{
    CellGrid g{};
    const int64_t cap = cell_cap(n > 0 ? n : 1);
    for (int a = 0; a < 3; ++a) {
        int k = (int)std::floor(box.L[a] / (rlist * (1.0 + 1e-9)));
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
    return g;
}

mbmd_status status_to_code(mbmd_ctx* c, unsigned st)
{
    if (st & ST_TYPES) return fail(c, MBMD_EINVAL, "atom type other than 0%s");
    if (st & ST_NONFINITE) return fail(c, MBMD_ENONFINITE, "non-finite position%s");
    if (st & ST_NEIGH_OVERFLOW)
        return fail(c, MBMD_ENEIGH, "neighbour list capacity exceeded; raise max_neighbors%s");
    if (st & ST_ASYMMETRIC) return fail(c, MBMD_EDEVICE, "internal: asymmetric neighbour data%s");
    return MBMD_OK;
}

// Reads the status word after draining the stream.
mbmd_status finish(mbmd_ctx* c)
{
    unsigned st = 0;
    hipError_t e = hipMemcpyAsync(&st, c->buf.status, sizeof st, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "stream synchronize");
    collect_profile(c);
    return status_to_code(c, st);
}

// Stages positions, clears status and overflow counters, builds the list.
mbmd_status begin(mbmd_ctx* c, int64_t n, const Box& box, const double* pos, const int32_t* types)
{
    mbmd_status s = ensure_workspace(c, n);
    if (s != MBMD_OK) return s;
    const Buffers& b = c->buf;
    hipError_t e = launch_fill_int((int*)b.status, 1, 0, c->stream);
    if (e == hipSuccess) e = launch_fill_int(b.ovf_count, 1, 0, c->stream);
    if (e == hipSuccess) {
        ProfScope ps(c, P_STAGE);
        e = launch_load_positions(pos, types, n, box, b.xw[0], b.status, c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "staging positions");
    return MBMD_OK;
}

// Builds the list and reads back its largest count (one stream sync per
// build), which decides whether the partials overflow pass is needed.
hipError_t build(mbmd_ctx* c, int cur, const Box& box)
{
    hipError_t e;
    {
        ProfScope ps(c, P_BUILD);
        const double rl = cutoff_of(c) + c->skin;
        e = launch_build_neighbors(c->buf, cur, box, make_grid(box, rl, c->buf.n), rl, c->stream);
    }
    int mx = kMaxSlots;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&mx, c->buf.maxnn, sizeof mx, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    c->max_nn = mx;
    return e;
}

template <class T>
hipError_t partials(mbmd_ctx* c, int cur, const Box& box, double* U)
{
    hipError_t e;
    for (int pass = 0; pass < 2; ++pass) {
        // the overflow pass only exists when a site can exceed the fast path
        if (pass == 1 && !(c->buf.M > kSiteFastBonds && c->max_nn > kSiteFastBonds)) break;
        ProfScope ps(c, pass ? P_PARTIALS_OVF : P_PARTIALS);
        if (c->potential == 1)
            e = launch_sw_partials<T>(c->buf, cur, box, c->sp, U, pass == 1, c->max_nn, c->stream);
        else
            e = launch_tersoff_partials<T>(c->buf, cur, box, c->tp, U, pass == 1, c->max_nn,
                                           c->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class T>
hipError_t gather(mbmd_ctx* c, const Box& box, const StepArgs& a, const double* U, double* vel,
                  double* F, double* W, double* J)
{
    ProfScope ps(c, P_GATHER);
    return launch_pair_gather<T>(c->buf, box, a, U, vel, F, W, J, c->stream);
}


template <class T>
mbmd_status compute_impl(mbmd_ctx* c, int64_t n, const Box& box, const double* pos,
                         const double* vel, const int32_t* types, double* U, double* F,
                         double* W, double* J)
{
    mbmd_status s = begin(c, n, box, pos, types);
    if (s != MBMD_OK) return s;
    hipError_t e = build(c, 0, box);
    if (e == hipSuccess) e = partials<T>(c, 0, box, U);
    StepArgs a{};
    a.cur = 0;
    if (e == hipSuccess) e = gather<T>(c, box, a, U, const_cast<double*>(vel), F, W, J);
    if (e != hipSuccess) return hip_fail(c, e, "compute launch");
    return finish(c);
}

// Folds the pending per-step partials into thermo rows.
hipError_t flush_thermo(mbmd_ctx* c, double* thermo)
{
    if (!thermo || c->fold_to <= c->fold_from) return hipSuccess;
    ProfScope ps(c, P_THERMO);
    hipError_t e = launch_thermo_fold(c->buf, c->fold_from, c->fold_to - c->fold_from, thermo,
                                      c->stream);
    c->fold_from = c->fold_to;
    return e;
}

// One MD step: force evaluation at the current positions, second half-kick,
// heat current and thermo row, then (unless last) first half-kick and drift.
template <class T>
hipError_t md_step(mbmd_ctx* c, const Box& box, StepArgs& a, int step, int n_steps, int cur,
                   bool check, unsigned long long* slot, double* U, double* vel, double* F,
                   double* W, double* J, double* thermo)
{
    hipError_t e = partials<T>(c, cur, box, U);
    a.cur = cur;
    a.kick_before = step > 0;
    a.advance = step < n_steps;
    a.check_skin = a.advance && check;
    a.disp_slot = slot;
    a.part_row = thermo ? c->buf.part_b + (size_t)(step % kThermoRing) * blocks_for(c->buf.n) *
                                              kPartialCols
                        : nullptr;
    if (e == hipSuccess) e = gather<T>(c, box, a, U, vel, F, W, J);
    if (e == hipSuccess && thermo) {
        if (step < c->fold_from || step > c->fold_to) c->fold_from = step;   // replayed steps
        c->fold_to = step + 1;
        if (c->fold_to - c->fold_from == kThermoRing) e = flush_thermo(c, thermo);
    }
    return e;
}

template <class T>
mbmd_status nve_impl(mbmd_ctx* c, int64_t n, const Box& box, double mass, double* pos,
                     double* vel, const int32_t* types, double dt, int n_steps, int every,
                     double* U, double* F, double* W, double* J, double* thermo)
{
    mbmd_status s = begin(c, n, box, pos, types);
    if (s != MBMD_OK) return s;
    const Buffers& b = c->buf;
    const double kappa = 9.64853321567e-3;   // eV/(A amu) in A/fs^2
    StepArgs a{};
    a.half_dt_acc = 0.5 * dt * kappa / mass;
    a.dt = dt;
    a.skin_half2 = 0.25 * c->skin * c->skin;
    a.kin_scale = 0.5 * mass / kappa;
    mbmd_run_stats st{};
    st.steps = n_steps;
    c->fold_from = c->fold_to = 0;
    int cur = 0, last_build = 0;
    hipError_t e = build(c, cur, box);
    st.rebuilds = 1;

    if (c->policy == MBMD_REBUILD_FIXED) {
        // The list is rebuilt every `every` steps whatever the atoms do; no
        // displacement is tracked (the statistics report -1).
        for (int step = 0; step <= n_steps && e == hipSuccess; ++step) {
            if (step - last_build == every) {
                e = build(c, cur, box);
                last_build = step;
                ++st.rebuilds;
            }
            if (e != hipSuccess) break;
            e = md_step<T>(c, box, a, step, n_steps, cur, false, nullptr, U, vel, F, W, J, thermo);
            if (step < n_steps) cur ^= 1;
        }
        if (e == hipSuccess) e = flush_thermo(c, thermo);
        if (e == hipSuccess) e = launch_store_positions(b.xw[cur], n, pos, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "nve launch");
        s = finish(c);
        st.max_displacement = -1.0;
        c->stats = st;
        return s;
    }

    // Rebuild on skin: chunks of steps are enqueued from a snapshot of the
    // state; after each chunk the per-step largest displacement is read
    // back.  If the positions of some step moved more than skin/2 from the
    // last build, the chunk is replayed from the snapshot (bit-identically)
    // up to that step and the list is rebuilt there.
    int step = 0;
    int chunk = every < kMaxChunk ? every : kMaxChunk;
    std::vector<unsigned long long> disp(kMaxChunk);
    double committed_max2 = 0.0;
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
            const bool check = (sk + 1 - last_build) != every;
            e = md_step<T>(c, box, a, sk, n_steps, cur, check, b.step_disp2 + k, U, vel, F, W, J,
                           thermo);
            if (sk < n_steps) cur ^= 1;
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
            if (d2 > a.skin_half2) {
                bad = cs + k + 1;
                break;
            }
            if (d2 > committed_max2) committed_max2 = d2;
        }
        if (bad < 0) {
            step = cend;
            if (step <= n_steps && step - last_build == every) {
                e = build(c, cur, box);
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
        for (int sk = cs; sk < bad && e == hipSuccess; ++sk) {
            e = md_step<T>(c, box, a, sk, n_steps, cur, false, nullptr, U, vel, F, W, J, thermo);
            if (sk < n_steps) cur ^= 1;
        }
        if (e == hipSuccess) e = build(c, cur, box);
        last_build = bad;
        step = bad;
        ++st.rebuilds;
        ++st.rollbacks;
        chunk = bad - cs > 0 ? bad - cs : 1;
    }
    if (e == hipSuccess) e = flush_thermo(c, thermo);
    if (e == hipSuccess) e = launch_store_positions(b.xw[cur], n, pos, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "nve launch");
    s = finish(c);
    st.max_displacement = std::sqrt(committed_max2);
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
    *out = c;
    return MBMD_OK;
}

void mbmd_destroy(mbmd_ctx* c)
{
    if (!c) return;
    for (const ProfRec& r : c->prof_pending) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    if (c->ws && c->ws_owned) {
        hipSetDevice(c->device);
        hipFree(c->ws);
    }
    delete c;
}

const char* mbmd_last_error(const mbmd_ctx* c) { return c ? c->err.c_str() : "null context"; }

mbmd_status mbmd_set_tersoff(mbmd_ctx* c, const mbmd_tersoff_params* p)
{
    if (!c || !p) return MBMD_EINVAL;
    const double v[] = {p->A, p->B, p->lambda, p->mu, p->beta, p->n, p->c, p->d, p->h, p->R, p->S};
    for (double x : v)
        if (!std::isfinite(x)) return fail(c, MBMD_EINVAL, "non-finite Tersoff parameter%s");
    if (!(p->R > 0.0) || !(p->S > p->R) || !(p->n > 0.0) || !(p->beta > 0.0) || p->d == 0.0)
        return fail(c, MBMD_EINVAL, "Tersoff parameters need 0 < R < S, n > 0, beta > 0, d != 0%s");
    c->tp = TersoffParams{p->A, p->B, p->lambda, p->mu, p->beta, p->n, p->c, p->d, p->h, p->R, p->S};
    c->potential = 0;
    c->laid_n = -1;
    return MBMD_OK;
}

mbmd_status mbmd_set_sw(mbmd_ctx* c, const mbmd_sw_params* p)
{
    if (!c || !p) return MBMD_EINVAL;
    const double v[] = {p->epsilon, p->sigma, p->a, p->lambda, p->gamma, p->A, p->B, p->p, p->q};
    for (double x : v)
        if (!std::isfinite(x)) return fail(c, MBMD_EINVAL, "non-finite SW parameter%s");
    if (!(p->sigma > 0.0) || !(p->a > 0.0))
        return fail(c, MBMD_EINVAL, "SW parameters need sigma > 0 and a > 0%s");
    c->sp = SWParams{p->epsilon, p->sigma, p->a, p->lambda, p->gamma, p->A, p->B, p->p, p->q};
    c->potential = 1;
    c->laid_n = -1;
    return MBMD_OK;
}

mbmd_status mbmd_set_neighbor(mbmd_ctx* c, double skin, int max_neighbors)
{
    if (!c) return MBMD_EINVAL;
    if (!std::isfinite(skin) || skin < 0.0) return fail(c, MBMD_EINVAL, "skin must be >= 0%s");
    if (max_neighbors < 0 || max_neighbors > kMaxSlots)
        return fail(c, MBMD_EINVAL, "max_neighbors must be in 0..64%s");
    c->skin = skin;
    c->max_nb = max_neighbors;
    c->laid_n = -1;
    return MBMD_OK;
}

mbmd_status mbmd_set_rebuild_policy(mbmd_ctx* c, mbmd_rebuild_policy policy)
{
    if (!c) return MBMD_EINVAL;
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
    *bytes = layout(n_atoms, resolved_M(c), nullptr, nullptr);
    return MBMD_OK;
}

mbmd_status mbmd_bind_workspace(mbmd_ctx* c, void* dev_ptr, size_t bytes)
{
    if (!c) return MBMD_EINVAL;
    if (dev_ptr && ((uintptr_t)dev_ptr % kAlign) != 0)
        return fail(c, MBMD_EINVAL, "workspace must be 256-byte aligned%s");
    if (c->ws && c->ws_owned) {
        hipSetDevice(c->device);
        hipFree(c->ws);
    }
    c->ws = dev_ptr;
    c->ws_bytes = dev_ptr ? bytes : 0;
    c->ws_owned = false;
    c->laid_n = -1;
    return MBMD_OK;
}

mbmd_status mbmd_neighbors(mbmd_ctx* c, int64_t n, const double box[3], const double* pos,
                           int32_t* nn, int32_t* nl)
{
    if (!c) return MBMD_EINVAL;
    Box b{};
    mbmd_status s = common_checks(c, n, box, &b);
    if (s != MBMD_OK) return s;
    if (n == 0) return MBMD_OK;
    if (!pos || !nn || !nl) return fail(c, MBMD_EINVAL, "null device pointer%s");
    s = begin(c, n, b, pos, nullptr);
    if (s != MBMD_OK) return s;
    hipError_t e = build(c, 0, b);
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
    if (!std::isfinite(mass_amu) || !(mass_amu > 0.0) || !std::isfinite(dt_fs) || n_steps < 0 ||
        rebuild_every < 1)
        return fail(c, MBMD_EINVAL, "need mass > 0, finite dt, n_steps >= 0, rebuild_every >= 1%s");
    if (n == 0) return MBMD_OK;
    if (!pos || !vel || !U || !F || !W || !J) return fail(c, MBMD_EINVAL, "null device pointer%s");
    if (prec == MBMD_MIXED)
        return nve_impl<float>(c, n, b, mass_amu, pos, vel, types, dt_fs, n_steps, rebuild_every,
                               U, F, W, J, thermo);
    return nve_impl<double>(c, n, b, mass_amu, pos, vel, types, dt_fs, n_steps, rebuild_every, U,
                            F, W, J, thermo);
}

}  // extern "C"
