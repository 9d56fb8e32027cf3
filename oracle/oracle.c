/*
 * CPU FP64 oracle for the many-body force path (Fan, Chen, Vierimaa, Harju,
 * "Efficient molecular dynamics simulations with many-body potentials on
 * graphics processing units").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * HIP path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the HIP library.  Build: gcc -O2 -ffp-contract=off
 * (no fused multiply-add, no fast-math), see build.py beside this file.
 *
 * What it computes, in the paper's order:
 *   - neighbour lists (Section 2.1, the cutoff-function paragraph): every
 *     j != i with minimum-image |r_j - r_i|^2 < r_list^2, ascending index;
 *     a brute-force O(N^2) definition and a linked-cell version;
 *   - the Tersoff energy (Section 2.1, Eqs. for U, U_ij, b_ij, zeta_ij, g_ijk,
 *     cos theta_ijk) and forces by the conventional three-loop scatter of
 *     Algorithm 1 with the force terms F^(ij)_i, F^(ij)_j, F^(ijk)_{i,j,k}
 *     (Section 2.2);
 *   - a capture of every force the iteration over atom i scatters: all of
 *     them are minus gradients of U_i, so the capture yields dU_i/dr_j for
 *     each neighbour j, from which the paper's pairwise quantities follow:
 *     F_ij = dU_i/dr_ij - dU_j/dr_ji (Section 2.3), the per-atom virial
 *     W_i = -1/2 sum_j r_ij (x) F_ij and the per-atom heat current
 *     J_i = sum_j r_ij (dU_j/dr_ji . v_i) (Section 2.3 and Section 2.4);
 *   - the LAMMPS-form per-atom virial of Algorithm 1 and the stress-based
 *     heat current J_i = W_i . v_i (Section 2.3), kept for comparison only;
 *   - the Stillinger-Weber energy with the same scatter-and-capture scheme
 *     (the paper names SW in Section 2.4 but prints no formula; the form is
 *     the 1985 one: two-body phi_2 split half/half, three-body h_ijk assigned
 *     wholly to its vertex atom i);
 *   - velocity-Verlet NVE integration (Section 3);
 *   - velocity-Verlet in the NPT ensemble with the Berendsen weak-coupling
 *     thermostat and barostat, the ensemble of the paper's benchmarks
 *     (Section 3; the paper names it without formulas: the scaling factors
 *     are Berendsen's, applied after each step's second half-kick).
 *
 * Readings where the paper is silent:
 *   - f_C, f_R, f_A are Tersoff's 1989 forms: f_R = A exp(-lambda r),
 *     f_A = B exp(-mu r), f_C = 1 (r < R), 1/2 + 1/2 cos(pi (r-R)/(S-R))
 *     (R <= r < S), 0 (r >= S);
 *   - g is evaluated in the algebraically identical cancellation-free form
 *     g = 1 + c^2 t^2 / (d^2 (d^2 + t^2)), t = h - cos theta;
 *   - db/dzeta is defined as 0 at zeta = 0 (it multiplies a zero gradient
 *     there);
 *   - minimum image d <- d - L rint(d / L), boxes with L >= 2 r_list.
 *
 * Layout: every array here is row-major per atom, positions pos[i*3 + a],
 * lists nl[i*maxnb + m], virials w[i*9 + 3*alpha + beta].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_OK 0
#define ORA_EINVAL 1
#define ORA_ENEIGH 2
#define ORA_EBOX 3
#define ORA_ENOMEM 4

typedef struct { double A, B, lam, mu, beta, n, c, d, h, R, S; } ora_tersoff_t;
typedef struct { double epsilon, sigma, a, lam, gamma, A, B, p, q; } ora_sw_t;

static const double ORA_PI = 3.14159265358979323846;

/* ------------------------------------------------------------- threads
 * The timing baseline on all host cores runs the loops over atoms i with
 * OpenMP.  The conventional scatter writes forces (and the LAMMPS-form
 * virial) of neighbours, so each thread scatters into its own buffer and
 * the buffers are summed in thread order afterwards: a fixed order for a
 * given thread count.  Per-atom energies, captured partials and everything
 * formed from them are written by atom i's own iteration only and do not
 * depend on the thread count.  With one thread (the default) every loop
 * runs serially on the output arrays, operation for operation as written. */
static int g_threads = 1;

void ora_set_threads(int t) { g_threads = t < 1 ? 1 : t; }

int ora_threads(void)
{
#ifdef _OPENMP
    return g_threads;
#else
    return 1;
#endif
}

static int thread_id(void)
{
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

/* dst[x] = sum over threads t = 0..T-1 of buf[t][x], in that order (the
 * entries x are independent, so they are split over the threads too). */
static void reduce_threads(double *dst, const double *buf, int T, size_t len)
{
#pragma omp parallel for num_threads(T) schedule(static)
    for (size_t x = 0; x < len; ++x) {
        double acc = 0.0;
        for (int t = 0; t < T; ++t) acc += buf[(size_t)t * len + x];
        dst[x] = acc;
    }
}

/* ---------------------------------------------------------------- geometry */

static double wrap1(double x, double L)
{
    double r = x - L * floor(x / L);
    if (r < 0.0) r += L;
    if (r >= L) r -= L;
    if (r < 0.0 || r >= L) r = 0.0;
    return r;
}

/* r_ij = r_j - r_i under the minimum-image convention. */
static void min_image(const double *box, const double *ri, const double *rj, double *d)
{
    for (int a = 0; a < 3; ++a) {
        double x = rj[a] - ri[a];
        x = x - box[a] * rint(x / box[a]);
        d[a] = x;
    }
}

static double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static int check_box(const double *box, double rlist)
{
    for (int a = 0; a < 3; ++a)
        if (!(box[a] >= 2.0 * rlist) || !isfinite(box[a])) return ORA_EBOX;
    return ORA_OK;
}

void ora_wrap(long n, const double *box, double *pos)
{
    for (long i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) pos[i * 3 + a] = wrap1(pos[i * 3 + a], box[a]);
}

static void sort_ints(int *v, int n)
{
    for (int a = 1; a < n; ++a) {
        int key = v[a], b = a - 1;
        while (b >= 0 && v[b] > key) { v[b + 1] = v[b]; --b; }
        v[b + 1] = key;
    }
}

/* Neighbour list by definition: all pairs, O(N^2).  Returns ORA_ENEIGH when
 * some atom has more than maxnb neighbours (nn[] then holds the true counts,
 * the stored entries are the first maxnb in ascending order). */
int ora_neighbors_brute(long n, const double *box, const double *pos, double rlist,
                        int maxnb, int *nn, int *nl)
{
    int st = check_box(box, rlist);
    if (st) return st;
    double rl2 = rlist * rlist;
    int overflow = 0;
    for (long i = 0; i < n; ++i) {
        int cnt = 0;
        for (long j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(box, &pos[i * 3], &pos[j * 3], d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < rl2) {
                if (cnt < maxnb) nl[i * maxnb + cnt] = (int)j;
                ++cnt;
            }
        }
        nn[i] = cnt;
        if (cnt > maxnb) overflow = 1;
    }
    return overflow ? ORA_ENEIGH : ORA_OK;
}

/* Neighbour list by definition with a radius per pair of atom types (the
 * multi-element Tersoff form, whose cutoff depends on the pair): atom j is
 * listed for atom i iff r_ij^2 < rpair[t_i * nt + t_j]^2.  All pairs,
 * O(N^2); overflow as in ora_neighbors_brute. */
int ora_neighbors_brute_typed(long n, const double *box, const double *pos, const int *types,
                              int nt, const double *rpair, int maxnb, int *nn, int *nl)
{
    if (nt < 1) return ORA_EINVAL;
    double rmax = 0.0;
    for (int k = 0; k < nt * nt; ++k) {
        if (!(rpair[k] > 0.0)) return ORA_EINVAL;
        if (rpair[k] > rmax) rmax = rpair[k];
    }
    for (long i = 0; i < n; ++i)
        if (types[i] < 0 || types[i] >= nt) return ORA_EINVAL;
    int st = check_box(box, rmax);
    if (st) return st;
    int overflow = 0;
    for (long i = 0; i < n; ++i) {
        int cnt = 0;
        for (long j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            min_image(box, &pos[i * 3], &pos[j * 3], d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            const double rl = rpair[types[i] * nt + types[j]];
            if (r2 < rl * rl) {
                if (cnt < maxnb) nl[i * maxnb + cnt] = (int)j;
                ++cnt;
            }
        }
        nn[i] = cnt;
        if (cnt > maxnb) overflow = 1;
    }
    return overflow ? ORA_ENEIGH : ORA_OK;
}

/* Neighbour list through a linked cell list (cells of side >= r_list). */
int ora_neighbors_cells(long n, const double *box, const double *pos, double rlist,
                        int maxnb, int *nn, int *nl)
{
    int st = check_box(box, rlist);
    if (st) return st;
    int nc[3];
    for (int a = 0; a < 3; ++a) {
        /* a small margin keeps the cell side above r_list after rounding */
        nc[a] = (int)floor(box[a] / (rlist * (1.0 + 1e-9)));
        if (nc[a] < 1) nc[a] = 1;
    }
    long ncell = (long)nc[0] * nc[1] * nc[2];
    long *head = (long *)malloc(sizeof(long) * (size_t)ncell);
    long *next = (long *)malloc(sizeof(long) * (size_t)(n > 0 ? n : 1));
    int *cand = (int *)malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!head || !next || !cand) { free(head); free(next); free(cand); return ORA_ENOMEM; }
    for (long c = 0; c < ncell; ++c) head[c] = -1;
    int *cell_of = (int *)malloc(sizeof(int) * 3 * (size_t)(n > 0 ? n : 1));
    if (!cell_of) { free(head); free(next); free(cand); return ORA_ENOMEM; }
    for (long i = n - 1; i >= 0; --i) {
        long c = 0;
        for (int a = 2; a >= 0; --a) {
            double x = wrap1(pos[i * 3 + a], box[a]);
            int ci = (int)floor(x / (box[a] / nc[a]));
            if (ci < 0) ci = 0;
            if (ci >= nc[a]) ci = nc[a] - 1;
            cell_of[i * 3 + a] = ci;
            c = c * nc[a] + ci;
        }
        next[i] = head[c];
        head[c] = i;
    }
    double rl2 = rlist * rlist;
    int overflow = 0;
    const int T = ora_threads();
    int *cand_all = T > 1 ? (int *)malloc(sizeof(int) * (size_t)T * (size_t)(n > 0 ? n : 1)) : cand;
    if (!cand_all) { free(head); free(next); free(cand); free(cell_of); return ORA_ENOMEM; }
#pragma omp parallel for num_threads(T) schedule(static) reduction(| : overflow) if (T > 1)
    for (long i = 0; i < n; ++i) {
        int *cand = cand_all + (size_t)thread_id() * (size_t)(n > 0 ? n : 1);
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            if (nc[a] >= 3) { lo[a] = -1; hi[a] = 1; }
            else if (nc[a] == 2) { lo[a] = 0; hi[a] = 1; }
            else { lo[a] = 0; hi[a] = 0; }
        }
        int ncand = 0;
        for (int oz = lo[2]; oz <= hi[2]; ++oz)
            for (int oy = lo[1]; oy <= hi[1]; ++oy)
                for (int ox = lo[0]; ox <= hi[0]; ++ox) {
                    int cx = (cell_of[i * 3 + 0] + ox + nc[0]) % nc[0];
                    int cy = (cell_of[i * 3 + 1] + oy + nc[1]) % nc[1];
                    int cz = (cell_of[i * 3 + 2] + oz + nc[2]) % nc[2];
                    long c = ((long)cz * nc[1] + cy) * nc[0] + cx;
                    for (long j = head[c]; j >= 0; j = next[j]) {
                        if (j == i) continue;
                        double d[3];
                        min_image(box, &pos[i * 3], &pos[j * 3], d);
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (r2 < rl2) cand[ncand++] = (int)j;
                    }
                }
        sort_ints(cand, ncand);
        for (int m = 0; m < ncand && m < maxnb; ++m) nl[i * maxnb + m] = cand[m];
        nn[i] = ncand;
        if (ncand > maxnb) overflow = 1;
    }
    if (cand_all != cand) free(cand_all);
    free(head); free(next); free(cand); free(cell_of);
    return overflow ? ORA_ENEIGH : ORA_OK;
}

/* ------------------------------------------------- Tersoff scalar functions */

static double t_fc(const ora_tersoff_t *p, double r)
{
    if (r < p->R) return 1.0;
    if (r >= p->S) return 0.0;
    return 0.5 + 0.5 * cos(ORA_PI * (r - p->R) / (p->S - p->R));
}

static double t_dfc(const ora_tersoff_t *p, double r)
{
    if (r < p->R || r >= p->S) return 0.0;
    return -0.5 * ORA_PI / (p->S - p->R) * sin(ORA_PI * (r - p->R) / (p->S - p->R));
}

static double t_fr(const ora_tersoff_t *p, double r) { return p->A * exp(-p->lam * r); }
static double t_dfr(const ora_tersoff_t *p, double r) { return -p->lam * p->A * exp(-p->lam * r); }
static double t_fa(const ora_tersoff_t *p, double r) { return p->B * exp(-p->mu * r); }
static double t_dfa(const ora_tersoff_t *p, double r) { return -p->mu * p->B * exp(-p->mu * r); }

/* g(cos theta) = 1 + c^2/d^2 - c^2/(d^2 + (h - cos theta)^2), written without
 * the cancellation of the two large terms. */
static double t_g(const ora_tersoff_t *p, double cs)
{
    double t = p->h - cs;
    double c2 = p->c * p->c, d2 = p->d * p->d;
    return 1.0 + c2 * t * t / (d2 * (d2 + t * t));
}

static double t_dg(const ora_tersoff_t *p, double cs)
{
    double t = p->h - cs;
    double c2 = p->c * p->c, d2 = p->d * p->d;
    double q = d2 + t * t;
    return -2.0 * c2 * t / (q * q);
}

/* Public for the tests: the literal printed form of g. */
double ora_tersoff_g_literal(const ora_tersoff_t *p, double cs)
{
    double t = p->h - cs;
    double c2 = p->c * p->c, d2 = p->d * p->d;
    return 1.0 + c2 / d2 - c2 / (d2 + t * t);
}

double ora_tersoff_g(const ora_tersoff_t *p, double cs) { return t_g(p, cs); }

static double t_b(const ora_tersoff_t *p, double zeta)
{
    if (zeta <= 0.0) return 1.0;
    return pow(1.0 + pow(p->beta * zeta, p->n), -1.0 / (2.0 * p->n));
}

static double t_db(const ora_tersoff_t *p, double zeta)
{
    if (zeta <= 0.0) return 0.0;
    double u = pow(p->beta * zeta, p->n);
    double b = pow(1.0 + u, -1.0 / (2.0 * p->n));
    return -b * u / (2.0 * zeta * (1.0 + u));
}

double ora_tersoff_b(const ora_tersoff_t *p, double zeta) { return t_b(p, zeta); }
double ora_tersoff_db(const ora_tersoff_t *p, double zeta) { return t_db(p, zeta); }

/* Gradients of f_C(r_ik) g(cos theta_ijk) with respect to the absolute
 * positions r_i, r_j and r_k (used by F^(ijk)_{i,j,k}). */
static void t_grad_fcg(const ora_tersoff_t *p, const double *rij, double r_ij,
                       const double *rik, double r_ik,
                       double *gi, double *gj, double *gk)
{
    double cs = dot3(rij, rik) / (r_ij * r_ik);
    double fc = t_fc(p, r_ik), dfc = t_dfc(p, r_ik);
    double g = t_g(p, cs), dg = t_dg(p, cs);
    for (int a = 0; a < 3; ++a) {
        double uij = rij[a] / r_ij, uik = rik[a] / r_ik;
        double dcos_j = (uik - cs * uij) / r_ij;   /* d cos / d r_j */
        double dcos_k = (uij - cs * uik) / r_ik;   /* d cos / d r_k */
        double dcos_i = -(dcos_j + dcos_k);        /* d cos / d r_i */
        gj[a] = fc * dg * dcos_j;
        gk[a] = dfc * uik * g + fc * dg * dcos_k;
        gi[a] = -dfc * uik * g + fc * dg * dcos_i;
    }
}

static int find_slot(const int *nn, const int *nl, int maxnb, long j, long i)
{
    int cnt = nn[j] < maxnb ? nn[j] : maxnb;
    for (int s = 0; s < cnt; ++s)
        if (nl[j * maxnb + s] == (int)i) return s;
    return -1;
}

/* Pairwise post-pass shared by both potentials: from the captured
 * G[i][m] = dU_i/dr_{NL_im} build F_ij, W_i, J_i and sum_j F_ij. */
static int pairwise_post(long n, const double *box, const double *pos, const double *vel,
                         const int *nn, const int *nl, int maxnb, const double *G,
                         double *W, double *J, double *Fpair)
{
    int bad = 0;
    const int T = ora_threads();
#pragma omp parallel for num_threads(T) schedule(static) reduction(| : bad) if (T > 1)
    for (long i = 0; i < n; ++i) {
        double w[9] = {0}, jj[3] = {0}, fp[3] = {0};
        int cnt = nn[i];
        for (int m = 0; m < cnt; ++m) {
            long j = nl[i * maxnb + m];
            int s = find_slot(nn, nl, maxnb, j, i);
            if (s < 0) { bad = 1; break; }         /* lists must be symmetric */
            const double *dij = &G[((size_t)i * maxnb + m) * 3];
            const double *dji = &G[((size_t)j * maxnb + s) * 3];
            double rij[3];
            min_image(box, &pos[i * 3], &pos[j * 3], rij);
            double fij[3];
            for (int a = 0; a < 3; ++a) fij[a] = dij[a] - dji[a];
            for (int a = 0; a < 3; ++a) fp[a] += fij[a];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) w[3 * a + b] -= 0.5 * rij[a] * fij[b];
            if (vel) {
                double proj = dot3(dji, &vel[i * 3]);
                for (int a = 0; a < 3; ++a) jj[a] += rij[a] * proj;
            }
        }
        if (W) memcpy(&W[i * 9], w, sizeof w);
        if (J) memcpy(&J[i * 3], jj, sizeof jj);
        if (Fpair) memcpy(&Fpair[i * 3], fp, sizeof fp);
    }
    return bad ? ORA_EINVAL : ORA_OK;
}

static void stress_current(long n, const double *WL, const double *vel, double *JL)
{
    for (long i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            double s = 0.0;
            for (int b = 0; b < 3; ++b) s += WL[i * 9 + 3 * a + b] * (vel ? vel[i * 3 + b] : 0.0);
            JL[i * 3 + a] = s;
        }
}

/* Tersoff, conventional Algorithm 1 with capture, for nt atom types.
 * P[ti*nt + tj] holds the parameters of the ordered pair (i, j): A, B, lambda,
 * mu, R, S of the pair (bond i-j terms, and f_C(r_ik) when used as the pair
 * (i, k)) and beta, n, c, d, h of the centre atom i; chi[ti*nt + tj] (or NULL:
 * 1) multiplies b_ij.  types == NULL means every atom is type 0.
 * In:  pos[n*3] (wrapped), vel[n*3] or NULL, nn[n], nl[n*maxnb] (symmetric,
 *      ascending).
 * Out: U[n], F[n*3] (scatter), W[n*9], J[n*3] (pairwise, the paper's), and
 *      optionally Fpair[n*3] = sum_j F_ij, WL[n*9] (LAMMPS form), JL[n*3]
 *      (stress-based), G[n*maxnb*3] = dU_i/dr_{NL_im}.  NULL skips an output. */
static int tersoff_core(long n, const double *box, const double *pos, const double *vel,
                        const int *types, int nt, const ora_tersoff_t *P, const double *chi,
                        const int *nn, const int *nl, int maxnb,
                        double *U, double *F, double *W, double *J,
                        double *Fpair, double *WL, double *JL, double *Gout)
{
    for (long i = 0; i < n; ++i)
        if (nn[i] > maxnb) return ORA_ENEIGH;
    size_t gsz = (size_t)(n > 0 ? n : 1) * maxnb * 3;
    double *G = Gout ? Gout : (double *)malloc(sizeof(double) * gsz);
    double *wl = (double *)calloc((size_t)(n > 0 ? n : 1) * 9, sizeof(double));
    if (!G || !wl) { if (!Gout) free(G); free(wl); return ORA_ENOMEM; }
    memset(G, 0, sizeof(double) * gsz);
    for (long i = 0; i < n; ++i) {          /* Algorithm 1, lines 1-3 */
        U[i] = 0.0;
        F[i * 3 + 0] = F[i * 3 + 1] = F[i * 3 + 2] = 0.0;
    }
    const int T = ora_threads();
    const size_t nf = (size_t)(n > 0 ? n : 1) * 3, nw = (size_t)(n > 0 ? n : 1) * 9;
    double *Fbuf = T > 1 ? (double *)malloc(sizeof(double) * (size_t)T * nf) : NULL;
    double *wbuf = T > 1 ? (double *)malloc(sizeof(double) * (size_t)T * nw) : NULL;
    if (T > 1 && (!Fbuf || !wbuf)) {
        free(Fbuf); free(wbuf);
        if (!Gout) free(G);
        free(wl);
        return ORA_ENOMEM;
    }
#pragma omp parallel num_threads(T) if (T > 1)
    {
    double *const F_out = F, *const wl_out = wl;
    double *F = T > 1 ? Fbuf + (size_t)thread_id() * nf : F_out;     /* this thread's scatter */
    double *wl = T > 1 ? wbuf + (size_t)thread_id() * nw : wl_out;
    if (T > 1) {                       /* each thread clears its own buffers */
        memset(F, 0, sizeof(double) * nf);
        memset(wl, 0, sizeof(double) * nw);
    }
#pragma omp for schedule(static)
    for (long i = 0; i < n; ++i) {
        int cnt = nn[i];
        const int ti = types ? types[i] : 0;
        for (int m = 0; m < cnt; ++m) {
            long j = nl[i * maxnb + m];
            const int tj = types ? types[j] : 0;
            const ora_tersoff_t *p = &P[ti * nt + tj];
            double rij[3];
            min_image(box, &pos[i * 3], &pos[j * 3], rij);
            double r = sqrt(dot3(rij, rij));
            if (r >= p->S) continue;          /* f_C(r_ij) = 0: no contribution */
            /* zeta_ij and the bond order, recomputed here: the conventional
             * method has no precompute. */
            double zeta = 0.0;
            for (int q = 0; q < cnt; ++q) {
                if (q == m) continue;
                long k = nl[i * maxnb + q];
                const ora_tersoff_t *pk = &P[ti * nt + (types ? types[k] : 0)];
                double rik[3];
                min_image(box, &pos[i * 3], &pos[k * 3], rik);
                double rk = sqrt(dot3(rik, rik));
                if (rk >= pk->S) continue;
                double cs = dot3(rij, rik) / (r * rk);
                zeta += t_fc(pk, rk) * t_g(pk, cs);
            }
            double b = t_b(p, zeta), db = t_db(p, zeta);
            if (chi) {
                b *= chi[ti * nt + tj];
                db *= chi[ti * nt + tj];
            }
            double fc = t_fc(p, r), dfc = t_dfc(p, r);
            double fr = t_fr(p, r), dfr = t_dfr(p, r);
            double fa = t_fa(p, r), dfa = t_dfa(p, r);
            U[i] += 0.5 * fc * (fr - b * fa);                       /* line 7 */
            /* F^(ij)_i and F^(ij)_j: d/dr_j f(r_ij) = f' u_ij, d/dr_i = -f' u_ij */
            double d_fcfr = dfc * fr + fc * dfr, d_fcfa = dfc * fa + fc * dfa;
            double fij_i[3], fij_j[3];
            for (int a = 0; a < 3; ++a) {
                double u = rij[a] / r;
                fij_i[a] = -0.5 * d_fcfr * (-u) + 0.5 * b * d_fcfa * (-u);
                fij_j[a] = -0.5 * d_fcfr * u + 0.5 * b * d_fcfa * u;
            }
            for (int a = 0; a < 3; ++a) {
                F[i * 3 + a] += fij_i[a];                          /* line 8 */
                F[j * 3 + a] += fij_j[a];                          /* line 9 */
                G[((size_t)i * maxnb + m) * 3 + a] -= fij_j[a];
            }
            /* Line 10 credits atom i with half the two-body virial of this
             * term; the other half goes to j, as LAMMPS's per-atom tally does,
             * so that the LAMMPS-form per-atom virials sum to the total. */
            for (int a = 0; a < 3; ++a)
                for (int bb = 0; bb < 3; ++bb) {
                    wl[i * 9 + 3 * a + bb] -= 0.5 * rij[a] * fij_i[bb];
                    wl[j * 9 + 3 * a + bb] -= 0.5 * rij[a] * fij_i[bb];
                }
            double pref = 0.5 * fc * fa * db;
            for (int q = 0; q < cnt; ++q) {                        /* lines 11-25 */
                if (q == m) continue;
                long k = nl[i * maxnb + q];
                const ora_tersoff_t *pk = &P[ti * nt + (types ? types[k] : 0)];
                double rik[3];
                min_image(box, &pos[i * 3], &pos[k * 3], rik);
                double rk = sqrt(dot3(rik, rik));
                if (rk >= pk->S) continue;
                double gi[3], gj[3], gk[3];
                t_grad_fcg(pk, rij, r, rik, rk, gi, gj, gk);
                double fi[3], fj[3], fk[3];
                for (int a = 0; a < 3; ++a) {
                    fi[a] = pref * gi[a];
                    fj[a] = pref * gj[a];
                    fk[a] = pref * gk[a];
                }
                for (int a = 0; a < 3; ++a) {
                    F[i * 3 + a] += fi[a];
                    F[j * 3 + a] += fj[a];
                    F[k * 3 + a] += fk[a];
                    G[((size_t)i * maxnb + m) * 3 + a] -= fj[a];
                    G[((size_t)i * maxnb + q) * 3 + a] -= fk[a];
                }
                for (int a = 0; a < 3; ++a)
                    for (int bb = 0; bb < 3; ++bb) {
                        double w = (rij[a] * fj[bb] + rik[a] * fk[bb]) / 3.0;
                        wl[i * 9 + 3 * a + bb] += w;
                        wl[j * 9 + 3 * a + bb] += w;
                        wl[k * 9 + 3 * a + bb] += w;
                    }
            }
        }
    }
    (void)F_out; (void)wl_out;
    }
    if (T > 1) {
        reduce_threads(F, Fbuf, T, nf);
        reduce_threads(wl, wbuf, T, nw);
        free(Fbuf);
        free(wbuf);
    }
    int st = pairwise_post(n, box, pos, vel, nn, nl, maxnb, G, W, J, Fpair);
    if (WL) memcpy(WL, wl, sizeof(double) * 9 * (size_t)n);
    if (JL) stress_current(n, wl, vel, JL);
    if (!Gout) free(G);
    free(wl);
    return st;
}

/* Single-element Tersoff (the form the paper prints in Section 2.1). */
int ora_tersoff(long n, const double *box, const double *pos, const double *vel,
                const int *nn, const int *nl, int maxnb, const ora_tersoff_t *p,
                double *U, double *F, double *W, double *J,
                double *Fpair, double *WL, double *JL, double *Gout)
{
    return tersoff_core(n, box, pos, vel, NULL, 1, p, NULL, nn, nl, maxnb, U, F, W, J, Fpair,
                        WL, JL, Gout);
}

/* Tersoff's multicomponent form (Tersoff 1989, the potential the paper
 * cites; the paper states its method covers several atom types, Section
 * 2.1): per-element parameters elem[nt] with the mixing rules
 *   A_ij = sqrt(A_i A_j), B_ij = sqrt(B_i B_j), lambda_ij = (lambda_i + lambda_j)/2,
 *   mu_ij = (mu_i + mu_j)/2, R_ij = sqrt(R_i R_j), S_ij = sqrt(S_i S_j),
 * b_ij = chi_ij (1 + beta_i^n_i zeta_ij^n_i)^(-1/(2 n_i)), zeta_ij summing
 * f_C(r_ik) with the (i, k) cutoff and g with atom i's c, d, h.  chi[nt*nt]
 * (NULL: all 1) must be symmetric; types[n] in [0, nt). */
int ora_tersoff_multi(long n, const double *box, const double *pos, const double *vel,
                      const int *types, int nt, const ora_tersoff_t *elem, const double *chi,
                      const int *nn, const int *nl, int maxnb,
                      double *U, double *F, double *W, double *J,
                      double *Fpair, double *WL, double *JL, double *Gout)
{
    if (nt < 1 || nt > 8 || !elem || !types) return ORA_EINVAL;
    for (long i = 0; i < n; ++i)
        if (types[i] < 0 || types[i] >= nt) return ORA_EINVAL;
    if (chi)
        for (int a = 0; a < nt; ++a)
            for (int b = 0; b < nt; ++b)
                if (chi[a * nt + b] != chi[b * nt + a]) return ORA_EINVAL;
    ora_tersoff_t P[64];
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b < nt; ++b) {
            const ora_tersoff_t *x = &elem[a], *y = &elem[b];
            ora_tersoff_t *q = &P[a * nt + b];
            q->A = sqrt(x->A * y->A);
            q->B = sqrt(x->B * y->B);
            q->lam = 0.5 * (x->lam + y->lam);
            q->mu = 0.5 * (x->mu + y->mu);
            q->R = sqrt(x->R * y->R);
            q->S = sqrt(x->S * y->S);
            q->beta = x->beta;
            q->n = x->n;
            q->c = x->c;
            q->d = x->d;
            q->h = x->h;
        }
    return tersoff_core(n, box, pos, vel, types, nt, P, chi, nn, nl, maxnb, U, F, W, J, Fpair,
                        WL, JL, Gout);
}

/* ----------------------------------------------------- Stillinger-Weber */

static double sw_phi2(const ora_sw_t *p, double r)
{
    double rc = p->a * p->sigma;
    if (r >= rc) return 0.0;
    double sr = p->sigma / r;
    return p->epsilon * p->A * (p->B * pow(sr, p->p) - pow(sr, p->q)) *
           exp(p->sigma / (r - rc));
}

static double sw_dphi2(const ora_sw_t *p, double r)
{
    double rc = p->a * p->sigma;
    if (r >= rc) return 0.0;
    double e = exp(p->sigma / (r - rc));
    double poly = p->B * pow(p->sigma / r, p->p) - pow(p->sigma / r, p->q);
    double dpoly = (-p->p * p->B * pow(p->sigma / r, p->p) + p->q * pow(p->sigma / r, p->q)) / r;
    double de = -e * p->sigma / ((r - rc) * (r - rc));
    return p->epsilon * p->A * (dpoly * e + poly * de);
}

/* SW per-atom energy U_i = 1/2 sum_j phi_2(r_ij) + sum_{j<k} h_ijk with
 * h_ijk = eps lambda exp(gamma sigma/(r_ij - a sigma) + gamma sigma/(r_ik - a sigma))
 *         (cos theta_ijk + 1/3)^2, scattered conventionally with capture. */
int ora_sw(long n, const double *box, const double *pos, const double *vel,
           const int *nn, const int *nl, int maxnb, const ora_sw_t *p,
           double *U, double *F, double *W, double *J,
           double *Fpair, double *WL, double *JL, double *Gout)
{
    for (long i = 0; i < n; ++i)
        if (nn[i] > maxnb) return ORA_ENEIGH;
    size_t gsz = (size_t)(n > 0 ? n : 1) * maxnb * 3;
    double *G = Gout ? Gout : (double *)malloc(sizeof(double) * gsz);
    double *wl = (double *)calloc((size_t)(n > 0 ? n : 1) * 9, sizeof(double));
    if (!G || !wl) { if (!Gout) free(G); free(wl); return ORA_ENOMEM; }
    memset(G, 0, sizeof(double) * gsz);
    double rc = p->a * p->sigma;
    for (long i = 0; i < n; ++i) {
        U[i] = 0.0;
        F[i * 3 + 0] = F[i * 3 + 1] = F[i * 3 + 2] = 0.0;
    }
    const int T = ora_threads();
    const size_t nf = (size_t)(n > 0 ? n : 1) * 3, nw = (size_t)(n > 0 ? n : 1) * 9;
    double *Fbuf = T > 1 ? (double *)malloc(sizeof(double) * (size_t)T * nf) : NULL;
    double *wbuf = T > 1 ? (double *)malloc(sizeof(double) * (size_t)T * nw) : NULL;
    if (T > 1 && (!Fbuf || !wbuf)) {
        free(Fbuf); free(wbuf);
        if (!Gout) free(G);
        free(wl);
        return ORA_ENOMEM;
    }
#pragma omp parallel num_threads(T) if (T > 1)
    {
    double *const F_out = F, *const wl_out = wl;
    double *F = T > 1 ? Fbuf + (size_t)thread_id() * nf : F_out;     /* this thread's scatter */
    double *wl = T > 1 ? wbuf + (size_t)thread_id() * nw : wl_out;
    if (T > 1) {                       /* each thread clears its own buffers */
        memset(F, 0, sizeof(double) * nf);
        memset(wl, 0, sizeof(double) * nw);
    }
#pragma omp for schedule(static)
    for (long i = 0; i < n; ++i) {
        int cnt = nn[i];
        for (int m = 0; m < cnt; ++m) {
            long j = nl[i * maxnb + m];
            double rij[3];
            min_image(box, &pos[i * 3], &pos[j * 3], rij);
            double r = sqrt(dot3(rij, rij));
            if (r >= rc) continue;
            U[i] += 0.5 * sw_phi2(p, r);
            double dp = sw_dphi2(p, r);
            double fj[3], fi[3];
            for (int a = 0; a < 3; ++a) {
                double u = rij[a] / r;
                fj[a] = -0.5 * dp * u;     /* -d(phi_2/2)/dr_j */
                fi[a] = 0.5 * dp * u;      /* -d(phi_2/2)/dr_i */
            }
            for (int a = 0; a < 3; ++a) {
                F[i * 3 + a] += fi[a];
                F[j * 3 + a] += fj[a];
                G[((size_t)i * maxnb + m) * 3 + a] -= fj[a];
            }
            for (int a = 0; a < 3; ++a)
                for (int bb = 0; bb < 3; ++bb) {
                    wl[i * 9 + 3 * a + bb] -= 0.5 * rij[a] * fi[bb];
                    wl[j * 9 + 3 * a + bb] -= 0.5 * rij[a] * fi[bb];
                }
            for (int q = m + 1; q < cnt; ++q) {
                long k = nl[i * maxnb + q];
                double rik[3];
                min_image(box, &pos[i * 3], &pos[k * 3], rik);
                double rk = sqrt(dot3(rik, rik));
                if (rk >= rc) continue;
                double cs = dot3(rij, rik) / (r * rk);
                double ex = p->epsilon * p->lam *
                            exp(p->gamma * p->sigma / (r - rc) + p->gamma * p->sigma / (rk - rc));
                double ang = cs + 1.0 / 3.0;
                double h = ex * ang * ang;
                U[i] += h;
                double dh_drij = -h * p->gamma * p->sigma / ((r - rc) * (r - rc));
                double dh_drik = -h * p->gamma * p->sigma / ((rk - rc) * (rk - rc));
                double dh_dcos = 2.0 * ex * ang;
                double gj[3], gk[3], gi[3];
                for (int a = 0; a < 3; ++a) {
                    double uij = rij[a] / r, uik = rik[a] / rk;
                    double dcos_j = (uik - cs * uij) / r;
                    double dcos_k = (uij - cs * uik) / rk;
                    gj[a] = dh_drij * uij + dh_dcos * dcos_j;    /* dh/dr_j */
                    gk[a] = dh_drik * uik + dh_dcos * dcos_k;    /* dh/dr_k */
                    gi[a] = -(gj[a] + gk[a]);                    /* dh/dr_i */
                }
                double f3i[3], f3j[3], f3k[3];
                for (int a = 0; a < 3; ++a) {
                    f3i[a] = -gi[a]; f3j[a] = -gj[a]; f3k[a] = -gk[a];
                }
                for (int a = 0; a < 3; ++a) {
                    F[i * 3 + a] += f3i[a];
                    F[j * 3 + a] += f3j[a];
                    F[k * 3 + a] += f3k[a];
                    G[((size_t)i * maxnb + m) * 3 + a] -= f3j[a];
                    G[((size_t)i * maxnb + q) * 3 + a] -= f3k[a];
                }
                for (int a = 0; a < 3; ++a)
                    for (int bb = 0; bb < 3; ++bb) {
                        double w = (rij[a] * f3j[bb] + rik[a] * f3k[bb]) / 3.0;
                        wl[i * 9 + 3 * a + bb] += w;
                        wl[j * 9 + 3 * a + bb] += w;
                        wl[k * 9 + 3 * a + bb] += w;
                    }
            }
        }
    }
    (void)F_out; (void)wl_out;
    }
    if (T > 1) {
        reduce_threads(F, Fbuf, T, nf);
        reduce_threads(wl, wbuf, T, nw);
        free(Fbuf);
        free(wbuf);
    }
    int st = pairwise_post(n, box, pos, vel, nn, nl, maxnb, G, W, J, Fpair);
    if (WL) memcpy(WL, wl, sizeof(double) * 9 * (size_t)n);
    if (JL) stress_current(n, wl, vel, JL);
    if (!Gout) free(G);
    free(wl);
    return st;
}

/* ------------------------------------------------------------------- NVE */

#define ORA_KAPPA 9.64853321567e-3     /* eV/(A amu) in A/fs^2 */
#define ORA_KB 8.617333262e-5          /* eV/K */

/* Parameters of potential 2 (multicomponent Tersoff) for the integrators. */
typedef struct {
    int ntypes;
    const int *types;
    const ora_tersoff_t *elem;
    const double *chi;
} ora_tersoff_multi_t;

static int evaluate(int potential, const void *params, long n, const double *box,
                    const double *pos, const double *vel, const int *nn, const int *nl,
                    int maxnb, double *U, double *F, double *W, double *J, double *G)
{
    if (potential == 0)
        return ora_tersoff(n, box, pos, vel, nn, nl, maxnb, (const ora_tersoff_t *)params,
                           U, F, W, J, NULL, NULL, NULL, G);
    if (potential == 2) {
        const ora_tersoff_multi_t *m = (const ora_tersoff_multi_t *)params;
        return ora_tersoff_multi(n, box, pos, vel, m->types, m->ntypes, m->elem, m->chi, nn, nl,
                                 maxnb, U, F, W, J, NULL, NULL, NULL, G);
    }
    return ora_sw(n, box, pos, vel, nn, nl, maxnb, (const ora_sw_t *)params,
                  U, F, W, J, NULL, NULL, NULL, G);
}

/* masses: per-atom masses, or NULL for `mass` on every atom. */
static void thermo_row(long n, double mass, const double *masses, const double *U,
                       const double *vel, const double *W, const double *J, double *row)
{
    memset(row, 0, sizeof(double) * 16);
    double ep = 0.0, ek = 0.0;
    for (long i = 0; i < n; ++i) {
        const double m = masses ? masses[i] : mass;
        ep += U[i];
        ek += 0.5 * m * dot3(&vel[i * 3], &vel[i * 3]) / ORA_KAPPA;
        for (int c = 0; c < 9; ++c) row[2 + c] += W[i * 9 + c];
        for (int c = 0; c < 3; ++c) row[11 + c] += J[i * 3 + c];
    }
    row[0] = ep;
    row[1] = ek;
    row[14] = ep + ek;
    row[15] = n > 1 ? 2.0 * ek / ((3.0 * n - 3.0) * ORA_KB) : 0.0;
}

/* Velocity-Verlet NVE.  pos/vel are advanced in place.  The list (cell
 * method, radius rlist) is built before the evaluation of step 0 and rebuilt
 * before step s when s - (step of the last build) == rebuild_every, or, with
 * check_skin, when some atom of step s moved more than skin/2 from its
 * position at the last build.  thermo is [n_steps + 1][16]: 0 E_pot,
 * 1 E_kin, 2..10 W (row-major), 11..13 J, 14 E_pot + E_kin, 15 kinetic
 * temperature (3N - 3 degrees of freedom).  U, F, W, J hold the final step's
 * per-atom values; *n_builds (may be NULL) the number of list builds. */
static double max_disp2(long n, const double *box, const double *pos, const double *ref)
{
    double worst = 0.0;
    for (long i = 0; i < n; ++i) {
        double d[3];
        min_image(box, &ref[i * 3], &pos[i * 3], d);
        double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (d2 > worst) worst = d2;
    }
    return worst;
}

static int masses_ok(long n, double mass, const double *masses)
{
    if (!masses) return mass > 0.0;
    for (long i = 0; i < n; ++i)
        if (!(masses[i] > 0.0)) return 0;
    return 1;
}

/* masses: per-atom masses (amu), or NULL for `mass` on every atom. */
int ora_nve(int potential, const void *params, long n, const double *box, double mass,
            const double *masses, double *pos, double *vel, int n_steps, double dt,
            double rlist, double skin, int rebuild_every, int check_skin, int maxnb, double *U,
            double *F, double *W, double *J, double *thermo, long *n_builds)
{
    if (n < 1 || n_steps < 0 || rebuild_every < 1 || maxnb < 1 || !masses_ok(n, mass, masses))
        return ORA_EINVAL;
    int st = check_box(box, rlist);
    if (st) return st;
    int *nn = (int *)malloc(sizeof(int) * (size_t)n);
    int *nl = (int *)malloc(sizeof(int) * (size_t)n * maxnb);
    double *G = (double *)malloc(sizeof(double) * (size_t)n * maxnb * 3);
    double *xb = (double *)malloc(sizeof(double) * (size_t)n * 3);
    if (!nn || !nl || !G || !xb) { free(nn); free(nl); free(G); free(xb); return ORA_ENOMEM; }
    ora_wrap(n, box, pos);
    st = ora_neighbors_cells(n, box, pos, rlist, maxnb, nn, nl);
    memcpy(xb, pos, sizeof(double) * (size_t)n * 3);
    long builds = 1;
    int last_build = 0;
    double lim = 0.25 * skin * skin;
    if (!st) st = evaluate(potential, params, n, box, pos, vel, nn, nl, maxnb, U, F, W, J, G);
    if (!st && thermo) thermo_row(n, mass, masses, U, vel, W, J, &thermo[0]);
    for (int s = 1; s <= n_steps && !st; ++s) {
        for (long i = 0; i < n; ++i) {
            const double half = 0.5 * dt * ORA_KAPPA / (masses ? masses[i] : mass);
            for (int a = 0; a < 3; ++a) {
                vel[i * 3 + a] += half * F[i * 3 + a];
                pos[i * 3 + a] += dt * vel[i * 3 + a];
            }
        }
        ora_wrap(n, box, pos);
        if (s - last_build == rebuild_every ||
            (check_skin && max_disp2(n, box, pos, xb) > lim)) {
            st = ora_neighbors_cells(n, box, pos, rlist, maxnb, nn, nl);
            if (st) break;
            memcpy(xb, pos, sizeof(double) * (size_t)n * 3);
            last_build = s;
            ++builds;
        }
        /* Forces at the new positions.  J needs the full-step velocity, so it
         * is formed from the captured partials after the second half-kick. */
        st = evaluate(potential, params, n, box, pos, NULL, nn, nl, maxnb, U, F, W, J, G);
        if (st) break;
        for (long i = 0; i < n; ++i) {
            const double half = 0.5 * dt * ORA_KAPPA / (masses ? masses[i] : mass);
            for (int a = 0; a < 3; ++a) vel[i * 3 + a] += half * F[i * 3 + a];
        }
        st = pairwise_post(n, box, pos, vel, nn, nl, maxnb, G, NULL, J, NULL);
        if (!st && thermo) thermo_row(n, mass, masses, U, vel, W, J, &thermo[(size_t)s * 16]);
    }
    free(G);
    free(xb);
    free(nn);
    free(nl);
    if (n_builds) *n_builds = builds;
    return st;
}

/* Pressure (eV/A^3) of a thermo row in a box of volume V: the kinetic part
 * 2 E_kin / 3 plus a third of the trace of the total virial, over V. */
static double row_pressure(const double *row, double volume)
{
    return (2.0 * row[1] + row[2] + row[6] + row[10]) / (3.0 * volume);
}

/* Velocity-Verlet with Berendsen weak coupling (NPT).  The step sequence of
 * ora_nve, and after the thermo row of every step except the last:
 *   lambda = sqrt(1 + (dt / tau_T) (T0 / T - 1))   (T from that row; 1 if
 *            tau_T <= 0 or T <= 0),
 *   mu = (1 - (beta dt / tau_P) (P0 - P))^(1/3)     (P from that row and the
 *            current volume; 1 if tau_P <= 0),
 *   v <- lambda v,  x <- mu x,  box <- mu box  (isotropic).
 * P0 in eV/A^3, beta (compressibility) in A^3/eV.  box is updated in place;
 * box_traj (or NULL) receives [n_steps + 1][3], the box each step's forces
 * were evaluated in.  The list is built at step 0 and every rebuild_every
 * steps (in the box of that moment).  With tau_T <= 0 and tau_P <= 0 the
 * run is ora_nve's with check_skin off, operation for operation. */
int ora_npt(int potential, const void *params, long n, double *box, double mass,
            const double *masses, double *pos, double *vel, int n_steps, double dt,
            double rlist, int rebuild_every, int maxnb, double T0, double tau_T, double P0,
            double tau_P, double beta, double *U, double *F, double *W, double *J,
            double *thermo, double *box_traj, long *n_builds)
{
    if (n < 2 || n_steps < 0 || rebuild_every < 1 || maxnb < 1 ||
        !masses_ok(n, mass, masses) || !thermo)
        return ORA_EINVAL;
    int st = check_box(box, rlist);
    if (st) return st;
    int *nn = (int *)malloc(sizeof(int) * (size_t)n);
    int *nl = (int *)malloc(sizeof(int) * (size_t)n * maxnb);
    double *G = (double *)malloc(sizeof(double) * (size_t)n * maxnb * 3);
    if (!nn || !nl || !G) { free(nn); free(nl); free(G); return ORA_ENOMEM; }
    ora_wrap(n, box, pos);
    st = ora_neighbors_cells(n, box, pos, rlist, maxnb, nn, nl);
    long builds = 1;
    int last_build = 0;
    for (int s = 0; s <= n_steps && !st; ++s) {
        if (s > 0) {
            for (long i = 0; i < n; ++i) {
                const double half = 0.5 * dt * ORA_KAPPA / (masses ? masses[i] : mass);
                for (int a = 0; a < 3; ++a) {
                    vel[i * 3 + a] += half * F[i * 3 + a];
                    pos[i * 3 + a] += dt * vel[i * 3 + a];
                }
            }
            ora_wrap(n, box, pos);
            if (s - last_build == rebuild_every) {
                st = check_box(box, rlist);
                if (!st) st = ora_neighbors_cells(n, box, pos, rlist, maxnb, nn, nl);
                if (st) break;
                last_build = s;
                ++builds;
            }
        }
        /* J pairs r(s) with v(s): at step 0 the evaluation forms it from the
         * given velocities, later from the captured partials after the
         * second half-kick (as in ora_nve) */
        st = evaluate(potential, params, n, box, pos, s == 0 ? vel : NULL, nn, nl, maxnb, U, F,
                      W, J, G);
        if (st) break;
        if (s > 0) {
            for (long i = 0; i < n; ++i) {
                const double half = 0.5 * dt * ORA_KAPPA / (masses ? masses[i] : mass);
                for (int a = 0; a < 3; ++a) vel[i * 3 + a] += half * F[i * 3 + a];
            }
            st = pairwise_post(n, box, pos, vel, nn, nl, maxnb, G, NULL, J, NULL);
            if (st) break;
        }
        double *row = &thermo[(size_t)s * 16];
        thermo_row(n, mass, masses, U, vel, W, J, row);
        if (box_traj)
            for (int a = 0; a < 3; ++a) box_traj[(size_t)s * 3 + a] = box[a];
        if (s == n_steps) break;
        /* weak coupling */
        const double T = row[15];
        double lambda = 1.0, mu = 1.0;
        if (tau_T > 0.0 && T > 0.0) lambda = sqrt(1.0 + dt / tau_T * (T0 / T - 1.0));
        if (tau_P > 0.0) {
            const double P = row_pressure(row, box[0] * box[1] * box[2]);
            const double mu3 = 1.0 - beta * dt / tau_P * (P0 - P);
            if (!(mu3 > 0.0)) { st = ORA_EINVAL; break; }
            mu = cbrt(mu3);
        }
        for (long i = 0; i < n; ++i)
            for (int a = 0; a < 3; ++a) {
                vel[i * 3 + a] *= lambda;
                pos[i * 3 + a] *= mu;
            }
        for (int a = 0; a < 3; ++a) box[a] *= mu;
    }
    free(G);
    free(nn);
    free(nl);
    if (n_builds) *n_builds = builds;
    return st;
}
