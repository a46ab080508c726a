/*
 * mdlj_oracle.c -- plain, slow, FP64 CPU oracle for the short-range
 * Lennard-Jones 12-6 force path of "Tuning of Vectorization Parameters for
 * Molecular Dynamics Simulations in AutoPas" (arXiv 2512.03565).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no code,
 * header, table or helper with the HIP implementation, and the HIP
 * implementation never calls it.
 *
 * What it computes (all in IEEE binary64, built with -ffp-contract=off):
 *
 *   - the force on each particle as the plain sum of pair forces,
 *     F_i = sum_{j != i} F_ij                      (paper section 2.1, Eq. 1)
 *     restricted to pairs inside the cutoff, r_ij < r_c   (section 2.1)
 *     with F_ij = -F_ji                          (section 2.1, Newton's third law)
 *   - the pair law: the textbook Lennard-Jones 12-6 potential, which the
 *     paper names (section 4.1) but does not write out:
 *         u(r)  = 4 eps [ (sig/r)^12 - (sig/r)^6 ] - u_shift
 *         F_ij  = 24 eps s6 (2 s6 - 1) / r^2 * d_ij ,  s6 = (sig^2/r^2)^3
 *         r.F   = 24 eps s6 (2 s6 - 1)                  (pair virial)
 *     the force is truncated (not shifted); the energy shift, when on, is
 *     u_shift = 4 eps [ (sig/rc)^12 - (sig/rc)^6 ] so u(rc-) = 0.
 *   - Lorentz-Berthelot mixing for several species:
 *         sig_ab = (sig_a + sig_b)/2 ,  eps_ab = sqrt(eps_a eps_b)
 *   - the minimum-image separation in an orthorhombic periodic box,
 *         d = x_i - x_j ;  d -= L * rint(d / L)   (per axis, in that order)
 *   - totals U = sum_{i<j} u(r_ij), W = sum_{i<j} r_ij . F_ij, and the
 *     per-particle energy u_i = 1/2 sum_j u(r_ij).
 *   - two neighbour searches that must agree: O(N^2) brute force, and
 *     linked cells (section 2.1.1: equal cells, own cell plus neighbour
 *     cells) with cell edge l = L / floor(L / r_c) >= r_c and the 27-cell
 *     stencil; it needs at least 3 cells per axis.
 *   - velocity-Verlet integration, the integrator the paper's background
 *     names for turning forces into motion (section 2.1).
 *   - the small fully-connected network of the learned tuner (a
 *     data-driven alternative to full search, section 6): dense layers
 *     with ReLU, softmax, cross-entropy loss, its gradient by the chain
 *     rule, and one Adam step (Kingma & Ba 2015, Algorithm 1).
 *
 * Nothing here is blocked, fused or reordered beyond what these
 * definitions say.  OpenMP is used only to split the outer loop over
 * particles i; every F_i is still the sum over its own j in j order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_SPECIES 8

/* ------------------------------------------------------------------ */
/* Pair law (textbook LJ 12-6; section 4.1 names it).                  */
/* ------------------------------------------------------------------ */

/* Lorentz-Berthelot mixing of species a and b. */
void oracle_mix(double eps_a, double sig_a, double eps_b, double sig_b,
                double *eps_ab, double *sig_ab)
{
    *sig_ab = 0.5 * (sig_a + sig_b);
    *eps_ab = sqrt(eps_a * eps_b);
}

/* Energy shift so that u(rc) = 0 (zero when shift_on == 0). */
double oracle_shift(double eps, double sig, double rc, int shift_on)
{
    if (!shift_on) return 0.0;
    double sr = sig / rc;
    double sr6 = sr * sr * sr * sr * sr * sr;
    return 4.0 * eps * (sr6 * sr6 - sr6);
}

/*
 * One pair at squared distance r2 (the caller decides r2 < rc^2).
 * fscal: F_ij = fscal * d_ij (d_ij = x_i - x_j).  u: pair energy
 * (shifted when shift_on).  w: pair virial r_ij . F_ij.
 */
void oracle_lj_pair(double r2, double eps, double sig, double rc, int shift_on,
                    double *fscal, double *u, double *w)
{
    double sr2 = (sig * sig) / r2;
    double s6 = sr2 * sr2 * sr2;
    double rf = 24.0 * eps * s6 * (2.0 * s6 - 1.0); /* r . F */
    *fscal = rf / r2;
    *w = rf;
    *u = 4.0 * eps * s6 * (s6 - 1.0) - oracle_shift(eps, sig, rc, shift_on);
}

/* ------------------------------------------------------------------ */
/* Geometry                                                            */
/* ------------------------------------------------------------------ */

static double min_image(double d, double L)
{
    return d - L * rint(d / L);
}

/* Wrap into [0, L): x - L floor(x / L). */
double oracle_wrap(double x, double L)
{
    return x - L * floor(x / L);
}

/*
 * Linked-cell index of a wrapped coordinate: ncell cells of edge L/ncell;
 * c = (int)(x * (ncell / L)), clamped to ncell - 1 (a coordinate that
 * rounds to exactly L lands in the last cell).
 */
int oracle_cell_coord(double xw, double L, int ncell)
{
    double inv = (double)ncell / L;
    int c = (int)(xw * inv);
    if (c >= ncell) c = ncell - 1;
    if (c < 0) c = 0;
    return c;
}

/* Number of linked cells along an axis: floor(L / r) (edge >= r). */
int oracle_ncell(double L, double r)
{
    return (int)floor(L / r);
}

/*
 * Cell of every particle for a grid of nc[0] x nc[1] x nc[2] cells, x
 * fastest: cell = cx + nc0 * (cy + nc1 * cz).  Used to check binning
 * bit-exactly.
 */
void oracle_bin(int64_t n, const double *x, const double *y, const double *z,
                const double *box, const int *nc, int32_t *cell_of)
{
    for (int64_t i = 0; i < n; ++i) {
        int cx = oracle_cell_coord(oracle_wrap(x[i], box[0]), box[0], nc[0]);
        int cy = oracle_cell_coord(oracle_wrap(y[i], box[1]), box[1], nc[1]);
        int cz = oracle_cell_coord(oracle_wrap(z[i], box[2]), box[2], nc[2]);
        cell_of[i] = cx + nc[0] * (cy + nc[1] * cz);
    }
}

/* ------------------------------------------------------------------ */
/* Force sums                                                          */
/* ------------------------------------------------------------------ */

typedef struct {
    int nspec;
    double eps[ORC_MAX_SPECIES * ORC_MAX_SPECIES];
    double sig[ORC_MAX_SPECIES * ORC_MAX_SPECIES];
    double rc;
    int shift_on;
} pair_table;

static int make_table(pair_table *t, int nspec, const double *eps, const double *sig,
                      double rc, int shift_on)
{
    if (nspec < 1 || nspec > ORC_MAX_SPECIES) return -1;
    t->nspec = nspec;
    t->rc = rc;
    t->shift_on = shift_on;
    for (int a = 0; a < nspec; ++a)
        for (int b = 0; b < nspec; ++b)
            oracle_mix(eps[a], sig[a], eps[b], sig[b], &t->eps[a * nspec + b],
                       &t->sig[a * nspec + b]);
    return 0;
}

/*
 * Contribution of j to i (F_ij added to F_i, half of u and w to the
 * per-particle and total sums, so that each unordered pair counts once
 * after both i and j have been visited).  Returns 1 if within cutoff.
 */
static int add_pair(const pair_table *t, int ti, int tj, double dx, double dy, double dz,
                    double *fx, double *fy, double *fz, double *u_half, double *w_half)
{
    double r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 < t->rc * t->rc)) return 0;
    int k = ti * t->nspec + tj;
    double fscal, u, w;
    oracle_lj_pair(r2, t->eps[k], t->sig[k], t->rc, t->shift_on, &fscal, &u, &w);
    *fx += fscal * dx;
    *fy += fscal * dy;
    *fz += fscal * dz;
    *u_half += 0.5 * u;
    *w_half += 0.5 * w;
    return 1;
}

/*
 * O(N^2) brute force over all j != i with the minimum image.  Valid for
 * any box with L >= 2 rc on each axis.  u_i may be NULL.
 */
int oracle_forces_brute(int64_t n, const double *x, const double *y, const double *z,
                        const int32_t *type, int nspec, const double *eps, const double *sig,
                        const double *box, double rc, int shift_on,
                        double *fx, double *fy, double *fz, double *u_i,
                        double *U, double *W)
{
    pair_table t;
    if (make_table(&t, nspec, eps, sig, rc, shift_on)) return -1;
    if (box[0] < 2 * rc || box[1] < 2 * rc || box[2] < 2 * rc) return -2;
    double Us = 0.0, Ws = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double ax = 0, ay = 0, az = 0, ui = 0, wi = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = min_image(x[i] - x[j], box[0]);
            double dy = min_image(y[i] - y[j], box[1]);
            double dz = min_image(z[i] - z[j], box[2]);
            add_pair(&t, type ? type[i] : 0, type ? type[j] : 0, dx, dy, dz,
                     &ax, &ay, &az, &ui, &wi);
        }
        fx[i] = ax; fy[i] = ay; fz[i] = az;
        if (u_i) u_i[i] = ui;
        Us += ui;
        Ws += wi;
    }
    *U = Us;
    *W = Ws;
    return 0;
}

/* Linked-cell structure: particles listed per cell (head/next chains). */
typedef struct {
    int nc[3];
    int64_t ncells;
    int64_t *head;
    int64_t *next;
} cell_list;

static int build_cells(cell_list *cl, int64_t n, const double *x, const double *y,
                       const double *z, const double *box, double rcell)
{
    for (int a = 0; a < 3; ++a) {
        cl->nc[a] = oracle_ncell(box[a], rcell);
        if (cl->nc[a] < 3) return -2;
    }
    cl->ncells = (int64_t)cl->nc[0] * cl->nc[1] * cl->nc[2];
    cl->head = (int64_t *)malloc(sizeof(int64_t) * cl->ncells);
    cl->next = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    if (!cl->head || !cl->next) return -3;
    for (int64_t c = 0; c < cl->ncells; ++c) cl->head[c] = -1;
    /* insert in reverse so each chain lists its particles in index order */
    for (int64_t i = n - 1; i >= 0; --i) {
        int cx = oracle_cell_coord(oracle_wrap(x[i], box[0]), box[0], cl->nc[0]);
        int cy = oracle_cell_coord(oracle_wrap(y[i], box[1]), box[1], cl->nc[1]);
        int cz = oracle_cell_coord(oracle_wrap(z[i], box[2]), box[2], cl->nc[2]);
        int64_t c = cx + (int64_t)cl->nc[0] * (cy + (int64_t)cl->nc[1] * cz);
        cl->next[i] = cl->head[c];
        cl->head[c] = i;
    }
    return 0;
}

static void free_cells(cell_list *cl)
{
    free(cl->head);
    free(cl->next);
}

static int cell_of_particle(const cell_list *cl, const double *box, double xi, double yi,
                            double zi, int *cc)
{
    cc[0] = oracle_cell_coord(oracle_wrap(xi, box[0]), box[0], cl->nc[0]);
    cc[1] = oracle_cell_coord(oracle_wrap(yi, box[1]), box[1], cl->nc[1]);
    cc[2] = oracle_cell_coord(oracle_wrap(zi, box[2]), box[2], cl->nc[2]);
    return 0;
}

/* Sum over the 27 cells around i's cell (periodic), all j != i. */
static void lc_particle(const pair_table *t, const cell_list *cl, int64_t i, const double *x,
                        const double *y, const double *z, const int32_t *type,
                        const double *box, double *f3, double *ui, double *wi)
{
    int cc[3];
    cell_of_particle(cl, box, x[i], y[i], z[i], cc);
    double ax = 0, ay = 0, az = 0, uu = 0, ww = 0;
    for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                int nx = (cc[0] + ox + cl->nc[0]) % cl->nc[0];
                int ny = (cc[1] + oy + cl->nc[1]) % cl->nc[1];
                int nz = (cc[2] + oz + cl->nc[2]) % cl->nc[2];
                int64_t c = nx + (int64_t)cl->nc[0] * (ny + (int64_t)cl->nc[1] * nz);
                for (int64_t j = cl->head[c]; j >= 0; j = cl->next[j]) {
                    if (j == i) continue;
                    double dx = min_image(x[i] - x[j], box[0]);
                    double dy = min_image(y[i] - y[j], box[1]);
                    double dz = min_image(z[i] - z[j], box[2]);
                    add_pair(t, type ? type[i] : 0, type ? type[j] : 0, dx, dy, dz,
                             &ax, &ay, &az, &uu, &ww);
                }
            }
    f3[0] = ax; f3[1] = ay; f3[2] = az;
    *ui = uu;
    *wi = ww;
}

/*
 * Linked cells, cell edge L/floor(L/rc) >= rc, 27-cell stencil.
 * nthreads <= 0 uses the OpenMP default.  Returns -2 if fewer than 3
 * cells fit along an axis.
 */
int oracle_forces_lc(int64_t n, const double *x, const double *y, const double *z,
                     const int32_t *type, int nspec, const double *eps, const double *sig,
                     const double *box, double rc, int shift_on,
                     double *fx, double *fy, double *fz, double *u_i,
                     double *U, double *W, int nthreads)
{
    pair_table t;
    if (make_table(&t, nspec, eps, sig, rc, shift_on)) return -1;
    cell_list cl;
    int rcode = build_cells(&cl, n, x, y, z, box, rc);
    if (rcode) { if (rcode != -2) free_cells(&cl); return rcode; }
    double Us = 0.0, Ws = 0.0;
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : Us, Ws) num_threads(nt)
#endif
    for (int64_t i = 0; i < n; ++i) {
        double f3[3], ui, wi;
        lc_particle(&t, &cl, i, x, y, z, type, box, f3, &ui, &wi);
        fx[i] = f3[0]; fy[i] = f3[1]; fz[i] = f3[2];
        if (u_i) u_i[i] = ui;
        Us += ui;
        Ws += wi;
    }
    (void)nthreads;
    free_cells(&cl);
    *U = Us;
    *W = Ws;
    return 0;
}

/*
 * Forces on a subset of particles only (idx[0..m-1]); used to check a
 * large system at sampled particles.  Uses the same linked cells.
 */
int oracle_forces_lc_subset(int64_t n, const double *x, const double *y, const double *z,
                            const int32_t *type, int nspec, const double *eps,
                            const double *sig, const double *box, double rc, int shift_on,
                            int64_t m, const int64_t *idx, double *fx, double *fy, double *fz,
                            double *u_i, int nthreads)
{
    pair_table t;
    if (make_table(&t, nspec, eps, sig, rc, shift_on)) return -1;
    cell_list cl;
    int rcode = build_cells(&cl, n, x, y, z, box, rc);
    if (rcode) { if (rcode != -2) free_cells(&cl); return rcode; }
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nt)
#endif
    for (int64_t k = 0; k < m; ++k) {
        double f3[3], ui, wi;
        lc_particle(&t, &cl, idx[k], x, y, z, type, box, f3, &ui, &wi);
        fx[k] = f3[0]; fy[k] = f3[1]; fz[k] = f3[2];
        if (u_i) u_i[k] = ui;
    }
    (void)nthreads;
    free_cells(&cl);
    return 0;
}

/*
 * All unordered pairs {i, j} with r^2 < r^2_max (minimum image), found
 * by linked cells with edge >= rmax.  Writes up to cap pairs (i < j) and
 * returns the total count, or a negative code.
 */
int64_t oracle_pairs_within(int64_t n, const double *x, const double *y, const double *z,
                            const double *box, double rmax, int64_t cap, int64_t *pi,
                            int64_t *pj, double *pr2)
{
    cell_list cl;
    int rcode = build_cells(&cl, n, x, y, z, box, rmax);
    if (rcode) { if (rcode != -2) free_cells(&cl); return rcode; }
    int64_t cnt = 0;
    double r2max = rmax * rmax;
    for (int64_t i = 0; i < n; ++i) {
        int cc[3];
        cell_of_particle(&cl, box, x[i], y[i], z[i], cc);
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    int nx = (cc[0] + ox + cl.nc[0]) % cl.nc[0];
                    int ny = (cc[1] + oy + cl.nc[1]) % cl.nc[1];
                    int nz = (cc[2] + oz + cl.nc[2]) % cl.nc[2];
                    int64_t c = nx + (int64_t)cl.nc[0] * (ny + (int64_t)cl.nc[1] * nz);
                    for (int64_t j = cl.head[c]; j >= 0; j = cl.next[j]) {
                        if (j <= i) continue;
                        double dx = min_image(x[i] - x[j], box[0]);
                        double dy = min_image(y[i] - y[j], box[1]);
                        double dz = min_image(z[i] - z[j], box[2]);
                        double r2 = dx * dx + dy * dy + dz * dz;
                        if (r2 < r2max) {
                            if (cnt < cap) {
                                pi[cnt] = i;
                                pj[cnt] = j;
                                if (pr2) pr2[cnt] = r2;
                            }
                            ++cnt;
                        }
                    }
                }
    }
    free_cells(&cl);
    return cnt;
}

/* ------------------------------------------------------------------ */
/* Velocity Verlet (section 2.1 names Verlet integration)              */
/* ------------------------------------------------------------------ */

/*
 * nsteps velocity-Verlet steps with linked-cell forces:
 *   v += F dt / (2m);  x += v dt;  (wrap);  F = F(x);  v += F dt / (2m)
 * which equals x += v dt + F dt^2/(2m), v += (F_old + F_new) dt / (2m).
 * fx/fy/fz hold F(x) on entry (computed by the caller) and on exit.
 * epot/ekin (length nsteps + 1, may be NULL) receive U and the kinetic
 * energy before the first and after every step.
 */
int oracle_vv(int64_t n, double *x, double *y, double *z, double *vx, double *vy, double *vz,
              double *fx, double *fy, double *fz, const int32_t *type, int nspec,
              const double *eps, const double *sig, const double *mass, const double *box,
              double rc, int shift_on, double dt, int nsteps, double *epot, double *ekin,
              int nthreads)
{
    double U, W;
    int rcode = oracle_forces_lc(n, x, y, z, type, nspec, eps, sig, box, rc, shift_on, fx, fy,
                                 fz, NULL, &U, &W, nthreads);
    if (rcode) return rcode;
    for (int s = 0; s <= nsteps; ++s) {
        if (s > 0) {
            for (int64_t i = 0; i < n; ++i) {
                double m = mass[type ? type[i] : 0];
                vx[i] += 0.5 * dt * fx[i] / m;
                vy[i] += 0.5 * dt * fy[i] / m;
                vz[i] += 0.5 * dt * fz[i] / m;
                x[i] = oracle_wrap(x[i] + dt * vx[i], box[0]);
                y[i] = oracle_wrap(y[i] + dt * vy[i], box[1]);
                z[i] = oracle_wrap(z[i] + dt * vz[i], box[2]);
            }
            rcode = oracle_forces_lc(n, x, y, z, type, nspec, eps, sig, box, rc, shift_on, fx,
                                     fy, fz, NULL, &U, &W, nthreads);
            if (rcode) return rcode;
            for (int64_t i = 0; i < n; ++i) {
                double m = mass[type ? type[i] : 0];
                vx[i] += 0.5 * dt * fx[i] / m;
                vy[i] += 0.5 * dt * fy[i] / m;
                vz[i] += 0.5 * dt * fz[i] / m;
            }
        }
        if (epot) epot[s] = U;
        if (ekin) {
            double k = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                double m = mass[type ? type[i] : 0];
                k += 0.5 * m * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
            }
            ekin[s] = k;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Learned tuner network (data-driven tuning, section 6)               */
/* ------------------------------------------------------------------ */

/*
 * Dense layer y = W x + b with W stored row-major as [out][in].
 * Network: h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), z = W3 h2 + b3,
 * p = softmax(z).  X is [batch][d_in]; logits/probs are [batch][k].
 * The hidden activations (may be NULL) are [batch][h1] and [batch][h2].
 */
static void dense(int din, int dout, const double *W, const double *b, const double *x,
                  double *y)
{
    for (int o = 0; o < dout; ++o) {
        double s = b[o];
        for (int i = 0; i < din; ++i) s += W[o * din + i] * x[i];
        y[o] = s;
    }
}

void oracle_mlp_forward(int batch, int din, int dh1, int dh2, int k,
                        const double *W1, const double *b1, const double *W2, const double *b2,
                        const double *W3, const double *b3, const double *X,
                        double *H1, double *H2, double *logits, double *probs)
{
    double *h1 = (double *)malloc(sizeof(double) * dh1);
    double *h2 = (double *)malloc(sizeof(double) * dh2);
    for (int s = 0; s < batch; ++s) {
        dense(din, dh1, W1, b1, X + (int64_t)s * din, h1);
        for (int o = 0; o < dh1; ++o) h1[o] = h1[o] > 0.0 ? h1[o] : 0.0;
        dense(dh1, dh2, W2, b2, h1, h2);
        for (int o = 0; o < dh2; ++o) h2[o] = h2[o] > 0.0 ? h2[o] : 0.0;
        double *z = logits + (int64_t)s * k;
        dense(dh2, k, W3, b3, h2, z);
        double zmax = z[0];
        for (int o = 1; o < k; ++o) zmax = z[o] > zmax ? z[o] : zmax;
        double den = 0.0;
        for (int o = 0; o < k; ++o) den += exp(z[o] - zmax);
        for (int o = 0; o < k; ++o) probs[(int64_t)s * k + o] = exp(z[o] - zmax) / den;
        if (H1) memcpy(H1 + (int64_t)s * dh1, h1, sizeof(double) * dh1);
        if (H2) memcpy(H2 + (int64_t)s * dh2, h2, sizeof(double) * dh2);
    }
    free(h1);
    free(h2);
}

/*
 * Mean cross-entropy loss over the batch, L = -(1/B) sum_s log p_s[y_s],
 * and its gradient with respect to every weight and bias (chain rule:
 * dL/dz = (p - onehot(y)) / B, back through the dense layers and the
 * ReLU masks).  Gradients are written, not accumulated.  Returns L.
 */
double oracle_mlp_loss_grad(int batch, int din, int dh1, int dh2, int k,
                            const double *W1, const double *b1, const double *W2,
                            const double *b2, const double *W3, const double *b3,
                            const double *X, const int32_t *labels,
                            double *gW1, double *gb1, double *gW2, double *gb2, double *gW3,
                            double *gb3)
{
    double *H1 = (double *)malloc(sizeof(double) * batch * dh1);
    double *H2 = (double *)malloc(sizeof(double) * batch * dh2);
    double *Z = (double *)malloc(sizeof(double) * batch * k);
    double *P = (double *)malloc(sizeof(double) * batch * k);
    double *dz = (double *)malloc(sizeof(double) * k);
    double *dh2v = (double *)malloc(sizeof(double) * dh2);
    double *dh1v = (double *)malloc(sizeof(double) * dh1);
    oracle_mlp_forward(batch, din, dh1, dh2, k, W1, b1, W2, b2, W3, b3, X, H1, H2, Z, P);
    memset(gW1, 0, sizeof(double) * dh1 * din);
    memset(gb1, 0, sizeof(double) * dh1);
    memset(gW2, 0, sizeof(double) * dh2 * dh1);
    memset(gb2, 0, sizeof(double) * dh2);
    memset(gW3, 0, sizeof(double) * k * dh2);
    memset(gb3, 0, sizeof(double) * k);
    double loss = 0.0;
    for (int s = 0; s < batch; ++s) {
        const double *x = X + (int64_t)s * din;
        const double *h1 = H1 + (int64_t)s * dh1;
        const double *h2 = H2 + (int64_t)s * dh2;
        const double *p = P + (int64_t)s * k;
        loss -= log(p[labels[s]]) / batch;
        for (int o = 0; o < k; ++o) dz[o] = (p[o] - (o == labels[s] ? 1.0 : 0.0)) / batch;
        /* layer 3 */
        for (int o = 0; o < k; ++o) {
            gb3[o] += dz[o];
            for (int i = 0; i < dh2; ++i) gW3[o * dh2 + i] += dz[o] * h2[i];
        }
        for (int i = 0; i < dh2; ++i) {
            double g = 0.0;
            for (int o = 0; o < k; ++o) g += W3[o * dh2 + i] * dz[o];
            dh2v[i] = h2[i] > 0.0 ? g : 0.0;
        }
        /* layer 2 */
        for (int o = 0; o < dh2; ++o) {
            gb2[o] += dh2v[o];
            for (int i = 0; i < dh1; ++i) gW2[o * dh1 + i] += dh2v[o] * h1[i];
        }
        for (int i = 0; i < dh1; ++i) {
            double g = 0.0;
            for (int o = 0; o < dh2; ++o) g += W2[o * dh1 + i] * dh2v[o];
            dh1v[i] = h1[i] > 0.0 ? g : 0.0;
        }
        /* layer 1 */
        for (int o = 0; o < dh1; ++o) {
            gb1[o] += dh1v[o];
            for (int i = 0; i < din; ++i) gW1[o * din + i] += dh1v[o] * x[i];
        }
    }
    free(H1); free(H2); free(Z); free(P); free(dz); free(dh2v); free(dh1v);
    return loss;
}

/*
 * One Adam step (Kingma & Ba 2015) on n parameters, step number t >= 1:
 *   m = b1 m + (1-b1) g ;  v = b2 v + (1-b2) g^2
 *   w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 */
void oracle_adam_step(int64_t n, double *w, const double *g, double *m, double *v, int t,
                      double lr, double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, t);
    double c2 = 1.0 - pow(b2, t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        double mh = m[i] / c1;
        double vh = v[i] / c2;
        w[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
