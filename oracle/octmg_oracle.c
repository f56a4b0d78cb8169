/*
 * octmg_oracle.c -- FP64 CPU oracle for the octree multigrid solver.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference against which the HIP library is checked.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * library never does.  It shares no code with the library.
 *
 * What it implements (Teunissen & Schiavello, "Geometric multigrid method for
 * solving Poisson's equation on octree grids with irregular boundaries"):
 *   - block quadtree/octree with N^D-cell blocks, 2:1 balance      (Sec. 2.1)
 *   - standard (2D+1)-point Laplacian away from the interface      (eq. lpl-1d)
 *   - level set, boundary mask |f| < L |grad f|, L = 1.5 sqrt(D) dx (Sec. 3.6.1,
 *     eq. boundary-mask), grad f by central differences
 *   - relative interface distance d by bisection / golden-section bracket
 *     search with relative tolerance eps_tol                       (Sec. 3.2,
 *     eq. relative-distance)
 *   - unresolved boundaries on coarse grids: gradient descent with step
 *     w_min, at most dx/w_min steps, then a line search; the distance is
 *     used in the neighbour direction closest to the found point  (Sec. 3.6.3)
 *   - non-symmetric interface Laplacian, cut-link terms moved to the
 *     right-hand side                                               (Sec. 3.3,
 *     eqs. lpl-1d-lsf, lpl-2d-lsf)
 *   - red-black Gauss-Seidel smoothing                              (Sec. 2.2)
 *   - restriction = mean of the 2^D children, (bi/tri)linear
 *     prolongation, FAS V-cycle and FMG with N_down = N_up = 2    (Sec. 2.2,
 *     Sec. 3.4)
 *   - ghost cells filled so that coarse and averaged fine fluxes agree
 *     at refinement boundaries                                      (Sec. 2.2)
 *   - an exact direct (LU) solve on the 8^D coarse grid in place of the
 *     external coarse solver of Sec. 3.5.
 *
 * Readings where the paper is silent or garbled (all listed in the design
 * notes of the repository):
 *   * GSRB update: the printed 1D update has a flipped sign on the g term;
 *     the update used here solves the discrete equation L phi = g for the
 *     cell:  phi_i <- (g_i - b_i - sum_uncut c_ij phi_j) / c_ii.
 *   * red = (i+j+k) even in global level indices, red goes first; one
 *     smoothing step = red half-sweep + black half-sweep.
 *   * ghosts are refreshed before every half-sweep and every operator
 *     application and are constant within a half-sweep.
 *   * domain Dirichlet ghost: 2 phi_b(face centre) - phi_inside.
 *   * coarse-fine ghost: 1/2 C_k + 3/4 f1 - 1/4 f2, C_k = C + sum_t
 *     s_t (C_t+ - C_t-)/8 (flux-consistent, exact for linear phi).
 *   * prolongation: cell-centred tensor-product weights 3/4, 1/4 applied to
 *     e = phi_c - old_c; domain ghosts of e are odd reflections.
 *   * FMG without an initial guess (phi = 0): the rhs itself is restricted
 *     (nested iteration) and the first interpolation to each finer level is
 *     of the coarse solution, with Dirichlet ghosts 2 phi_b - phi_in (linear
 *     extrapolation along the first outside axis at edges and corners).
 *   * bisection: 27 halvings for eps_tol = 1e-8 (ceil(log2(1/eps))), d =
 *     midpoint of the final interval; golden section: <= 39 evaluations
 *     (ceil(ln eps / ln rho)), each new point tested for f(a)f(x) <= 0.
 *   * links leaving the domain are not searched.
 *   * the unresolved-boundary search runs only on parent (non-leaf) blocks
 *     with dx > w_min: its virtual links are a coarse-grid device and never
 *     enter the discretisation whose solution is returned.
 *   * every cell is an unknown, on both sides of the interface.
 *   * FAS rhs only on parent blocks; leaf blocks of coarse levels keep the
 *     user rhs.  old = phi on the whole coarse level after restriction.
 *   * adaptive trees: after each cycle phi is restricted top-down onto
 *     parent cells, so that the composite residual is defined.
 *   * zero-flux (Neumann) domain faces (Sec. 4.3): ghost = phi_inside;
 *     prolonged corrections are mirrored without the sign flip; the coarse
 *     operator folds the ghost into the diagonal.
 *   * sharp shapes (Sec. 4.2): p = 4 (x - 0.5), q = 4 (y - 0.5) (the
 *     printed division by 4 puts every shape outside the unit square); in
 *     3D p = 4 |(x, y) - (0.5, 0.5)|, q = 4 (z - 0.5) (rotation about the
 *     cube's vertical axis); |t|^(2/3) = cbrt(t^2) with a cube root made of
 *     + - * / only.
 *
 * Build: gcc -O2 -std=c99 -fPIC -shared -ffp-contract=off -fopenmp
 * (no fused multiply-add, so that level-set decisions are reproducible).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

#define MAXLEV 20

typedef struct {
    int dim, block_n, max_level, refine_kind;
    int lsf_kind, lsf_n, coarse_n, n_down;
    int n_up, neumann;        /* neumann: bit f set = zero-flux domain face f (x-,x+,y-,y+,z-,z+) */
    double refine_width, eps_tol, mask_factor, w_min;
    double lo[3];
    const double *lsf_params;
    int uniform_level, pad_;  /* levels <= uniform_level are complete (refinement) */
} orc_desc;

/* zero-flux (Neumann) domain face?  face = 2 axis + (side > 0) */
static int is_neumann(const orc_desc *d, int ax, int s) { return (d->neumann >> (2 * ax + (s > 0))) & 1; }

typedef struct {
    int blk, cell;  /* block index within the level, local cell index */
    double d[6];    /* relative distances per link (x-,x+,y-,y+,z-,z+) */
    double c[6];    /* link coefficients of eq. lpl-2d-lsf */
    double diag;    /* coefficient of phi_i */
    double b;       /* sum over cut links of c * phi_b (moved to the rhs) */
    int cut;        /* bitmask of cut links */
    long pt0;       /* first interface point of this record (level-local) */
    int inside;     /* f(cell centre) < 0 */
    double pb[6];   /* phi_b at the interface point of each cut link */
} Rec;

typedef struct {
    int n, Nb, nb;      /* cells per dim, block edge, blocks per dim */
    int nblocks, cpb;   /* existing blocks, cells per block */
    double dx;
    int *lut;           /* nb^D -> block index or -1 */
    int *pos;           /* [nblocks][3] block coordinates */
    int *leaf;          /* [nblocks] */
    double *phi, *g, *old, *r;
    int *rec_of;        /* per cell: record index or -1 */
    int nrec;
    Rec *rec;
    long npts;
    double *pts;        /* interface points x0, [npts][3] */
    double *bcv;        /* domain face values [2D][n^(D-1)] */
    long nface;         /* n^(D-1) */
} Level;

typedef struct {
    orc_desc d;
    double *lsfp;
    int D, nlev, nsub, adaptive;
    int nbisect, ngolden;
    Level L[MAXLEV];
} Orc;

/* ------------------------------------------------------------------ helpers */
static void *xcalloc(size_t n, size_t s) {
    void *p = calloc(n ? n : 1, s);
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}

/* Cube root of a >= 0 with + - * / only (so that every platform computes
 * the same bits): scale a by powers of 8 into [1/8, 1), six Newton steps
 * y <- (2y + m/y^2)/3 from y = 3/4 (the root lies in [1/2, 1), where the
 * iteration converges quadratically to a few ulp), scale back. */
static double cbrt_exact_ops(double a) {
    if (!(a > 0.0)) return 0.0;
    int k = 0;
    double m = a;
    while (m >= 1.0) { m = m * 0.125; k++; }
    while (m < 0.125) { m = m * 8.0; k--; }
    double y = 0.75;
    for (int i = 0; i < 6; i++) y = (2.0 * y + m / (y * y)) / 3.0;
    for (; k > 0; k--) y = y * 2.0;
    for (; k < 0; k++) y = y * 0.5;
    return y;
}

/* The four shapes of Sec. 4.2 (eqs. spheroid .. astroid) in coordinates
 * (p, q): 2D p = s (x - cx), q = s (y - cy); 3D, axisymmetric about the z
 * axis through (cx, cy): p = s (|(x - cx, y - cy)| - r0), q = s (z - cz);
 * params [cx, cy, cz, s, r0].  The paper prints p = (x - 0.5)/4, which puts
 * every shape outside the unit square; the scale used is 4 (x - 0.5).  Its
 * 3D form p = (sqrt(x^2 + y^2) - 0.5)/4 is cx = cy = 0, r0 = 0.5. */
static double shape_lsf(int kind, int D, const double *prm, const double *x) {
    double p, q;
    if (D == 2) {
        p = prm[3] * (x[0] - prm[0]);
        q = prm[3] * (x[1] - prm[1]);
    } else {
        double ex = x[0] - prm[0], ey = x[1] - prm[1];
        p = prm[3] * (sqrt(ex * ex + ey * ey) - prm[4]);
        q = prm[3] * (x[2] - prm[2]);
    }
    switch (kind) {
        case 3: return sqrt(8.0 * p * p + q * q) - 1.0;                       /* spheroid */
        case 4: return 8.0 * fabs(p) + fabs(q) - 1.5;                         /* rhombus */
        case 5: { double c = q - cbrt_exact_ops(p * p); return p * p + c * c - 1.0; } /* heart */
        default: return cbrt_exact_ops(p * p) / 0.8 + cbrt_exact_ops(q * q) / 1.5 - 0.8; /* astroid */
    }
}

/* Two electrodes (Sec. 4.3): a rod, the points within r_rod of the segment
 * a-b, and a sphere; f = min(dist(x, [a, b]) - r_rod, |x - c| - r_sph).
 * params [ax, ay, az, bx, by, bz, r_rod, cx, cy, cz, r_sph]. */
static double electrodes_lsf(const double *q, const double *x) {
    double ab[3], ax[3], t = 0.0, ll = 0.0, d2 = 0.0, s2 = 0.0;
    for (int c = 0; c < 3; c++) { ab[c] = q[3 + c] - q[c]; ax[c] = x[c] - q[c]; t += ax[c] * ab[c]; ll += ab[c] * ab[c]; }
    t = t / ll;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    for (int c = 0; c < 3; c++) { double e = x[c] - (q[c] + t * ab[c]); d2 += e * e; }
    for (int c = 0; c < 3; c++) { double e = x[c] - q[7 + c]; s2 += e * e; }
    double rod = sqrt(d2) - q[6], sph = sqrt(s2) - q[10];
    return rod < sph ? rod : sph;
}

/* level-set function (Sec. 3.1). Only + - * / sqrt and comparisons. */
static double lsf(const Orc *o, const double *x) {
    const double *p = o->lsfp;
    if (o->d.lsf_kind == 7) return electrodes_lsf(p, x);
    if (o->d.lsf_kind >= 3 && o->d.lsf_kind <= 6) return shape_lsf(o->d.lsf_kind, o->D, p, x);
    if (o->d.lsf_kind == 1) { /* union of spheres: min_m (|x - c_m| - r_m) */
        double f = 0.0;
        for (int m = 0; m < o->d.lsf_n; m++) {
            double dx = x[0] - p[4 * m + 0], dy = x[1] - p[4 * m + 1];
            double s = dx * dx + dy * dy;
            if (o->D == 3) { double dz = x[2] - p[4 * m + 2]; s = s + dz * dz; }
            double v = sqrt(s) - p[4 * m + 3];
            if (m == 0 || v < f) f = v;
        }
        return f;
    }
    if (o->d.lsf_kind == 2) { /* cylinder along z */
        double dx = x[0] - p[0], dy = x[1] - p[1];
        return sqrt(dx * dx + dy * dy) - p[2];
    }
    return 1.0; /* no interface */
}

static inline double centre(const Orc *o, const Level *L, int a, int gi) {
    return o->d.lo[a] + ((double)gi + 0.5) * L->dx;
}

static inline long local_index(int D, int Nb, const int *l) {
    return D == 3 ? ((long)l[2] * Nb + l[1]) * Nb + l[0] : (long)l[1] * Nb + l[0];
}

static inline void unravel(int D, int Nb, long li, int *l) {
    l[0] = (int)(li % Nb);
    l[1] = (int)((li / Nb) % Nb);
    l[2] = D == 3 ? (int)(li / ((long)Nb * Nb)) : 0;
}

/* flat field index of global cell g on level L: -2 outside the domain,
   -1 inside the domain but not covered by a block of this level. */
static long flat_of(const Orc *o, const Level *L, const int *g) {
    int D = o->D;
    for (int a = 0; a < D; a++)
        if (g[a] < 0 || g[a] >= L->n) return -2;
    int bp[3] = {g[0] / L->Nb, g[1] / L->Nb, D == 3 ? g[2] / L->Nb : 0};
    long li = D == 3 ? ((long)bp[2] * L->nb + bp[1]) * L->nb + bp[0] : (long)bp[1] * L->nb + bp[0];
    int blk = L->lut[li];
    if (blk < 0) return -1;
    int l[3] = {g[0] - bp[0] * L->Nb, g[1] - bp[1] * L->Nb, D == 3 ? g[2] - bp[2] * L->Nb : 0};
    return (long)blk * L->cpb + local_index(D, L->Nb, l);
}

static inline void cell_g(const Orc *o, const Level *L, int blk, long li, int *g) {
    int l[3];
    unravel(o->D, L->Nb, li, l);
    for (int a = 0; a < 3; a++) g[a] = L->pos[3 * blk + a] * L->Nb + l[a];
    if (o->D == 2) g[2] = 0;
}

/* index of the domain face value for cell g on face (axis a, side s) */
static long face_index(const Orc *o, const Level *L, int a, int s, const int *g) {
    long t;
    if (o->D == 3) {
        if (a == 0) t = (long)g[2] * L->n + g[1];
        else if (a == 1) t = (long)g[2] * L->n + g[0];
        else t = (long)g[1] * L->n + g[0];
    } else {
        t = (a == 0) ? g[1] : g[0];
    }
    return (long)(2 * a + (s > 0)) * L->nface + t;
}

static uint64_t morton(int D, const int *p) {
    uint64_t k = 0;
    for (int bit = 0; bit < 20; bit++)
        for (int a = 0; a < D; a++)
            k |= (uint64_t)((p[a] >> bit) & 1) << (D * bit + a);
    return k;
}

/* ------------------------------------------------------------- line search */
static void along(const double *a, const double *b, double t, double *x) {
    for (int c = 0; c < 3; c++) x[c] = a[c] + t * (b[c] - a[c]);
}

/* Bisection on [0, thi] of the segment a->b (Sec. 3.2): the sign test is
   f(a) f(x) <= 0; returns the midpoint of the final interval. */
static double bisect(const Orc *o, const double *a, const double *b, double fa, double thi) {
    double lo = 0.0, hi = thi, x[3];
    for (int it = 0; it < o->nbisect; it++) {
        double mid = 0.5 * (lo + hi);
        along(a, b, mid, x);
        if (fa * lsf(o, x) <= 0.0) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

/* Root search on a->b (Sec. 3.2, figure rootfinding): bisection when the
   segment is bracketed, else golden-section minimisation of f(a) f(x) until
   a bracket appears (then bisection on [a, x]) or the evaluation budget for
   eps_tol is spent (no root, d = 1). Returns t in (0,1]; *found = 1 if cut. */
static double line_search(const Orc *o, const double *a, const double *b, double fa, int *found) {
    double x[3];
    double fb = lsf(o, b);
    if (fa * fb <= 0.0) { *found = 1; return bisect(o, a, b, fa, 1.0); }
    const double rho = 0.5 * (sqrt(5.0) - 1.0);
    double lo = 0.0, hi = 1.0;
    double t1 = hi - rho * (hi - lo), t2 = lo + rho * (hi - lo);
    along(a, b, t1, x);
    double h1 = fa * lsf(o, x);
    if (h1 <= 0.0) { *found = 1; return bisect(o, a, b, fa, t1); }
    along(a, b, t2, x);
    double h2 = fa * lsf(o, x);
    if (h2 <= 0.0) { *found = 1; return bisect(o, a, b, fa, t2); }
    int nev = 2;
    while (nev < o->ngolden) {
        if (h1 < h2) {
            hi = t2; t2 = t1; h2 = h1;
            t1 = hi - rho * (hi - lo);
            along(a, b, t1, x);
            h1 = fa * lsf(o, x);
            nev++;
            if (h1 <= 0.0) { *found = 1; return bisect(o, a, b, fa, t1); }
        } else {
            lo = t1; t1 = t2; h1 = h2;
            t2 = lo + rho * (hi - lo);
            along(a, b, t2, x);
            h2 = fa * lsf(o, x);
            nev++;
            if (h2 <= 0.0) { *found = 1; return bisect(o, a, b, fa, t2); }
        }
    }
    *found = 0;
    return 1.0;
}

/* Unresolved-boundary search on coarse grids (Sec. 3.6.3): gradient descent
   towards f = 0 with step w_min, at most floor(dx/w_min) steps; when
   f(a) f(x) <= 0, a line search a->x gives the root x0, d = |x0-a|/dx and
   the direction of the neighbour centre closest to x. Returns 1 if found. */
static int coarse_search(const Orc *o, const Level *L, const double *a, double fa,
                         double *d_out, int *dir_out, double *x0_out) {
    double w = o->d.w_min, x[3] = {a[0], a[1], a[2]};
    double sgn = fa > 0.0 ? 1.0 : -1.0;
    int nsteps = (int)floor(L->dx / w), found = 0;
    for (int s = 0; s < nsteps; s++) {
        double gr[3] = {0, 0, 0}, nrm2 = 0.0;
        for (int c = 0; c < o->D; c++) {
            double xp[3] = {x[0], x[1], x[2]}, xm[3] = {x[0], x[1], x[2]};
            xp[c] = x[c] + w;
            xm[c] = x[c] - w;
            gr[c] = (lsf(o, xp) - lsf(o, xm)) / (2.0 * w);
            nrm2 = nrm2 + gr[c] * gr[c];
        }
        double nrm = sqrt(nrm2);
        if (!(nrm > 0.0)) break;
        int outside = 0;
        for (int c = 0; c < o->D; c++) {
            double step = -sgn * gr[c] / nrm;
            x[c] = x[c] + w * step;
            if (x[c] < o->d.lo[c] || x[c] > o->d.lo[c] + 1.0) outside = 1;
        }
        if (outside) break;
        if (fa * lsf(o, x) <= 0.0) { found = 1; break; }
    }
    if (!found) return 0;
    double t = bisect(o, a, x, fa, 1.0), x0[3] = {a[0], a[1], a[2]}, s2 = 0.0;
    along(a, x, t, x0);
    for (int c = 0; c < o->D; c++) s2 = s2 + (x0[c] - a[c]) * (x0[c] - a[c]);
    double d = sqrt(s2) / L->dx;
    if (!(d < 1.0)) return 0;
    double best = -1.0;
    int dir = 0;
    for (int c = 0; c < o->D; c++) {
        double v = x[c] - a[c];
        if (v > best) { best = v; dir = 2 * c + 1; }
        if (-v > best) { best = -v; dir = 2 * c; }
    }
    *d_out = d;
    *dir_out = dir;
    for (int c = 0; c < 3; c++) x0_out[c] = x0[c];
    return 1;
}

/* ---------------------------------------------------------------- the tree */
typedef struct { unsigned char *ex[MAXLEV]; int nb[MAXLEV]; } Flags;

static long lidx(int D, int nb, const int *p) {
    return D == 3 ? ((long)p[2] * nb + p[1]) * nb + p[0] : (long)p[1] * nb + p[0];
}

static void refine_block(Flags *F, int D, int l, const int *p) {
    int nch = 1 << D;
    for (int c = 0; c < nch; c++) {
        int q[3] = {2 * p[0] + (c & 1), 2 * p[1] + ((c >> 1) & 1), D == 3 ? 2 * p[2] + ((c >> 2) & 1) : 0};
        F->ex[l + 1][lidx(D, F->nb[l + 1], q)] = 1;
    }
}

/* make block p of tree level l exist (refining coarser blocks as needed) */
static void ensure(Flags *F, int D, int l, const int *p) {
    if (F->ex[l][lidx(D, F->nb[l], p)]) return;
    int q[3] = {p[0] / 2, p[1] / 2, p[2] / 2};
    ensure(F, D, l - 1, q);
    refine_block(F, D, l - 1, q);
}

typedef struct { uint64_t key; int p[3]; } KeyPos;
static int cmp_key(const void *a, const void *b) {
    uint64_t x = ((const KeyPos *)a)->key, y = ((const KeyPos *)b)->key;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static void build_levels(Orc *o) {
    int D = o->D, N = o->d.block_n, lmax = o->d.max_level;
    Flags F;
    memset(&F, 0, sizeof F);
    for (int l = 1; l <= lmax; l++) {
        F.nb[l] = 1 << (l - 1);
        long cnt = 1;
        for (int a = 0; a < D; a++) cnt *= F.nb[l];
        F.ex[l] = xcalloc(cnt, 1);
    }
    F.ex[1][0] = 1;
    /* refinement level by level */
    for (int l = 1; l < lmax; l++) {
        long cnt = 1;
        for (int a = 0; a < D; a++) cnt *= F.nb[l];
        for (long i = 0; i < cnt; i++) {
            if (!F.ex[l][i]) continue;
            int p[3] = {(int)(i % F.nb[l]), (int)((i / F.nb[l]) % F.nb[l]), D == 3 ? (int)(i / ((long)F.nb[l] * F.nb[l])) : 0};
            int refine = 1;
            if (o->d.refine_kind == 1 && l >= o->d.uniform_level) {
                double w = 1.0 / (double)F.nb[l], x[3] = {0, 0, 0};
                for (int a = 0; a < D; a++) x[a] = o->d.lo[a] + ((double)p[a] + 0.5) * w;
                refine = fabs(lsf(o, x)) < o->d.refine_width * w;
            }
            if (refine) refine_block(&F, D, l, p);
        }
    }
    /* 2:1 balance over face, edge and corner neighbours */
    for (int l = lmax; l >= 3; l--) {
        long cnt = 1;
        for (int a = 0; a < D; a++) cnt *= F.nb[l];
        for (long i = 0; i < cnt; i++) {
            if (!F.ex[l][i]) continue;
            int p[3] = {(int)(i % F.nb[l]), (int)((i / F.nb[l]) % F.nb[l]), D == 3 ? (int)(i / ((long)F.nb[l] * F.nb[l])) : 0};
            int nn = D == 3 ? 27 : 9;
            for (int m = 0; m < nn; m++) {
                int off[3] = {m % 3 - 1, (m / 3) % 3 - 1, D == 3 ? m / 9 - 1 : 0};
                int q[3], ok = 1;
                for (int a = 0; a < D; a++) {
                    q[a] = p[a] + off[a];
                    if (q[a] < 0 || q[a] >= F.nb[l]) ok = 0;
                }
                if (!ok) continue;
                int pq[3] = {q[0] / 2, q[1] / 2, D == 3 ? q[2] / 2 : 0};
                ensure(&F, D, l - 1, pq);
            }
        }
    }
    /* sub-root levels: single blocks halving down to coarse_n cells */
    int nsub = 0;
    for (int n = N; n > o->d.coarse_n; n /= 2) nsub++;
    o->nsub = nsub;
    o->nlev = nsub + lmax;
    o->adaptive = 0;
    for (int il = 0; il < o->nlev; il++) {
        Level *L = &o->L[il];
        int l = il - nsub + 1; /* tree level (<= 0 for sub-root) */
        if (l <= 0) {
            L->n = N >> (1 - l);
            L->Nb = L->n;
            L->nb = 1;
        } else {
            L->n = N << (l - 1);
            L->Nb = N;
            L->nb = 1 << (l - 1);
        }
        L->dx = 1.0 / (double)L->n;
        L->cpb = 1;
        L->nface = 1;
        for (int a = 0; a < D; a++) L->cpb *= L->Nb;
        for (int a = 0; a < D - 1; a++) L->nface *= L->n;
        long cnt = 1;
        for (int a = 0; a < D; a++) cnt *= L->nb;
        L->lut = xcalloc(cnt, sizeof(int));
        KeyPos *kp = xcalloc(cnt, sizeof(KeyPos));
        int nbk = 0;
        for (long i = 0; i < cnt; i++) {
            L->lut[i] = -1;
            if (l >= 1 && !F.ex[l][i]) continue;
            int p[3] = {(int)(i % L->nb), (int)((i / L->nb) % L->nb), D == 3 ? (int)(i / ((long)L->nb * L->nb)) : 0};
            kp[nbk].key = morton(D, p);
            memcpy(kp[nbk].p, p, sizeof p);
            nbk++;
        }
        qsort(kp, nbk, sizeof(KeyPos), cmp_key);
        L->nblocks = nbk;
        L->pos = xcalloc((size_t)nbk * 3, sizeof(int));
        L->leaf = xcalloc(nbk, sizeof(int));
        for (int b = 0; b < nbk; b++) {
            memcpy(&L->pos[3 * b], kp[b].p, 3 * sizeof(int));
            L->lut[lidx(D, L->nb, kp[b].p)] = b;
            if (l <= 0 || l == lmax) L->leaf[b] = (l == lmax);
            else {
                int q[3] = {2 * kp[b].p[0], 2 * kp[b].p[1], 2 * kp[b].p[2]};
                L->leaf[b] = !F.ex[l + 1][lidx(D, F.nb[l + 1], q)];
            }
            if (L->leaf[b] && l < lmax) o->adaptive = 1;
        }
        free(kp);
        size_t nc = (size_t)nbk * L->cpb;
        L->phi = xcalloc(nc, sizeof(double));
        L->g = xcalloc(nc, sizeof(double));
        L->old = xcalloc(nc, sizeof(double));
        L->r = xcalloc(nc, sizeof(double));
        L->rec_of = xcalloc(nc, sizeof(int));
        L->bcv = xcalloc((size_t)2 * D * L->nface, sizeof(double));
    }
    for (int l = 1; l <= lmax; l++) free(F.ex[l]);
}

/* ---------------------------------------------------------------- setup */
static void setup_level(Orc *o, int il) {
    Level *L = &o->L[il];
    int D = o->D;
    double dx = L->dx;
    double Lm = o->d.mask_factor * sqrt((double)D) * dx;
    int cap = 1024, nrec = 0;
    long capp = 1024, npts = 0;
    Rec *rec = xcalloc(cap, sizeof(Rec));
    double *pts = xcalloc(capp * 3, sizeof(double));
    for (int b = 0; b < L->nblocks; b++) {
        for (long li = 0; li < L->cpb; li++) {
            long fl = (long)b * L->cpb + li;
            L->rec_of[fl] = -1;
            int g[3];
            cell_g(o, L, b, li, g);
            double a[3] = {0, 0, 0};
            for (int c = 0; c < D; c++) a[c] = centre(o, L, c, g[c]);
            double fa = lsf(o, a);
            /* boundary mask, eq. boundary-mask */
            double nrm2 = 0.0;
            for (int c = 0; c < D; c++) {
                double xp[3] = {a[0], a[1], a[2]}, xm[3] = {a[0], a[1], a[2]};
                xp[c] = centre(o, L, c, g[c] + 1);
                xm[c] = centre(o, L, c, g[c] - 1);
                double gc = (lsf(o, xp) - lsf(o, xm)) / (2.0 * dx);
                nrm2 = nrm2 + gc * gc;
            }
            if (!(fabs(fa) < Lm * sqrt(nrm2))) continue;
            Rec R;
            memset(&R, 0, sizeof R);
            double x0[6][3];
            for (int k = 0; k < 2 * D; k++) R.d[k] = 1.0;
            for (int k = 0; k < 2 * D; k++) {
                int ax = k / 2, s = (k & 1) ? 1 : -1;
                if (g[ax] + s < 0 || g[ax] + s >= L->n) continue; /* leaves the domain */
                double bpt[3] = {a[0], a[1], a[2]};
                bpt[ax] = centre(o, L, ax, g[ax] + s);
                int found = 0;
                double t = line_search(o, a, bpt, fa, &found);
                if (found) {
                    R.d[k] = t;
                    R.cut |= 1 << k;
                    along(a, bpt, t, x0[k]);
                }
            }
            if (!R.cut && !L->leaf[b] && o->d.w_min > 0.0 && dx > o->d.w_min) {
                double d;
                int dir;
                double xx[3];
                if (coarse_search(o, L, a, fa, &d, &dir, xx)) {
                    R.d[dir] = d;
                    R.cut = 1 << dir;
                    memcpy(x0[dir], xx, sizeof xx);
                }
            }
            if (!R.cut) continue;
            R.blk = b;
            R.cell = (int)li;
            R.inside = fa < 0.0;
            double dx2 = dx * dx;
            R.diag = 0.0;
            for (int ax = 0; ax < D; ax++) {
                double dm = R.d[2 * ax], dp = R.d[2 * ax + 1];
                R.c[2 * ax] = 2.0 / ((dm + dp) * dm * dx2);
                R.c[2 * ax + 1] = 2.0 / ((dm + dp) * dp * dx2);
                R.diag = R.diag - R.c[2 * ax] - R.c[2 * ax + 1];
            }
            R.pt0 = npts;
            for (int k = 0; k < 2 * D; k++) {
                if (!(R.cut >> k & 1)) continue;
                if (npts == capp) { capp *= 2; pts = realloc(pts, capp * 3 * sizeof(double)); }
                for (int c = 0; c < 3; c++) pts[3 * npts + c] = c < D ? x0[k][c] : 0.0;
                npts++;
            }
            if (nrec == cap) { cap *= 2; rec = realloc(rec, cap * sizeof(Rec)); }
            L->rec_of[fl] = nrec;
            rec[nrec++] = R;
        }
    }
    L->rec = rec;
    L->nrec = nrec;
    L->pts = pts;
    L->npts = npts;
}

/* ------------------------------------------------------- operator & ghosts */
static double cf_ghost(const Orc *o, int il, const double *ff, const double *fc, const int *g, int ax, int s);

/* value of the uncut neighbour of cell g in direction (ax, s) on level il for
   field f (coarse field fc for refinement boundaries), ghosts included.
   Domain ghost: 2 phi_b(face centre) - phi_inside (Dirichlet), phi_inside
   (zero flux). */
static double nb_value(const Orc *o, int il, const double *f, const double *fc,
                       const int *g, long self, int ax, int s) {
    const Level *L = &o->L[il];
    int ng[3] = {g[0], g[1], g[2]};
    ng[ax] += s;
    long fl = flat_of(o, L, ng);
    if (fl >= 0) return f[fl];
    if (fl == -2) return is_neumann(&o->d, ax, s) ? f[self] : 2.0 * L->bcv[face_index(o, L, ax, s, g)] - f[self];
    return cf_ghost(o, il, f, fc, g, ax, s);
}

/* coarse value at coarse cell q (level il-1), with the coarse domain ghost
   2 phi_b - phi_in when q lies outside the domain in axis t */
static double coarse_val(const Orc *o, int ilc, const double *fc,
                         const int *q, const int *qin, int t, int s) {
    const Level *Lc = &o->L[ilc];
    long fl = flat_of(o, Lc, q);
    if (fl >= 0) return fc[fl];
    if (fl == -2)
        return is_neumann(&o->d, t, s) ? fc[flat_of(o, Lc, qin)]
                                       : 2.0 * Lc->bcv[face_index(o, Lc, t, s, qin)] - fc[flat_of(o, Lc, qin)];
    fprintf(stderr, "oracle: coarse cell missing (2:1 balance violated)\n");
    abort();
}

static double cf_ghost(const Orc *o, int il, const double *ff, const double *fc, const int *g, int ax, int s) {
    const Level *L = &o->L[il];
    int ng[3] = {g[0], g[1], g[2]};
    ng[ax] += s;
    int C[3] = {ng[0] / 2, ng[1] / 2, ng[2] / 2};
    long fC = flat_of(o, &o->L[il - 1], C);
    if (fC < 0) { fprintf(stderr, "oracle: coarse neighbour missing\n"); abort(); }
    double Ck = fc[fC];
    for (int t = 0; t < o->D; t++) {
        if (t == ax) continue;
        double st = (ng[t] & 1) ? 1.0 : -1.0;
        int qp[3] = {C[0], C[1], C[2]}, qm[3] = {C[0], C[1], C[2]};
        qp[t] += 1;
        qm[t] -= 1;
        double cp = coarse_val(o, il - 1, fc, qp, C, t, 1);
        double cm = coarse_val(o, il - 1, fc, qm, C, t, -1);
        Ck = Ck + st * (cp - cm) / 8.0;
    }
    int gi[3] = {g[0], g[1], g[2]};
    gi[ax] -= s;
    double f1 = ff[flat_of(o, L, g)], f2 = ff[flat_of(o, L, gi)];
    return 0.5 * Ck + 0.75 * f1 - 0.25 * f2;
}

/* sum_uncut c_k phi_k, diagonal and moved boundary term for cell (b, li) */
static void stencil(const Orc *o, int il, const double *f, const double *fc,
                    int b, long li, double *sum, double *diag, double *bterm) {
    const Level *L = &o->L[il];
    long fl = (long)b * L->cpb + li;
    int g[3];
    cell_g(o, L, b, li, g);
    int ri = L->rec_of[fl];
    double s = 0.0;
    if (ri < 0) {
        double inv = 1.0 / (L->dx * L->dx);
        for (int k = 0; k < 2 * o->D; k++)
            s = s + inv * nb_value(o, il, f, fc, g, fl, k / 2, (k & 1) ? 1 : -1);
        *diag = -2.0 * o->D * inv;
        *bterm = 0.0;
    } else {
        const Rec *R = &L->rec[ri];
        for (int k = 0; k < 2 * o->D; k++) {
            if (R->cut >> k & 1) continue;
            s = s + R->c[k] * nb_value(o, il, f, fc, g, fl, k / 2, (k & 1) ? 1 : -1);
        }
        *diag = R->diag;
        *bterm = R->b;
    }
    *sum = s;
}

static const double *coarse_phi(const Orc *o, int il) { return il > 0 ? o->L[il - 1].phi : NULL; }

/* one red-black Gauss-Seidel smoothing step on level il (Sec. 2.2) */
static void smooth_level(Orc *o, int il) {
    Level *L = &o->L[il];
    for (int color = 0; color < 2; color++) {
#pragma omp parallel for schedule(dynamic, 4)
        for (int b = 0; b < L->nblocks; b++) {
            for (long li = 0; li < L->cpb; li++) {
                int g[3];
                cell_g(o, L, b, li, g);
                if (((g[0] + g[1] + g[2]) & 1) != color) continue;
                double s, dg, bt;
                stencil(o, il, L->phi, coarse_phi(o, il), b, li, &s, &dg, &bt);
                L->phi[(long)b * L->cpb + li] = (L->g[(long)b * L->cpb + li] - bt - s) / dg;
            }
        }
    }
}

/* residual r = g - L phi on every cell of level il (eq. residual) */
static void level_residual(Orc *o, int il) {
    Level *L = &o->L[il];
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < L->nblocks; b++) {
        for (long li = 0; li < L->cpb; li++) {
            long fl = (long)b * L->cpb + li;
            double s, dg, bt;
            stencil(o, il, L->phi, coarse_phi(o, il), b, li, &s, &dg, &bt);
            L->r[fl] = L->g[fl] - (s + dg * L->phi[fl] + bt);
        }
    }
}

/* mean of the 2^D children of coarse cell C (fine level il) */
static double child_mean(const Orc *o, int il, const double *f, const int *C) {
    const Level *Lf = &o->L[il];
    int nch = 1 << o->D;
    double s = 0.0;
    for (int c = 0; c < nch; c++) {
        int q[3] = {2 * C[0] + (c & 1), 2 * C[1] + ((c >> 1) & 1), o->D == 3 ? 2 * C[2] + ((c >> 2) & 1) : 0};
        long fl = flat_of(o, Lf, q);
        if (fl < 0) { fprintf(stderr, "oracle: child missing\n"); abort(); }
        s = s + f[fl];
    }
    return s / (double)nch;
}

/* restriction of phi onto parent cells of level il-1 */
static void restrict_phi(Orc *o, int il) {
    Level *Lc = &o->L[il - 1];
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < Lc->nblocks; b++) {
        if (Lc->leaf[b]) continue;
        for (long li = 0; li < Lc->cpb; li++) {
            int C[3];
            cell_g(o, Lc, b, li, C);
            Lc->phi[(long)b * Lc->cpb + li] = child_mean(o, il, o->L[il].phi, C);
        }
    }
}

/* FAS restriction il -> il-1 (Sec. 2.2): phi_c and r_c are means of the
   children; on parent blocks g_c = L_c phi_c + r_c; old_c = phi_c. */
static void restrict_fas(Orc *o, int il) {
    Level *Lc = &o->L[il - 1];
    level_residual(o, il);
    restrict_phi(o, il);
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < Lc->nblocks; b++) {
        if (Lc->leaf[b]) continue;
        for (long li = 0; li < Lc->cpb; li++) {
            int C[3];
            cell_g(o, Lc, b, li, C);
            Lc->r[(long)b * Lc->cpb + li] = child_mean(o, il, o->L[il].r, C);
        }
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < Lc->nblocks; b++) {
        if (Lc->leaf[b]) continue;
        for (long li = 0; li < Lc->cpb; li++) {
            long fl = (long)b * Lc->cpb + li;
            double s, dg, bt;
            stencil(o, il - 1, Lc->phi, coarse_phi(o, il - 1), b, li, &s, &dg, &bt);
            Lc->g[fl] = (s + dg * Lc->phi[fl] + bt) + Lc->r[fl];
        }
    }
    memcpy(Lc->old, Lc->phi, sizeof(double) * (size_t)Lc->nblocks * Lc->cpb);
}

/* coarse correction e = phi_c - old_c at coarse cell q; outside the domain
   the correction is reflected, with a sign flip per outside axis across a
   Dirichlet face (homogeneous ghost -e) and none across a zero-flux face */
static double corr_at(const Orc *o, int ilc, const int *q) {
    const Level *Lc = &o->L[ilc];
    int qq[3] = {q[0], q[1], q[2]};
    double sign = 1.0;
    for (int a = 0; a < o->D; a++) {
        if (qq[a] < 0) { qq[a] = 0; if (!is_neumann(&o->d, a, -1)) sign = -sign; }
        else if (qq[a] >= Lc->n) { qq[a] = Lc->n - 1; if (!is_neumann(&o->d, a, 1)) sign = -sign; }
    }
    long fl = flat_of(o, Lc, qq);
    if (fl < 0) { fprintf(stderr, "oracle: prolongation source missing\n"); abort(); }
    return sign * (Lc->phi[fl] - Lc->old[fl]);
}

/* coarse solution phi_c at coarse cell q with Dirichlet ghosts: across one
   face 2 phi_b - phi_in; at edges and corners linear extrapolation along the
   first outside axis from two face-ghost values.  Across a zero-flux face
   (first outside axis) the value of the mirror cell. */
static double sol_at(const Orc *o, int ilc, const int *q) {
    const Level *Lc = &o->L[ilc];
    int out = -1;
    for (int a = 0; a < o->D; a++)
        if (q[a] < 0 || q[a] >= Lc->n) { out = a; break; }
    if (out < 0) return Lc->phi[flat_of(o, Lc, q)];
    int nout = 0;
    for (int a = 0; a < o->D; a++) nout += (q[a] < 0 || q[a] >= Lc->n);
    int s = q[out] < 0 ? -1 : 1;
    if (is_neumann(&o->d, out, s)) {  /* zero flux: the mirror image inside */
        int qi[3] = {q[0], q[1], q[2]};
        qi[out] -= s;
        return sol_at(o, ilc, qi);
    }
    if (nout == 1) {
        int qi[3] = {q[0], q[1], q[2]};
        qi[out] -= s;
        return 2.0 * Lc->bcv[face_index(o, Lc, out, s, qi)] - Lc->phi[flat_of(o, Lc, qi)];
    }
    int q1[3] = {q[0], q[1], q[2]}, q2[3] = {q[0], q[1], q[2]};
    q1[out] -= s;
    q2[out] -= 2 * s;
    return 2.0 * sol_at(o, ilc, q1) - sol_at(o, ilc, q2);
}

/* prolongation of the coarse correction onto level il (Sec. 2.2, 3.4):
   phi_f += sum_delta prod_a (3/4 or 1/4) e_c(C + delta o).  In solution
   mode (first FMG without initial guess) e_c = phi_c with Dirichlet ghosts. */
static void prolong(Orc *o, int il, int solution_mode) {
    Level *Lf = &o->L[il];
    int D = o->D, nch = 1 << D;
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < Lf->nblocks; b++) {
        for (long li = 0; li < Lf->cpb; li++) {
            int g[3];
            cell_g(o, Lf, b, li, g);
            int C[3] = {g[0] / 2, g[1] / 2, g[2] / 2}, od[3];
            for (int a = 0; a < 3; a++) od[a] = (g[a] & 1) ? 1 : -1;
            double e = 0.0;
            for (int c = 0; c < nch; c++) {
                double w = 1.0;
                int q[3] = {C[0], C[1], C[2]};
                for (int a = 0; a < D; a++) {
                    int on = (c >> a) & 1;
                    w = w * (on ? 0.25 : 0.75);
                    if (on) q[a] += od[a];
                }
                e = e + w * (solution_mode ? sol_at(o, il - 1, q) : corr_at(o, il - 1, q));
            }
            Lf->phi[(long)b * Lf->cpb + li] += e;
        }
    }
}

/* exact solve on the coarsest grid (replaces the external coarse solver of
   Sec. 3.5): dense matrix with domain ghosts folded in, LU with partial
   pivoting. */
static void coarse_solve(Orc *o) {
    Level *L = &o->L[0];
    int D = o->D;
    long n = (long)L->nblocks * L->cpb;
    double *A = xcalloc(n * n, sizeof(double)), *rhs = xcalloc(n, sizeof(double));
    double inv = 1.0 / (L->dx * L->dx);
    for (int b = 0; b < L->nblocks; b++) {
        for (long li = 0; li < L->cpb; li++) {
            long i = (long)b * L->cpb + li;
            int g[3];
            cell_g(o, L, b, li, g);
            int ri = L->rec_of[i];
            const Rec *R = ri >= 0 ? &L->rec[ri] : NULL;
            A[i * n + i] += R ? R->diag : -2.0 * D * inv;
            rhs[i] = L->g[i] - (R ? R->b : 0.0);
            for (int k = 0; k < 2 * D; k++) {
                if (R && (R->cut >> k & 1)) continue;
                double c = R ? R->c[k] : inv;
                int ax = k / 2, s = (k & 1) ? 1 : -1;
                int ng[3] = {g[0], g[1], g[2]};
                ng[ax] += s;
                long j = flat_of(o, L, ng);
                if (j >= 0) A[i * n + j] += c;
                else if (is_neumann(&o->d, ax, s)) A[i * n + i] += c;  /* ghost = phi_i */
                else {
                    A[i * n + i] -= c;
                    rhs[i] -= 2.0 * c * L->bcv[face_index(o, L, ax, s, g)];
                }
            }
        }
    }
    /* Gaussian elimination with partial pivoting */
    int *perm = xcalloc(n, sizeof(int));
    for (long i = 0; i < n; i++) perm[i] = (int)i;
    for (long k = 0; k < n; k++) {
        long p = k;
        for (long i = k + 1; i < n; i++)
            if (fabs(A[i * n + k]) > fabs(A[p * n + k])) p = i;
        if (p != k) {
            for (long j = 0; j < n; j++) { double t = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = t; }
            double t = rhs[k]; rhs[k] = rhs[p]; rhs[p] = t;
        }
        for (long i = k + 1; i < n; i++) {
            double m = A[i * n + k] / A[k * n + k];
            if (m == 0.0) continue;
            for (long j = k; j < n; j++) A[i * n + j] -= m * A[k * n + j];
            rhs[i] -= m * rhs[k];
        }
    }
    for (long i = n - 1; i >= 0; i--) {
        double s = rhs[i];
        for (long j = i + 1; j < n; j++) s -= A[i * n + j] * L->phi[j];
        L->phi[i] = s / A[i * n + i];
    }
    free(perm);
    free(A);
    free(rhs);
}

/* -------------------------------------------------------------- the cycles */
static void sync_down(Orc *o) {
    if (!o->adaptive) return;
    for (int il = o->nlev - 1; il > 0; il--) restrict_phi(o, il);
}

/* FAS V-cycle with top level `top` (Sec. 2.2, figure mg-cycles) */
static void vcycle(Orc *o, int top) {
    for (int il = top; il > 0; il--) {
        for (int s = 0; s < o->d.n_down; s++) smooth_level(o, il);
        restrict_fas(o, il);
    }
    coarse_solve(o);
    for (int il = 1; il <= top; il++) {
        prolong(o, il, 0);
        for (int s = 0; s < o->d.n_up; s++) smooth_level(o, il);
    }
}

/* plain restriction of the rhs onto parent cells of level il-1, phi_c =
   old_c = 0: the coarse problems of a first FMG without initial guess are
   the coarse discretisations of the same equation (nested iteration). */
static void restrict_rhs(Orc *o, int il) {
    Level *Lc = &o->L[il - 1];
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < Lc->nblocks; b++) {
        if (Lc->leaf[b]) continue;
        for (long li = 0; li < Lc->cpb; li++) {
            int C[3];
            cell_g(o, Lc, b, li, C);
            Lc->g[(long)b * Lc->cpb + li] = child_mean(o, il, o->L[il].g, C);
        }
    }
    memset(Lc->phi, 0, sizeof(double) * (size_t)Lc->nblocks * Lc->cpb);
    memset(Lc->old, 0, sizeof(double) * (size_t)Lc->nblocks * Lc->cpb);
}

/* FMG: restrict to the coarsest grid, solve, then V-cycles on successively
   finer levels after prolongating the correction (Sec. 2.2). With an initial
   guess the restriction is the FAS one; without (phi = 0 everywhere) the rhs
   itself is restricted. */
static void fmg(Orc *o, int have_guess) {
    int top = o->nlev - 1;
    for (int il = top; il > 0; il--) {
        if (have_guess) restrict_fas(o, il);
        else restrict_rhs(o, il);
    }
    coarse_solve(o);
    for (int il = 1; il <= top; il++) {
        prolong(o, il, !have_guess);
        vcycle(o, il);
    }
}

/* ------------------------------------------------------------- public API */
void *orc_create(const orc_desc *d) {
    if (!d || (d->dim != 2 && d->dim != 3) || d->max_level < 1 || d->max_level > 14) return NULL;
    if (d->block_n < d->coarse_n || d->coarse_n < 2 || (d->block_n & (d->block_n - 1))) return NULL;
    Orc *o = xcalloc(1, sizeof(Orc));
    o->d = *d;
    o->D = d->dim;
    int np = d->lsf_kind == 1 ? 4 * d->lsf_n
             : (d->lsf_kind == 2 ? 3 : (d->lsf_kind >= 3 && d->lsf_kind <= 6 ? 5 : (d->lsf_kind == 7 ? 11 : 0)));
    o->lsfp = xcalloc(np + 1, sizeof(double));
    if (np) memcpy(o->lsfp, d->lsf_params, np * sizeof(double));
    o->d.lsf_params = o->lsfp;
    o->nbisect = (int)ceil(-log(d->eps_tol) / log(2.0));
    o->ngolden = (int)ceil(log(d->eps_tol) / log(0.5 * (sqrt(5.0) - 1.0)));
    build_levels(o);
    for (int il = 0; il < o->nlev; il++) setup_level(o, il);
    return o;
}

void orc_destroy(void *h) {
    Orc *o = h;
    if (!o) return;
    for (int il = 0; il < o->nlev; il++) {
        Level *L = &o->L[il];
        free(L->lut); free(L->pos); free(L->leaf); free(L->phi); free(L->g); free(L->old);
        free(L->r); free(L->rec_of); free(L->rec); free(L->pts); free(L->bcv);
    }
    free(o->lsfp);
    free(o);
}

int orc_num_levels(void *h) { return ((Orc *)h)->nlev; }
int orc_is_adaptive(void *h) { return ((Orc *)h)->adaptive; }
int orc_search_counts(void *h, int *nb, int *ng) { *nb = ((Orc *)h)->nbisect; *ng = ((Orc *)h)->ngolden; return 0; }

/* out: n, Nb, nb, nblocks, nleaf_blocks, nrec, npts(long->int), nface */
void orc_level_info(void *h, int il, long *out) {
    Level *L = &((Orc *)h)->L[il];
    int nl = 0;
    for (int b = 0; b < L->nblocks; b++) nl += L->leaf[b];
    out[0] = L->n; out[1] = L->Nb; out[2] = L->nb; out[3] = L->nblocks;
    out[4] = nl; out[5] = L->nrec; out[6] = L->npts; out[7] = L->nface;
}

void orc_block_positions(void *h, int il, int *pos, int *leaf) {
    Level *L = &((Orc *)h)->L[il];
    memcpy(pos, L->pos, sizeof(int) * 3 * L->nblocks);
    memcpy(leaf, L->leaf, sizeof(int) * L->nblocks);
}

long orc_num_leaf_cells(void *h) {
    Orc *o = h;
    long n = 0;
    for (int il = 0; il < o->nlev; il++)
        for (int b = 0; b < o->L[il].nblocks; b++) n += o->L[il].leaf[b] ? o->L[il].cpb : 0;
    return n;
}

/* canonical leaf order: level, Morton block order, x-fastest cells */
static long leaf_walk(Orc *o, double *xyz, int *lvl, double *vals_in, double *vals_out, int field) {
    long n = 0;
    for (int il = 0; il < o->nlev; il++) {
        Level *L = &o->L[il];
        double *f = field == 0 ? L->phi : (field == 1 ? L->g : L->r);
        for (int b = 0; b < L->nblocks; b++) {
            if (!L->leaf[b]) continue;
            for (long li = 0; li < L->cpb; li++, n++) {
                long fl = (long)b * L->cpb + li;
                if (xyz) {
                    int g[3];
                    cell_g(o, L, b, li, g);
                    for (int c = 0; c < 3; c++) xyz[3 * n + c] = c < o->D ? centre(o, L, c, g[c]) : 0.0;
                }
                if (lvl) lvl[n] = il;
                if (vals_in) f[fl] = vals_in[n];
                if (vals_out) vals_out[n] = f[fl];
            }
        }
    }
    return n;
}

void orc_leaf_coords(void *h, double *xyz, int *lvl) { leaf_walk(h, xyz, lvl, NULL, NULL, 0); }
void orc_set_rhs(void *h, const double *g) { leaf_walk(h, NULL, NULL, (double *)g, NULL, 1); }
void orc_set_solution(void *h, const double *p) { leaf_walk(h, NULL, NULL, (double *)p, NULL, 0); }
void orc_get_solution(void *h, double *p) { leaf_walk(h, NULL, NULL, NULL, p, 0); }

void orc_zero_solution(void *h) {
    Orc *o = h;
    for (int il = 0; il < o->nlev; il++) {
        Level *L = &o->L[il];
        memset(L->phi, 0, sizeof(double) * (size_t)L->nblocks * L->cpb);
        memset(L->old, 0, sizeof(double) * (size_t)L->nblocks * L->cpb);
    }
}

long orc_num_iface_points(void *h) {
    Orc *o = h;
    long n = 0;
    for (int il = 0; il < o->nlev; il++) n += o->L[il].npts;
    return n;
}

void orc_iface_points(void *h, double *xyz) {
    Orc *o = h;
    long n = 0;
    for (int il = 0; il < o->nlev; il++) {
        memcpy(xyz + 3 * n, o->L[il].pts, sizeof(double) * 3 * o->L[il].npts);
        n += o->L[il].npts;
    }
}

long orc_num_domain_points(void *h) {
    Orc *o = h;
    long n = 0;
    for (int il = 0; il < o->nlev; il++) n += 2L * o->D * o->L[il].nface;
    return n;
}

/* domain face centres: level, face (x-,x+,y-,y+,z-,z+), lower tangential axis fastest */
void orc_domain_points(void *h, double *xyz) {
    Orc *o = h;
    long n = 0;
    int D = o->D;
    for (int il = 0; il < o->nlev; il++) {
        Level *L = &o->L[il];
        for (int f = 0; f < 2 * D; f++) {
            int ax = f / 2;
            for (long t = 0; t < L->nface; t++, n++) {
                int tg[2] = {(int)(t % L->n), (int)(t / L->n)};
                int m = 0;
                for (int c = 0; c < 3; c++) {
                    double v = 0.0;
                    if (c < D) {
                        if (c == ax) v = (f & 1) ? o->d.lo[c] + 1.0 : o->d.lo[c];
                        else v = centre(o, L, c, tg[m++]);
                    }
                    xyz[3 * n + c] = v;
                }
            }
        }
    }
}

/* boundary values: per interface point (phi_b(x0)) and per domain face */
void orc_set_boundary(void *h, const double *iface, const double *dom) {
    Orc *o = h;
    long pi = 0, di = 0;
    for (int il = 0; il < o->nlev; il++) {
        Level *L = &o->L[il];
        for (int r = 0; r < L->nrec; r++) {
            Rec *R = &L->rec[r];
            double b = 0.0;
            long p = pi + R->pt0;
            for (int k = 0; k < 2 * o->D; k++) {
                R->pb[k] = 0.0;
                if (!(R->cut >> k & 1)) continue;
                R->pb[k] = iface[p];
                b = b + R->c[k] * iface[p++];
            }
            R->b = b;
        }
        pi += L->npts;
        long nf = 2L * o->D * L->nface;
        memcpy(L->bcv, dom + di, sizeof(double) * nf);
        di += nf;
    }
}

/* setup export: per record blk, cell, cutmask, d[6], c[6], diag, b */
void orc_records(void *h, int il, int *ids, double *d, double *coef) {
    Level *L = &((Orc *)h)->L[il];
    for (int r = 0; r < L->nrec; r++) {
        Rec *R = &L->rec[r];
        ids[3 * r] = R->blk; ids[3 * r + 1] = R->cell; ids[3 * r + 2] = R->cut;
        for (int k = 0; k < 6; k++) { d[6 * r + k] = R->d[k]; coef[8 * r + k] = R->c[k]; }
        coef[8 * r + 6] = R->diag;
        coef[8 * r + 7] = R->b;
    }
}

/* level field access in canonical level order (blocks Morton, x-fastest):
   field 0 phi, 1 g, 2 old, 3 r */
static double *field_ptr(Level *L, int field) {
    return field == 0 ? L->phi : field == 1 ? L->g : field == 2 ? L->old : L->r;
}
void orc_get_field(void *h, int il, int field, double *out) {
    Level *L = &((Orc *)h)->L[il];
    memcpy(out, field_ptr(L, field), sizeof(double) * (size_t)L->nblocks * L->cpb);
}
void orc_set_field(void *h, int il, int field, const double *in) {
    Level *L = &((Orc *)h)->L[il];
    memcpy(field_ptr(L, field), in, sizeof(double) * (size_t)L->nblocks * L->cpb);
}

void orc_smooth(void *h, int il, int nsteps) { for (int s = 0; s < nsteps; s++) smooth_level(h, il); }
void orc_half_sweep(void *h, int il, int color) {
    /* one colour only (for kernel-level checks) */
    Orc *o = h;
    Level *L = &o->L[il];
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < L->nblocks; b++) {
        for (long li = 0; li < L->cpb; li++) {
            int g[3];
            cell_g(o, L, b, li, g);
            if (((g[0] + g[1] + g[2]) & 1) != color) continue;
            double s, dg, bt;
            stencil(o, il, L->phi, coarse_phi(o, il), b, li, &s, &dg, &bt);
            L->phi[(long)b * L->cpb + li] = (L->g[(long)b * L->cpb + li] - bt - s) / dg;
        }
    }
}
void orc_level_residual(void *h, int il) { level_residual(h, il); }
void orc_restrict_fas(void *h, int il) { restrict_fas(h, il); }
void orc_prolong(void *h, int il, int solution_mode) { prolong(h, il, solution_mode); }
void orc_restrict_rhs(void *h, int il) { restrict_rhs(h, il); }
void orc_coarse_solve(void *h) { coarse_solve(h); }
void orc_sync_down(void *h) { sync_down(h); }

void orc_vcycle(void *h) {
    Orc *o = h;
    vcycle(o, o->nlev - 1);
    sync_down(o);
}
void orc_fmg(void *h, int have_guess) {
    Orc *o = h;
    fmg(o, have_guess);
    sync_down(o);
}

/* max |r| over leaf cells of the composite grid; phi_zero != 0 evaluates
   the residual of phi = 0 (the reference for relative tolerances) */
double orc_residual_max(void *h, int phi_zero) {
    Orc *o = h;
    double **save = NULL;
    if (phi_zero) {
        save = xcalloc(o->nlev, sizeof(double *));
        for (int il = 0; il < o->nlev; il++) {
            Level *L = &o->L[il];
            size_t nc = (size_t)L->nblocks * L->cpb;
            save[il] = xcalloc(nc, sizeof(double));
            memcpy(save[il], L->phi, nc * sizeof(double));
            memset(L->phi, 0, nc * sizeof(double));
        }
    } else {
        sync_down(o);
    }
    double m = 0.0;
    for (int il = 0; il < o->nlev; il++) {
        Level *L = &o->L[il];
        level_residual(o, il);
        for (int b = 0; b < L->nblocks; b++) {
            if (!L->leaf[b]) continue;
            for (long li = 0; li < L->cpb; li++) {
                double v = fabs(L->r[(long)b * L->cpb + li]);
                if (v > m) m = v;
            }
        }
    }
    if (phi_zero) {
        for (int il = 0; il < o->nlev; il++) {
            Level *L = &o->L[il];
            memcpy(L->phi, save[il], sizeof(double) * (size_t)L->nblocks * L->cpb);
            free(save[il]);
        }
        free(save);
    }
    return m;
}

/* composite residual for a given leaf vector (dense-assembly probing) */
/* Gradient of phi at every leaf cell centre (Sec. 4.3): the derivative on
 * each cell face is (phi_nb - phi_i)/dx with the neighbour's value or ghost,
 * or (phi_b - phi_i)/(d dx) towards a boundary between the cells (taken on
 * the side of the cut link); each component is the mean of its two faces.
 * inside_zero: cells with a cut link whose centre is inside (f < 0) get 0.
 * out[n_leaf][3] in canonical leaf order. */
void orc_gradient(void *h, double *out, int inside_zero) {
    Orc *o = h;
    sync_down(o);
    long n = 0;
    for (int il = 0; il < o->nlev; il++) {
        Level *L = &o->L[il];
        const double *fc = coarse_phi(o, il);
        for (int b = 0; b < L->nblocks; b++) {
            if (!L->leaf[b]) continue;
            for (long li = 0; li < L->cpb; li++, n++) {
                long fl = (long)b * L->cpb + li;
                int g[3];
                cell_g(o, L, b, li, g);
                const Rec *R = L->rec_of[fl] >= 0 ? &L->rec[L->rec_of[fl]] : NULL;
                double phi = L->phi[fl];
                for (int c = 0; c < 3; c++) out[3 * n + c] = 0.0;
                if (inside_zero && R && R->inside) continue;
                for (int ax = 0; ax < o->D; ax++) {
                    double face[2];
                    for (int side = 0; side < 2; side++) {
                        int k = 2 * ax + side, s = side ? 1 : -1;
                        double dv;
                        if (R && (R->cut >> k & 1)) dv = (R->pb[k] - phi) / (R->d[k] * L->dx);
                        else dv = (nb_value(o, il, L->phi, fc, g, fl, ax, s) - phi) / L->dx;
                        face[side] = s * dv;  /* derivative along +axis on that face */
                    }
                    out[3 * n + ax] = 0.5 * (face[0] + face[1]);
                }
            }
        }
    }
}

void orc_leaf_residual(void *h, const double *phi_leaf, double *r_leaf) {
    Orc *o = h;
    orc_set_solution(o, phi_leaf);
    sync_down(o);
    for (int il = 0; il < o->nlev; il++) level_residual(o, il);
    leaf_walk(o, NULL, NULL, NULL, r_leaf, 3);
}

/* standalone line search for unit tests (level-set spec as in orc_desc) */
double orc_line_search(const orc_desc *d, const double *a, const double *b, int *found) {
    Orc o;
    memset(&o, 0, sizeof o);
    o.d = *d;
    o.D = d->dim;
    o.lsfp = (double *)d->lsf_params;
    o.nbisect = (int)ceil(-log(d->eps_tol) / log(2.0));
    o.ngolden = (int)ceil(log(d->eps_tol) / log(0.5 * (sqrt(5.0) - 1.0)));
    double fa = lsf(&o, a);
    return line_search(&o, a, b, fa, found);
}

double orc_cbrt(double a) { return cbrt_exact_ops(a); }

double orc_lsf(const orc_desc *d, const double *x) {
    Orc o;
    memset(&o, 0, sizeof o);
    o.d = *d;
    o.D = d->dim;
    o.lsfp = (double *)d->lsf_params;
    return lsf(&o, x);
}

/* standalone coarse-grid search for unit tests: cell centre a, spacing dx */
int orc_coarse_search(const orc_desc *d, const double *a, double dx, double *dout, int *dir, double *x0) {
    Orc o;
    memset(&o, 0, sizeof o);
    o.d = *d;
    o.D = d->dim;
    o.lsfp = (double *)d->lsf_params;
    o.nbisect = (int)ceil(-log(d->eps_tol) / log(2.0));
    o.ngolden = (int)ceil(log(d->eps_tol) / log(0.5 * (sqrt(5.0) - 1.0)));
    Level L;
    memset(&L, 0, sizeof L);
    L.dx = dx;
    return coarse_search(&o, &L, a, lsf(&o, a), dout, dir, x0);
}

/* OpenMP threads of the oracle's parallel loops (timing only: every loop
 * writes disjoint cells, so the results do not depend on the count) */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_get_threads(void) { return omp_get_max_threads(); }
