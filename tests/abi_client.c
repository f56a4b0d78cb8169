/*
 * A C99 client of the octmg C ABI (include/octmg.h), built and run by
 * tests/test_abi_client.py.  It uses only the header and the shared library.
 *
 *   abi_client plan    host-only tree planning (no device): prints the level
 *                      table of a 256^3 tree in 16^3 blocks
 *   abi_client solve   on device 0: the 64^3 manufactured sphere problem
 *                      (phi = exp(x) sin(pi y) cos(pi z), sphere r = 0.3 at
 *                      the centre, Dirichlet data from phi on the sphere and
 *                      the cube) solved to 1e-10 with the built-in level set
 *                      and again with the same level set given as a C
 *                      function; prints the cycles, the error against phi
 *                      and whether the two solutions are equal bit for bit
 *
 * Exit status 0 on success, 1 with a message on stderr otherwise.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "octmg.h"

#define CHECK(call)                                                                   \
    do {                                                                              \
        octmg_status st_ = (call);                                                    \
        if (st_ != OCTMG_OK) {                                                        \
            fprintf(stderr, "%s failed (%d): %s\n", #call, (int)st_, octmg_last_error()); \
            exit(1);                                                                  \
        }                                                                             \
    } while (0)

static const double kPi = 3.14159265358979323846;
static const double kSphere[4] = {0.5, 0.5, 0.5, 0.3};

static double exact(const double *x) { return exp(x[0]) * sin(kPi * x[1]) * cos(kPi * x[2]); }
static double rhs(const double *x) { return (1.0 - 2.0 * kPi * kPi) * exact(x); }

/* the sphere's level set as the library's built-in kind writes it: the
 * distance to the centre (sum of squares in x, y, z order), minus r */
static double sphere_lsf(const double *x, void *user) {
    const double *p = (const double *)user;
    const double ex = x[0] - p[0], ey = x[1] - p[1], ez = x[2] - p[2];
    return sqrt(ex * ex + ey * ey + ez * ez) - p[3];
}

static octmg_geom_desc describe(int max_level) {
    octmg_geom_desc d;
    memset(&d, 0, sizeof d);
    d.dim = 3;
    d.block_n = 16;
    d.max_level = max_level;
    d.refine_kind = OCTMG_REFINE_UNIFORM;
    d.lsf_kind = OCTMG_LSF_SPHERES;
    d.lsf_n = 1;
    d.coarse_n = 8;
    d.eps_tol = 1e-8;
    d.mask_factor = 1.5;
    d.w_min = 8e-3;
    d.lsf_params = kSphere;
    return d;
}

static int plan(void) {
    octmg_geom_desc d = describe(5);
    int n_levels = 0;
    int64_t info[4 * 24];
    CHECK(octmg_plan_levels(&d, &n_levels, info));
    printf("levels %d\n", n_levels);
    for (int l = 0; l < n_levels; l++)
        printf("level %d n %lld block %lld blocks %lld leaf_blocks %lld\n", l, (long long)info[4 * l],
               (long long)info[4 * l + 1], (long long)info[4 * l + 2], (long long)info[4 * l + 3]);
    return 0;
}

/* solve the manufactured problem on geometry g; the solution in *phi_out
 * (malloc'ed), the cycle count in *cycles, the max error in *err */
static void solve_on(octmg_geom g, double **phi_out, int *cycles, double *err) {
    int64_t gi[8];
    CHECK(octmg_geom_info(g, gi));
    const long long n_leaf = gi[1], n_iface = gi[2], n_dom = gi[3];
    double *xyz = malloc(sizeof(double) * 3 * (size_t)n_leaf);
    int *lev = malloc(sizeof(int) * (size_t)n_leaf);
    double *ip = malloc(sizeof(double) * 3 * (size_t)(n_iface > 0 ? n_iface : 1));
    double *dp = malloc(sizeof(double) * 3 * (size_t)n_dom);
    double *iv = malloc(sizeof(double) * (size_t)(n_iface > 0 ? n_iface : 1));
    double *dv = malloc(sizeof(double) * (size_t)n_dom);
    double *g_rhs = malloc(sizeof(double) * (size_t)n_leaf);
    double *phi = malloc(sizeof(double) * (size_t)n_leaf);
    if (!xyz || !lev || !ip || !dp || !iv || !dv || !g_rhs || !phi) {
        fprintf(stderr, "out of host memory\n");
        exit(1);
    }
    CHECK(octmg_geom_leaf_coords(g, xyz, lev));
    CHECK(octmg_geom_iface_points(g, ip));
    CHECK(octmg_geom_domain_points(g, dp));
    for (long long i = 0; i < n_iface; i++) iv[i] = exact(ip + 3 * i);
    for (long long i = 0; i < n_dom; i++) dv[i] = exact(dp + 3 * i);
    for (long long i = 0; i < n_leaf; i++) g_rhs[i] = rhs(xyz + 3 * i);

    octmg_state s = NULL;
    CHECK(octmg_state_create(g, 1, OCTMG_FP64, &s));
    CHECK(octmg_set_boundary(s, iv, dv, 0, NULL));
    CHECK(octmg_set_rhs(s, g_rhs, OCTMG_DTYPE_F64, 0, NULL));
    octmg_solve_opts o;
    memset(&o, 0, sizeof o);
    o.cycle_kind = OCTMG_CYCLE_V;
    o.max_cycles = 40;
    o.zero_start = 1;
    o.graph_mode = 0;
    o.rtol = 1e-10;
    octmg_solve_report rep;
    memset(&rep, 0, sizeof rep);
    CHECK(octmg_solve(s, &o, NULL, &rep));
    CHECK(octmg_get_solution(s, phi, OCTMG_DTYPE_F64, 0, NULL));
    double e = 0.0;
    for (long long i = 0; i < n_leaf; i++) {
        const double di = fabs(phi[i] - exact(xyz + 3 * i));
        if (di > e) e = di;
    }
    *cycles = rep.cycles;
    *err = e;
    *phi_out = phi;
    octmg_state_destroy(s);
    free(xyz);
    free(lev);
    free(ip);
    free(dp);
    free(iv);
    free(dv);
    free(g_rhs);
}

static int solve(void) {
    octmg_geom_desc d = describe(3);
    octmg_geom g = NULL;
    CHECK(octmg_geom_create(&d, 0, &g));
    int64_t gi[8];
    CHECK(octmg_geom_info(g, gi));
    double *phi_a = NULL, *phi_b = NULL;
    int cyc_a = 0, cyc_b = 0;
    double err_a = 0.0, err_b = 0.0;
    solve_on(g, &phi_a, &cyc_a, &err_a);

    /* the same level set as a host function */
    octmg_geom_desc dc = d;
    dc.lsf_kind = OCTMG_LSF_CALLBACK;
    dc.lsf_n = 0;
    dc.lsf_params = NULL;
    dc.lsf_fn = sphere_lsf;
    dc.lsf_user = (void *)kSphere;
    octmg_geom gc = NULL;
    CHECK(octmg_geom_create(&dc, 0, &gc));
    solve_on(gc, &phi_b, &cyc_b, &err_b);
    const long long n_leaf = gi[1];
    const int same = memcmp(phi_a, phi_b, sizeof(double) * (size_t)n_leaf) == 0;
    printf("leaf %lld records %lld cycles %d err %.6e callback_cycles %d callback_bitwise_equal %d\n", n_leaf,
           (long long)gi[4], cyc_a, err_a, cyc_b, same);
    free(phi_a);
    free(phi_b);
    octmg_geom_destroy(gc);
    octmg_geom_destroy(g);
    return 0;
}

int main(int argc, char **argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s plan|solve\n", argv[0]);
        return 1;
    }
    if (strcmp(argv[1], "plan") == 0) return plan();
    if (strcmp(argv[1], "solve") == 0) return solve();
    fprintf(stderr, "unknown mode %s\n", argv[1]);
    return 1;
}
