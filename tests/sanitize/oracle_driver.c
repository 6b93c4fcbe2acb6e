/* Sanitizer driver for the FP64 oracle (test infrastructure).  Reads a raw mesh
 * written by tests/test_sanitizers_cpu.py and calls every exported oracle
 * function on it; built with -fsanitize=address,undefined, a memory or
 * undefined-behaviour error aborts with a report.  Prints the FP64 mass after
 * the steps, for the test to compare with the unsanitized oracle. */
#include <stdio.h>
#include <stdlib.h>

typedef struct oracle oracle_t;
oracle_t *orc_create(int n_nodes, const double *xy, int n_cells, const int *cell_ptr, const int *cell_nodes,
                     int n_bf, const int *bface_nodes, const int *bface_group, int n_groups, const int *g_kind,
                     const int *g_internal, const double *g_u, const double *g_rho, int n_per, const int *per_pairs,
                     const double *per_shift, double tau, double dt, double cfl, double u_ref, int scheme, char *err,
                     int errlen);
void orc_destroy(oracle_t *o);
int orc_n_cells(const oracle_t *o);
double orc_dt(const oracle_t *o);
long orc_steps(const oracle_t *o);
int orc_maxf(void);
void orc_feq(double rho, double ux, double uy, double *out);
void orc_moments(const double *f, double *rho, double *ux, double *uy);
void orc_lattice(double *ex, double *ey, double *w);
void orc_geometry(const oracle_t *o, double *area, double *cx, double *cy, double *lx, double *ly, int *nf);
void orc_faces(const oracle_t *o, int *nbr, int *grp, double *fx, double *fy, double *nx, double *ny, double *len,
               double *stx, double *sty);
void orc_lsq_gradient(const oracle_t *o, const double *phi, const double *phi_bnd, double *grad);
void orc_rhs(const oracle_t *o, const double *f, double *rhs);
void orc_face_values(const oracle_t *o, const double *f, double *face_out);
int orc_wall_force(const oracle_t *o, const double *f, int g, double *force, double *face_p);
void orc_init(oracle_t *o, const double *rho, const double *u, double rho0, double ux0, double uy0);
void orc_set_f(oracle_t *o, const double *f);
void orc_get_f(const oracle_t *o, double *f);
void orc_step(oracle_t *o, long n);
void orc_macros(const oracle_t *o, double *rho, double *u);
double orc_mass(const oracle_t *o);
double orc_residual(int n, const double *u, const double *u_old);

static void *rd(FILE *fp, size_t n, size_t sz) {
    void *p = malloc(n * sz > 0 ? n * sz : 1);
    if (n && fread(p, sz, n, fp) != n) { fprintf(stderr, "short mesh file\n"); exit(2); }
    return p;
}

int main(int argc, char **argv) {
    if (argc < 6) { fprintf(stderr, "usage: mesh tau scheme steps wall_group\n"); return 2; }
    FILE *fp = fopen(argv[1], "rb");
    if (!fp) return 2;
    int h[6];   /* nodes, cells, cell-node entries, boundary faces, groups, periodic pairs */
    if (fread(h, sizeof(int), 6, fp) != 6) return 2;
    double *xy = rd(fp, 2 * (size_t)h[0], sizeof(double));
    int *cptr = rd(fp, (size_t)h[1] + 1, sizeof(int)), *cn = rd(fp, (size_t)h[2], sizeof(int));
    int *bfn = rd(fp, 2 * (size_t)h[3], sizeof(int)), *bfg = rd(fp, (size_t)h[3], sizeof(int));
    int *gk = rd(fp, (size_t)h[4], sizeof(int)), *gi = rd(fp, (size_t)h[4], sizeof(int));
    double *gu = rd(fp, 2 * (size_t)h[4], sizeof(double)), *gr = rd(fp, (size_t)h[4], sizeof(double));
    int *pp = rd(fp, 2 * (size_t)h[5], sizeof(int));
    double *ps = rd(fp, 2 * (size_t)h[5], sizeof(double));
    fclose(fp);
    char err[256];
    const double tau = atof(argv[2]);
    const int scheme = atoi(argv[3]), wall = atoi(argv[5]);
    const long steps = atol(argv[4]);
    oracle_t *o = orc_create(h[0], xy, h[1], cptr, cn, h[3], bfn, bfg, h[4], gk, gi, gu, gr, h[5], pp, ps, tau, 0.0,
                             0.5, 0.2, scheme, err, 256);
    if (!o) {
        printf("rejected: %s\n", err);
        free(xy); free(cptr); free(cn); free(bfn); free(bfg); free(gk); free(gi); free(gu); free(gr); free(pp); free(ps);
        return 3;
    }
    const int n = orc_n_cells(o), M = orc_maxf(), Q = 9;
    double *a = malloc(sizeof(double) * n * 5), *fc = malloc(sizeof(double) * n * M * 7);
    int *nf = malloc(sizeof(int) * n), *ib = malloc(sizeof(int) * n * M * 2);
    orc_geometry(o, a, a + n, a + 2 * n, a + 3 * n, a + 4 * n, nf);
    orc_faces(o, ib, ib + n * M, fc, fc + n * M, fc + 2 * n * M, fc + 3 * n * M, fc + 4 * n * M, fc + 5 * n * M,
              fc + 6 * n * M);
    double ex[9], ey[9], w[9], fe[9], r, ux, uy;
    orc_lattice(ex, ey, w);
    orc_feq(1.0, 0.05, -0.02, fe);
    orc_moments(fe, &r, &ux, &uy);
    orc_init(o, NULL, NULL, 1.0, 0.0, 0.0);
    orc_step(o, steps);
    double *f = malloc(sizeof(double) * n * Q), *g = malloc(sizeof(double) * n * Q * M);
    double *rho = malloc(sizeof(double) * n), *u = malloc(sizeof(double) * n * 2), *u0 = calloc(2 * (size_t)n, sizeof(double));
    orc_get_f(o, f);
    orc_rhs(o, f, g);
    orc_face_values(o, f, g);
    double *phi = malloc(sizeof(double) * n), *pb = calloc((size_t)n * M, sizeof(double)), *gr2 = malloc(sizeof(double) * n * 2);
    for (int i = 0; i < n; i++) phi[i] = a[n + i] + 2.0 * a[2 * n + i];
    orc_lsq_gradient(o, phi, pb, gr2);
    if (wall >= 0) {
        double force[2];
        double *fp2 = malloc(sizeof(double) * 4 * n);
        orc_wall_force(o, f, wall, force, fp2);
        free(fp2);
    }
    orc_set_f(o, f);
    orc_macros(o, rho, u);
    const double res = orc_residual(n, u, u0);
    printf("cells %d steps %ld dt %.17g mass %.17g residual %.17g\n", n, orc_steps(o), orc_dt(o), orc_mass(o), res);
    orc_destroy(o);
    free(xy); free(cptr); free(cn); free(bfn); free(bfg); free(gk); free(gi); free(gu); free(gr); free(pp); free(ps);
    free(a); free(fc); free(nf); free(ib); free(f); free(g); free(rho); free(u); free(u0); free(phi); free(pb); free(gr2);
    return 0;
}
