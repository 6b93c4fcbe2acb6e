/*
 * FP64 CPU oracle for the cell-centred finite-volume lattice Boltzmann method
 * (D2Q9, BGK) on 2D unstructured meshes of convex polygons.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the HIP library; both only read the same raw meshes.
 *
 * Written from the paper's Section 2 in the paper's step order:
 *   Step 0  f = f^eq(rho0, u0)                                  (Eq. 3)
 *   Step 1  wall values f_P and ghost values f_GC               (Eqs. 18-22)
 *   Step 2  weighted least-squares gradient of every f_alpha    (Eq. 12)
 *   Step 3  border-face values                                  (Eqs. 23-26)
 *   Step 4  RHS = -(1/A) sum_m (e.n) f_face dl - (f - f^eq)/tau  (Eqs. 10, 11)
 *   Step 5  forward Euler (Eq. 13), AB2 (Eq. 16) or four-stage RK (Eq. 17)
 *   Step 6  rho, u, p                                           (Eq. 5)
 * Plain loops, original cell order, faces in node order, alpha ascending,
 * compiled with -ffp-contract=off so no fused multiply-add changes rounding.
 *
 * Timing build: the same file compiled with -fopenmp runs the per-cell loops
 * of the operator and the integrator on several threads (the pragmas below).
 * Every iteration writes only its own cell's values and reads values that no
 * iteration of the same loop writes, and each cell's sums keep their order,
 * so that build's results are bitwise those of the one-thread build.
 *
 * Readings where the paper is silent or garbled (each also listed in the
 * design notes):
 *  - f lives at the polygon's area centroid (Section 2.2); area and centroid
 *    are formed on the corners relative to the cell's first corner.
 *  - The least-squares stencil is the face neighbours; a wall face contributes
 *    its midpoint P with value f_P; inlet/outlet/symmetry faces contribute a
 *    ghost at the mirror image of the cell centre across the face line;
 *    a periodic face contributes the neighbour at its shifted image.
 *  - A wall face carries f_P for every direction (incoming and outgoing).
 *  - Boundary formulas use the border cell's current-stage rho, u, f.
 *  - The four-stage RK reads f(k+1) = f(0) + beta_(k+1) dt RHS(f(k)): RHS is
 *    df/dt (Eq. 9), the printed minus sign and missing dt are the residual
 *    convention of the cited scheme.
 *  - CFL time step: min over cells of A/(Lx+Ly) with Lx, Ly the cell's
 *    bounding-box extents, |e|max = sqrt(2), |U|max = the reference speed;
 *    the final dt is the smaller of that and 2 tau (Eqs. 14, 15).
 *  - Velocity residual: sqrt(sum du^2+dv^2) / sqrt(sum u^2+v^2)  (Eq. 32).
 *  - Mass: sum_i A_i rho_i.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define Q 9
#define MAXF 8

enum { BC_WALL = 1, BC_INLET = 2, BC_OUTLET = 3, BC_SYMMETRY = 4 };
enum { SCHEME_EULER = 0, SCHEME_RK4 = 1, SCHEME_AB2 = 2 };

/* D2Q9 lattice, Eq. (2) with c = 1 evaluated exactly, and weights Eq. (4). */
static const double EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const double EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[Q] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

typedef struct {
    int kind, internal;
    double ux, uy, rho;
} group_t;

typedef struct {
    int n_cells;
    int *nf;                 /* faces per cell */
    /* per (cell, face slot), index c*MAXF + k */
    int *nbr;                /* neighbour cell, or -1 on a boundary face */
    int *grp;                /* boundary group, or -1 */
    double *shx, *shy;       /* shift added to the neighbour centre (periodic image) */
    double *fx, *fy;         /* face midpoint */
    double *nx, *ny, *len;   /* outward unit normal and length */
    double *stx, *sty;       /* least-squares stencil point */
    /* per cell */
    double *area, *cx, *cy, *lx, *ly;
    double *m11, *m12, *m22; /* inverse of the least-squares matrix */
    group_t *groups;
    int n_groups;
    double tau, dt;
    int scheme;
    double *f, *tmp0, *tmp1, *rhs_prev;
    int n_bf;                /* boundary faces as given, and the (cell * MAXF + slot) each lies on */
    int *bf_slot;
    int *bf_group;
    int have_prev;
    long steps;
} oracle_t;

/* ------------------------------------------------------------------ */
/* lattice functions                                                    */
/* ------------------------------------------------------------------ */

/* Eq. (3): f_eq = rho w [1 + e.u/cs2 + (e.u)^2/(2 cs2^2) - u^2/(2 cs2)], cs2 = 1/3. */
void orc_feq(double rho, double ux, double uy, double *out) {
    double uu = ux * ux + uy * uy;
    for (int a = 0; a < Q; a++) {
        double eu = EX[a] * ux + EY[a] * uy;
        out[a] = rho * W[a] * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

/* Eq. (5): rho = sum f, rho u = sum f e. */
void orc_moments(const double *f, double *rho, double *ux, double *uy) {
    double r = 0, mx = 0, my = 0;
    for (int a = 0; a < Q; a++) {
        r += f[a];
        mx += f[a] * EX[a];
        my += f[a] * EY[a];
    }
    *rho = r;
    *ux = mx / r;
    *uy = my / r;
}

void orc_lattice(double *ex, double *ey, double *w) {
    for (int a = 0; a < Q; a++) { ex[a] = EX[a]; ey[a] = EY[a]; w[a] = W[a]; }
}

/* ------------------------------------------------------------------ */
/* mesh, topology and geometry                                          */
/* ------------------------------------------------------------------ */

typedef struct { int64_t key; int cell, slot; } edge_t;

static int edge_cmp(const void *a, const void *b) {
    const edge_t *x = (const edge_t *)a, *y = (const edge_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
    return x->slot - y->slot;
}

static int64_t edge_key(int a, int b) {
    int lo = a < b ? a : b, hi = a < b ? b : a;
    return ((int64_t)lo << 32) | (int64_t)(uint32_t)hi;
}

/* Find the (cell, slot) holding edge `key` in the sorted list, or -1. */
static int find_edge(const edge_t *e, int n, int64_t key, int skip_cell) {
    int lo = 0, hi = n - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (e[mid].key < key) lo = mid + 1;
        else if (e[mid].key > key) hi = mid - 1;
        else {
            int s = mid;
            while (s > 0 && e[s - 1].key == key) s--;
            for (; s < n && e[s].key == key; s++)
                if (e[s].cell != skip_cell) return s;
            return -1;
        }
    }
    return -1;
}

void orc_destroy(oracle_t *o);

static void set_err(char *err, int errlen, const char *msg) {
    if (err && errlen > 0) { strncpy(err, msg, (size_t)errlen - 1); err[errlen - 1] = 0; }
}

oracle_t *orc_create(int n_nodes, const double *xy, int n_cells, const int *cell_ptr,
                     const int *cell_nodes, int n_bf, const int *bface_nodes,
                     const int *bface_group, int n_groups, const int *g_kind,
                     const int *g_internal, const double *g_u, const double *g_rho,
                     int n_per, const int *per_pairs, const double *per_shift,
                     double tau, double dt, double cfl, double u_ref, int scheme,
                     char *err, int errlen) {
    oracle_t *o = (oracle_t *)calloc(1, sizeof(oracle_t));
    int N = n_cells, NS = n_cells * MAXF;
    o->n_cells = N;
    o->nf = (int *)calloc(N, sizeof(int));
    o->nbr = (int *)malloc(NS * sizeof(int));
    o->grp = (int *)malloc(NS * sizeof(int));
    double **arrs[] = {&o->shx, &o->shy, &o->fx, &o->fy, &o->nx, &o->ny, &o->len, &o->stx, &o->sty};
    for (unsigned i = 0; i < sizeof(arrs) / sizeof(arrs[0]); i++) *arrs[i] = (double *)calloc(NS, sizeof(double));
    double **carr[] = {&o->area, &o->cx, &o->cy, &o->lx, &o->ly, &o->m11, &o->m12, &o->m22};
    for (unsigned i = 0; i < sizeof(carr) / sizeof(carr[0]); i++) *carr[i] = (double *)calloc(N, sizeof(double));
    o->n_groups = n_groups;
    o->groups = (group_t *)calloc(n_groups > 0 ? n_groups : 1, sizeof(group_t));
    for (int g = 0; g < n_groups; g++) {
        o->groups[g].kind = g_kind[g];
        o->groups[g].internal = g_internal[g];
        o->groups[g].ux = g_u[2 * g];
        o->groups[g].uy = g_u[2 * g + 1];
        o->groups[g].rho = g_rho[g];
    }
    o->tau = tau;
    o->scheme = scheme;
    o->f = (double *)calloc((size_t)N * Q, sizeof(double));
    o->tmp0 = (double *)calloc((size_t)N * Q, sizeof(double));
    o->tmp1 = (double *)calloc((size_t)N * Q, sizeof(double));
    o->rhs_prev = (double *)calloc((size_t)N * Q, sizeof(double));
    for (int i = 0; i < NS; i++) { o->nbr[i] = -1; o->grp[i] = -1; }

    /* cell geometry: shoelace area and area centroid (Section 2.2), bbox extents.
     * The corners are taken relative to the cell's first node (ox, oy): the same
     * area and centroid in exact arithmetic, but the cross products then scale
     * with the cell's size rather than its distance from the origin, which for a
     * small cell far from the origin would cancel away most of their digits. */
    for (int c = 0; c < N; c++) {
        int p0 = cell_ptr[c], m = cell_ptr[c + 1] - p0;
        if (m < 3 || m > MAXF) { set_err(err, errlen, "cell with fewer than 3 or more than 8 nodes"); orc_destroy(o); return NULL; }
        o->nf[c] = m;
        double a2 = 0, sx = 0, sy = 0;
        double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
        const double ox = xy[2 * cell_nodes[p0]], oy = xy[2 * cell_nodes[p0] + 1];
        for (int k = 0; k < m; k++) {
            int na = cell_nodes[p0 + k], nb = cell_nodes[p0 + (k + 1) % m];
            double xa = xy[2 * na] - ox, ya = xy[2 * na + 1] - oy, xb = xy[2 * nb] - ox, yb = xy[2 * nb + 1] - oy;
            double cr = xa * yb - xb * ya;
            a2 += cr;
            sx += (xa + xb) * cr;
            sy += (ya + yb) * cr;
            if (xa < xmin) xmin = xa;
            if (xa > xmax) xmax = xa;
            if (ya < ymin) ymin = ya;
            if (ya > ymax) ymax = ya;
        }
        if (!(a2 > 0)) { set_err(err, errlen, "cell with non-positive area (not CCW)"); orc_destroy(o); return NULL; }
        o->area[c] = 0.5 * a2;
        o->cx[c] = ox + sx / (3.0 * a2);
        o->cy[c] = oy + sy / (3.0 * a2);
        o->lx[c] = xmax - xmin;
        o->ly[c] = ymax - ymin;
        for (int k = 0; k < m; k++) {
            int na = cell_nodes[p0 + k], nb = cell_nodes[p0 + (k + 1) % m];
            double dx = xy[2 * nb] - xy[2 * na], dy = xy[2 * nb + 1] - xy[2 * na + 1];
            double l = sqrt(dx * dx + dy * dy);
            int s = c * MAXF + k;
            o->len[s] = l;
            o->nx[s] = dy / l;            /* outward for a CCW polygon */
            o->ny[s] = -dx / l;
            o->fx[s] = 0.5 * (xy[2 * na] + xy[2 * nb]);
            o->fy[s] = 0.5 * (xy[2 * na + 1] + xy[2 * nb + 1]);
        }
    }

    /* topology: match every cell edge with another cell or a boundary edge */
    int ne = cell_ptr[N];
    edge_t *edges = (edge_t *)malloc((size_t)ne * sizeof(edge_t));
    for (int c = 0, q = 0; c < N; c++) {
        int p0 = cell_ptr[c], m = o->nf[c];
        for (int k = 0; k < m; k++, q++) {
            edges[q].key = edge_key(cell_nodes[p0 + k], cell_nodes[p0 + (k + 1) % m]);
            edges[q].cell = c;
            edges[q].slot = k;
        }
    }
    qsort(edges, (size_t)ne, sizeof(edge_t), edge_cmp);
    for (int q = 0; q < ne; q++) {
        int cnt = 1;
        while (q + cnt < ne && edges[q + cnt].key == edges[q].key) cnt++;
        if (cnt > 2) { free(edges); set_err(err, errlen, "edge shared by more than two cells"); orc_destroy(o); return NULL; }
        if (cnt == 2) {
            int s0 = edges[q].cell * MAXF + edges[q].slot, s1 = edges[q + 1].cell * MAXF + edges[q + 1].slot;
            o->nbr[s0] = edges[q + 1].cell;
            o->nbr[s1] = edges[q].cell;
        }
        q += cnt - 1;
    }
    /* boundary edges: groups */
    int *bf_slot = (int *)malloc((n_bf > 0 ? n_bf : 1) * sizeof(int));
    for (int b = 0; b < n_bf; b++) {
        int64_t key = edge_key(bface_nodes[2 * b], bface_nodes[2 * b + 1]);
        int e = find_edge(edges, ne, key, -1);
        if (e < 0) { free(edges); free(bf_slot); set_err(err, errlen, "boundary edge not found in any cell"); orc_destroy(o); return NULL; }
        int s = edges[e].cell * MAXF + edges[e].slot;
        if (o->nbr[s] >= 0) { free(edges); free(bf_slot); set_err(err, errlen, "boundary edge is interior"); orc_destroy(o); return NULL; }
        bf_slot[b] = s;
        int g = bface_group[b];
        if (g >= n_groups) { free(edges); free(bf_slot); set_err(err, errlen, "bad boundary group"); orc_destroy(o); return NULL; }
        o->grp[s] = g;
    }
    /* periodic pairs: the face on edge a sees the owner of b shifted by `shift`, and vice versa */
    for (int p = 0; p < n_per; p++) {
        int a = per_pairs[2 * p], b = per_pairs[2 * p + 1];
        if (a < 0 || b < 0 || a >= n_bf || b >= n_bf) { free(edges); free(bf_slot); set_err(err, errlen, "bad periodic pair"); orc_destroy(o); return NULL; }
        int sa = bf_slot[a], sb = bf_slot[b];
        o->nbr[sa] = sb / MAXF;  o->shx[sa] = per_shift[2 * p];  o->shy[sa] = per_shift[2 * p + 1];
        o->nbr[sb] = sa / MAXF;  o->shx[sb] = -per_shift[2 * p]; o->shy[sb] = -per_shift[2 * p + 1];
        o->grp[sa] = -1; o->grp[sb] = -1;
    }
    free(edges);
    o->n_bf = n_bf;
    o->bf_slot = bf_slot;
    o->bf_group = (int *)malloc((n_bf > 0 ? n_bf : 1) * sizeof(int));
    for (int b = 0; b < n_bf; b++) o->bf_group[b] = bface_group[b];
    for (int c = 0; c < N; c++)
        for (int k = 0; k < o->nf[c]; k++) {
            int s = c * MAXF + k;
            if (o->nbr[s] < 0 && o->grp[s] < 0) { set_err(err, errlen, "open boundary edge without a group"); orc_destroy(o); return NULL; }
        }

    /* least-squares stencil points and matrices (Eq. 12) */
    for (int c = 0; c < N; c++) {
        double a = 0, b = 0, d = 0;
        for (int k = 0; k < o->nf[c]; k++) {
            int s = c * MAXF + k;
            if (o->nbr[s] >= 0) {
                o->stx[s] = o->cx[o->nbr[s]] + o->shx[s];
                o->sty[s] = o->cy[o->nbr[s]] + o->shy[s];
            } else if (o->groups[o->grp[s]].kind == BC_WALL) {
                o->stx[s] = o->fx[s];          /* wall-face centre P */
                o->sty[s] = o->fy[s];
            } else {                           /* ghost: mirror of the centre across the face */
                double dn = (o->fx[s] - o->cx[c]) * o->nx[s] + (o->fy[s] - o->cy[c]) * o->ny[s];
                o->stx[s] = o->cx[c] + 2.0 * dn * o->nx[s];
                o->sty[s] = o->cy[c] + 2.0 * dn * o->ny[s];
            }
            double dx = o->stx[s] - o->cx[c], dy = o->sty[s] - o->cy[c];
            double w = 1.0 / (dx * dx + dy * dy);
            a += w * dx * dx;
            b += w * dx * dy;
            d += w * dy * dy;
        }
        double det = a * d - b * b;
        if (!(det > 1e-12 * (a + d) * (a + d))) { set_err(err, errlen, "singular least-squares stencil"); orc_destroy(o); return NULL; }
        o->m11[c] = d / det;
        o->m12[c] = -b / det;
        o->m22[c] = a / det;
    }

    /* time step, Eqs. (14)-(15) */
    if (dt > 0) {
        o->dt = dt;
    } else {
        double amin = 1e300;
        for (int c = 0; c < N; c++) {
            double r = o->area[c] / (o->lx[c] + o->ly[c]);
            if (r < amin) amin = r;
        }
        double dcfl = cfl * amin / (sqrt(2.0) + u_ref);
        o->dt = dcfl < 2.0 * tau ? dcfl : 2.0 * tau;
    }
    return o;
}

void orc_destroy(oracle_t *o) {
    if (!o) return;
    free(o->nf); free(o->nbr); free(o->grp);
    free(o->shx); free(o->shy); free(o->fx); free(o->fy); free(o->nx); free(o->ny); free(o->len);
    free(o->stx); free(o->sty);
    free(o->area); free(o->cx); free(o->cy); free(o->lx); free(o->ly);
    free(o->m11); free(o->m12); free(o->m22);
    free(o->groups); free(o->f); free(o->tmp0); free(o->tmp1); free(o->rhs_prev);
    free(o->bf_slot); free(o->bf_group);
    free(o);
}

int orc_n_cells(const oracle_t *o) { return o->n_cells; }
double orc_dt(const oracle_t *o) { return o->dt; }
long orc_steps(const oracle_t *o) { return o->steps; }
int orc_maxf(void) { return MAXF; }

void orc_geometry(const oracle_t *o, double *area, double *cx, double *cy, double *lx, double *ly, int *nf) {
    for (int c = 0; c < o->n_cells; c++) {
        area[c] = o->area[c]; cx[c] = o->cx[c]; cy[c] = o->cy[c];
        lx[c] = o->lx[c]; ly[c] = o->ly[c]; nf[c] = o->nf[c];
    }
}

void orc_faces(const oracle_t *o, int *nbr, int *grp, double *fx, double *fy, double *nx,
               double *ny, double *len, double *stx, double *sty) {
    size_t n = (size_t)o->n_cells * MAXF;
    memcpy(nbr, o->nbr, n * sizeof(int)); memcpy(grp, o->grp, n * sizeof(int));
    memcpy(fx, o->fx, n * sizeof(double)); memcpy(fy, o->fy, n * sizeof(double));
    memcpy(nx, o->nx, n * sizeof(double)); memcpy(ny, o->ny, n * sizeof(double));
    memcpy(len, o->len, n * sizeof(double));
    memcpy(stx, o->stx, n * sizeof(double)); memcpy(sty, o->sty, n * sizeof(double));
}

/* ------------------------------------------------------------------ */
/* the operator                                                         */
/* ------------------------------------------------------------------ */

/* Eq. (12): gradient = M^-1 sum_n w_n d_n (phi_n - phi_i), for one scalar field. */
static void lsq_gradient(const oracle_t *o, int c, double phi_c, const double *phi_st, double *gx, double *gy) {
    double bx = 0, by = 0;
    for (int k = 0; k < o->nf[c]; k++) {
        int s = c * MAXF + k;
        double dx = o->stx[s] - o->cx[c], dy = o->sty[s] - o->cy[c];
        double w = 1.0 / (dx * dx + dy * dy);
        bx += w * dx * (phi_st[k] - phi_c);
        by += w * dy * (phi_st[k] - phi_c);
    }
    *gx = o->m11[c] * bx + o->m12[c] * by;
    *gy = o->m12[c] * bx + o->m22[c] * by;
}

/* Gradient of one scalar field given per-cell values and values at the
 * boundary stencil points (slot c*MAXF+k, read only where the slot has no
 * neighbour cell).  Exposed so tests can check exactness on linear fields. */
void orc_lsq_gradient(const oracle_t *o, const double *phi, const double *phi_bnd, double *grad) {
    double st[MAXF];
    for (int c = 0; c < o->n_cells; c++) {
        for (int k = 0; k < o->nf[c]; k++) {
            int s = c * MAXF + k;
            st[k] = o->nbr[s] >= 0 ? phi[o->nbr[s]] : phi_bnd[s];
        }
        lsq_gradient(o, c, phi[c], st, &grad[2 * c], &grad[2 * c + 1]);
    }
}

/* Steps 1-4 for the whole mesh.  f, rhs: [cell*9 + alpha].  If face_out is
 * not NULL it receives the face values [ (cell*MAXF + k)*9 + alpha ]. */
static void operator_rhs(const oracle_t *o, const double *f, double *rhs, double *face_out) {
    int N = o->n_cells;
    double *rho = (double *)malloc(N * sizeof(double));
    double *ux = (double *)malloc(N * sizeof(double));
    double *uy = (double *)malloc(N * sizeof(double));
    double *feq = (double *)malloc((size_t)N * Q * sizeof(double));
    double *bval = (double *)calloc((size_t)N * MAXF * Q, sizeof(double));   /* f_P or f_GC per slot */
    double *gx = (double *)malloc((size_t)N * Q * sizeof(double));
    double *gy = (double *)malloc((size_t)N * Q * sizeof(double));

    /* macroscopic values and equilibrium of every cell (Eqs. 3, 5) */
#pragma omp parallel for schedule(static)
    for (int c = 0; c < N; c++) {
        orc_moments(&f[c * Q], &rho[c], &ux[c], &uy[c]);
        orc_feq(rho[c], ux[c], uy[c], &feq[c * Q]);
    }
    /* Step 1 and the ghost values of Step 3 (Eqs. 18-22) */
#pragma omp parallel for schedule(static)
    for (int c = 0; c < N; c++)
        for (int k = 0; k < o->nf[c]; k++) {
            int s = c * MAXF + k;
            if (o->nbr[s] >= 0) continue;
            const group_t *g = &o->groups[o->grp[s]];
            double *bv = &bval[(size_t)s * Q];
            double eq[Q];
            switch (g->kind) {
            case BC_WALL:          /* Eq. (18): f_P = f_eq(rho_k, u_w) + f_k - f_eq,k */
                orc_feq(rho[c], g->ux, g->uy, eq);
                for (int a = 0; a < Q; a++) bv[a] = eq[a] + f[c * Q + a] - feq[c * Q + a];
                break;
            case BC_INLET:         /* Eq. (19): rho* = rho_inf (external) or rho_k (internal) */
                orc_feq(g->internal ? rho[c] : g->rho, g->ux, g->uy, eq);
                for (int a = 0; a < Q; a++) bv[a] = eq[a] + f[c * Q + a] - feq[c * Q + a];
                break;
            case BC_OUTLET:
                if (!g->internal) { /* Eq. (20): f_GC = f_i */
                    for (int a = 0; a < Q; a++) bv[a] = f[c * Q + a];
                } else {            /* Eq. (21): f_eq(rho_inf, u_i) + f_k - f_eq,k */
                    orc_feq(g->rho, ux[c], uy[c], eq);
                    for (int a = 0; a < Q; a++) bv[a] = eq[a] + f[c * Q + a] - feq[c * Q + a];
                }
                break;
            case BC_SYMMETRY: {    /* Eq. (22): mirrored normal velocity */
                double un = ux[c] * o->nx[s] + uy[c] * o->ny[s];
                orc_feq(rho[c], ux[c] - 2.0 * un * o->nx[s], uy[c] - 2.0 * un * o->ny[s], eq);
                for (int a = 0; a < Q; a++) bv[a] = eq[a];
                break;
            }
            default:
                for (int a = 0; a < Q; a++) bv[a] = NAN;
            }
        }
    /* Step 2: least-squares gradient of every f_alpha (Eq. 12) */
#pragma omp parallel for schedule(static)
    for (int c = 0; c < N; c++)
        for (int a = 0; a < Q; a++) {
            double st[MAXF];
            for (int k = 0; k < o->nf[c]; k++) {
                int s = c * MAXF + k;
                st[k] = o->nbr[s] >= 0 ? f[o->nbr[s] * Q + a] : bval[(size_t)s * Q + a];
            }
            lsq_gradient(o, c, f[c * Q + a], st, &gx[c * Q + a], &gy[c * Q + a]);
        }
    /* Steps 3-4: face values (Eqs. 11, 23-26) and the RHS (Eq. 10) */
#pragma omp parallel for schedule(static)
    for (int c = 0; c < N; c++) {
        double flux[Q] = {0};
        for (int k = 0; k < o->nf[c]; k++) {
            int s = c * MAXF + k;
            int j = o->nbr[s];
            const group_t *g = j >= 0 ? NULL : &o->groups[o->grp[s]];
            for (int a = 0; a < Q; a++) {
                double en = EX[a] * o->nx[s] + EY[a] * o->ny[s];
                double own = f[c * Q + a] + gx[c * Q + a] * (o->fx[s] - o->cx[c]) + gy[c * Q + a] * (o->fy[s] - o->cy[c]);
                double phi;
                if (j >= 0) {
                    if (en > 0) {
                        phi = own;
                    } else {       /* upwind neighbour, reconstructed from its (image) centre */
                        double xj = o->cx[j] + o->shx[s], yj = o->cy[j] + o->shy[s];
                        phi = f[j * Q + a] + gx[j * Q + a] * (o->fx[s] - xj) + gy[j * Q + a] * (o->fy[s] - yj);
                    }
                } else if (g->kind == BC_WALL) {
                    phi = bval[(size_t)s * Q + a];
                } else if (g->kind == BC_INLET || (g->kind == BC_OUTLET && g->internal)) {
                    phi = en > 0 ? own : bval[(size_t)s * Q + a];          /* Eqs. (23), (24) */
                } else if (g->kind == BC_OUTLET) {
                    phi = f[c * Q + a];                                     /* Eq. (25) */
                } else {
                    phi = 0.5 * (f[c * Q + a] + bval[(size_t)s * Q + a]);   /* Eq. (26) */
                }
                if (face_out) face_out[(size_t)s * Q + a] = phi;
                flux[a] += en * o->len[s] * phi;
            }
        }
        for (int a = 0; a < Q; a++)
            rhs[c * Q + a] = -flux[a] / o->area[c] - (f[c * Q + a] - feq[c * Q + a]) / o->tau;
    }
    free(rho); free(ux); free(uy); free(feq); free(bval); free(gx); free(gy);
}

void orc_rhs(const oracle_t *o, const double *f, double *rhs) { operator_rhs(o, f, rhs, NULL); }

void orc_face_values(const oracle_t *o, const double *f, double *face_out) {
    double *rhs = (double *)malloc((size_t)o->n_cells * Q * sizeof(double));
    operator_rhs(o, f, rhs, face_out);
    free(rhs);
}

/* Step 0: f = f_eq(rho0, u0); rho/u may be NULL for uniform values. */
/* Force on wall group g: the momentum flux through the group's faces, with the
 * scheme's face values (at a wall, f_P of Eq. 18 for every direction):
 *   F = sum over the group's faces of sum_a e_a (e_a . n) dl phi_a,
 * n the outward unit normal of the fluid cell.  Also p = rho/3 of each face's
 * border cell, faces in the order of the boundary-face arrays.  Returns the
 * number of faces. */
int orc_wall_force(const oracle_t *o, const double *f, int g, double *force, double *face_p) {
    double *face = (double *)malloc((size_t)o->n_cells * MAXF * Q * sizeof(double));
    double *rhs = (double *)malloc((size_t)o->n_cells * Q * sizeof(double));
    operator_rhs(o, f, rhs, face);
    double fx = 0.0, fy = 0.0;
    int n = 0;
    for (int b = 0; b < o->n_bf; b++) {
        if (o->bf_group[b] != g) continue;
        const int s = o->bf_slot[b], c = s / MAXF;
        for (int a = 0; a < Q; a++) {
            const double en = (EX[a] * o->nx[s] + EY[a] * o->ny[s]) * o->len[s];
            fx += EX[a] * en * face[(size_t)s * Q + a];
            fy += EY[a] * en * face[(size_t)s * Q + a];
        }
        if (face_p) {
            double rho = 0.0;
            for (int a = 0; a < Q; a++) rho += f[(size_t)c * Q + a];
            face_p[n] = rho / 3.0;
        }
        n++;
    }
    force[0] = fx;
    force[1] = fy;
    free(face);
    free(rhs);
    return n;
}

void orc_init(oracle_t *o, const double *rho, const double *u, double rho0, double ux0, double uy0) {
    for (int c = 0; c < o->n_cells; c++)
        orc_feq(rho ? rho[c] : rho0, u ? u[2 * c] : ux0, u ? u[2 * c + 1] : uy0, &o->f[c * Q]);
    o->have_prev = 0;
    o->steps = 0;
}

void orc_set_f(oracle_t *o, const double *f) {
    memcpy(o->f, f, (size_t)o->n_cells * Q * sizeof(double));
    o->have_prev = 0;
}
void orc_get_f(const oracle_t *o, double *f) { memcpy(f, o->f, (size_t)o->n_cells * Q * sizeof(double)); }

/* Step 5 */
void orc_step(oracle_t *o, long n) {
    size_t M = (size_t)o->n_cells * Q;
    static const double beta[4] = {0.25, 1.0 / 3.0, 0.5, 1.0};
    for (long it = 0; it < n; it++) {
        if (o->scheme == SCHEME_EULER) {             /* Eq. (13) */
            operator_rhs(o, o->f, o->tmp0, NULL);
#pragma omp parallel for schedule(static)
            for (size_t i = 0; i < M; i++) o->f[i] = o->f[i] + o->dt * o->tmp0[i];
        } else if (o->scheme == SCHEME_AB2) {        /* Eq. (16), Euler on the first step */
            operator_rhs(o, o->f, o->tmp0, NULL);
            if (!o->have_prev) {
                for (size_t i = 0; i < M; i++) o->f[i] = o->f[i] + o->dt * o->tmp0[i];
            } else {
                for (size_t i = 0; i < M; i++)
                    o->f[i] = o->f[i] + 0.5 * o->dt * (3.0 * o->tmp0[i] - o->rhs_prev[i]);
            }
            memcpy(o->rhs_prev, o->tmp0, M * sizeof(double));
            o->have_prev = 1;
        } else {                                     /* Eq. (17) */
            memcpy(o->tmp1, o->f, M * sizeof(double));           /* f(0) */
            for (int k = 0; k < 4; k++) {
                operator_rhs(o, o->f, o->tmp0, NULL);
#pragma omp parallel for schedule(static)
                for (size_t i = 0; i < M; i++) o->f[i] = o->tmp1[i] + beta[k] * o->dt * o->tmp0[i];
            }
        }
        o->steps++;
    }
}

/* Step 6 */
void orc_macros(const oracle_t *o, double *rho, double *u) {
    for (int c = 0; c < o->n_cells; c++) {
        double r, x, y;
        orc_moments(&o->f[c * Q], &r, &x, &y);
        rho[c] = r;
        u[2 * c] = x;
        u[2 * c + 1] = y;
    }
}

double orc_mass(const oracle_t *o) {
    double m = 0;
    for (int c = 0; c < o->n_cells; c++) {
        double r = 0;
        for (int a = 0; a < Q; a++) r += o->f[c * Q + a];
        m += o->area[c] * r;
    }
    return m;
}

/* Eq. (32) with the squared denominator: u, u_old are [2*N]. */
double orc_residual(int n, const double *u, const double *u_old) {
    double num = 0, den = 0;
    for (int c = 0; c < n; c++) {
        double du = u[2 * c] - u_old[2 * c], dv = u[2 * c + 1] - u_old[2 * c + 1];
        num += du * du + dv * dv;
        den += u_old[2 * c] * u_old[2 * c] + u_old[2 * c + 1] * u_old[2 * c + 1];
    }
    return sqrt(num) / sqrt(den);
}

/* Threads of the timing build's loops (the one-thread build ignores it);
 * returns the number the loops will use. */
int orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
