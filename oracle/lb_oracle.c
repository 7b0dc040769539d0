/*
 * Plain FP64 CPU oracle of the semi-discrete compressible lattice Boltzmann
 * step with tau = 1 (Komeili, Mirzaei, Shabouei, arXiv 1602.02675).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP path.
 *
 * It is written to be read against the paper, not to be fast:
 *   - one node's equilibrium follows Sec. III.B in the paper's order:
 *     e = E - v^2/2 (below eq. 15), phi (eq. 15), c'_1, c'_2 (eq. 26),
 *     d_0 (Sec. III.B, "d_0 is an arbitrary portion"), d_1, d_2 (eq. 24-25);
 *   - the interpolation fractions alpha_k = rho_k / rho (eq. 23) come from the
 *     linear split of eq. 28 (1-D) and the bilinear split of eq. 29 (2-D);
 *   - every packet carries eta' = {m, m(v + c'), m[(v + c')^2/2 + phi]}
 *     (eq. 21) with m = alpha_k d_v (eq. 23) to x + v_k + c'_jv (eq. 10-13,
 *     eq. 30), and the new moments are the sums of what lands on each node
 *     (Sec. V.A, eq. 6 and 22);
 *   - the step is a literal scatter: sources in ascending order (rows, then
 *     columns), lanes and corners in a fixed order.
 *   - boundaries (Sec. V.B): transmissive ends use explicit ghost nodes that
 *     copy the edge node and are refilled every step; packets that leave the
 *     interior are dropped.  Periodic directions wrap.
 *   - reflecting walls (the shock reflection the conclusions name as an
 *     extension): a wall stands on the outer face of each edge node, half a
 *     node beyond it.  A packet whose destination lies past the wall is
 *     reflected specularly: it lands as far inside the wall as it would have
 *     landed outside (index -1 - i below the low end, 2n - 1 - i above the
 *     high end), and the component of its momentum normal to the wall changes
 *     sign; its mass and energy are unchanged.
 *
 * Readings of points the paper leaves open:
 *   - "int" in eq. 26 is the floor of a non-negative real; c'_1 is the largest
 *     integer with c'_1^2 <= A, decided by exact comparison.
 *   - d_0 = delta0 * rho with delta0 a parameter (paper: 0.4 .. 0.55).
 *   - e is clamped at 0 (a negative e is rounding error of E - v^2/2).
 *   - corner k of eq. 28/29: corner 0 is the node floor(v), corner 1 the
 *     node floor(v) + 1 (per axis); its weight is the length (1-D) or area
 *     (2-D) opposite to it.
 *   - a node with rho <= 0 emits nothing.
 *   - 2-D lanes are the four axis directions at speeds c'_1, c'_2.
 *   - two gases (the different gases on the two sides of the tube that the
 *     conclusions name as an extension): both ideal with one gas constant R,
 *     ratios gamma (gas 1) and gamma2 (gas 2).  A species moment rho chi
 *     (chi = mass fraction of gas 1) is carried as a further field: every
 *     packet carries m chi of its source, as it carries its mass.  A node's
 *     gas is the mixture: c_v = chi c_v1 + (1 - chi) c_v2 with
 *     c_vi = R / (gamma_i - 1), so gamma - 1 = R / c_v =
 *     1 / (chi / (gamma - 1) + (1 - chi) / (gamma2 - 1)), which then enters
 *     phi (eq. 15) and A (eq. 26).
 *   - the square lattice with a rest level (delta0 > 0 in 2-D: the 2-D
 *     triple-level set, which the paper's eq. 24-26 cover through b_0 but
 *     whose figures show only the dual-level set): one rest particle group,
 *     b_0 = 1, d_0 = delta0 * rho, next to the four directions at c'_1, c'_2
 *     (b_1 = b_2 = 4).  delta0 = 0 is the paper's dual-level set.
 *   - the hexagonal lattice (Fig. 1; Sec. III.B with b_v = 6): nodes at
 *     i e_1 + j e_2 with e_1 = (1, 0), e_2 = (1/2, sqrt(3)/2) (unit spacing),
 *     stored as Y[.][j][i]; velocities and momenta are Cartesian.  Its six
 *     directions are the unit vectors at multiples of 60 degrees, axial
 *     (1,0), (0,1), (-1,1), (-1,0), (0,-1), (1,-1), each at c'_1 and c'_2
 *     (b_1 = b_2 = 6; eq. 16-18 hold with b_v / D = 3), plus a rest group
 *     when delta0 > 0.  The end point of v, v = a e_1 + b e_2, lies in the
 *     lattice triangle with vertices (f_a, f_b) + {(1,0), (0,1)} and either
 *     (0,0) (when r_a + r_b <= 1, r = (a,b) - f) or (1,1); "the nodes that
 *     surround the end point of v" are these three, and alpha_k (eq. 23) is
 *     the barycentric weight of vertex k: the only split of the unit mass on
 *     three nodes with sum alpha_k v'_k = 0.  tri 0: alpha = (1 - r_a - r_b,
 *     r_a, r_b) at (0,0), (1,0), (0,1); tri 1: alpha = (r_a + r_b - 1, 1 - r_b,
 *     1 - r_a) at (1,1), (1,0), (0,1).  Boundaries along both axial
 *     directions: transmissive or periodic (no walls).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OC_GHOSTS 8       /* ghost nodes per transmissive end (>= any reach) */
#define OC_MAX_PACKETS 40 /* 10 in 1-D, 32 square (36 with the rest level), 36 hexagonal (39) */

typedef struct {
    int dim;        /* 1: 1-D triple-level lattice; 2: square dual-level lattice */
    long nx, ny;    /* ny = 1 when dim = 1 */
    int bc_x, bc_y; /* 0: transmissive (ghost nodes copy the edge); 1: periodic;
                       2: reflecting wall at each end */
    double gamma;   /* ratio of specific heats */
    double delta0;  /* d_0 = delta0 * rho; in 2-D, delta0 > 0 adds the rest level */
    int species;    /* 1: two gases, a species field rho chi after rho E */
    double gamma2;  /* ratio of specific heats of gas 2 (species only) */
    int hex;        /* dim 2 only: 1 for the hexagonal lattice, 0 for the square one */
} oc_problem;

typedef struct {
    int valid;   /* 0 when rho <= 0: the node emits nothing */
    double rho, v[2], E, e, phi, A;
    int c1, c2;
    double d0, d1, d2;
    int b0, b1, b2;
    int f[2];     /* floor of v per axis: corner 0 is x + f */
    double vp0[2]; /* v'_1 = (x + f) - (x + v): towards corner 0 */
    double vp1[2]; /* v'_2 = (x + f + 1) - (x + v): towards corner 1 */
    double chi;    /* mass fraction of gas 1 (two gases) */
    double gm1;    /* gamma - 1 of the node's gas */
    /* hexagonal lattice: f = floor of the axial coordinates (a, b) of v,
     * r = (a, b) - f, tri = which triangle of the cell holds the end point */
    double r[2];
    int tri;
} oc_levels;

/* Number of moment fields: rho, rho*v (dim components), rho*E. */
static int oc_nf(const oc_problem* P) { return P->dim + 2 + (P->species ? 1 : 0); }

/* Largest integer c with c*c <= A (A >= 0): the floor of sqrt(A), eq. 26. */
static int oc_isqrt_floor(double A)
{
    int c = (int)floor(sqrt(A));
    while (c > 0 && (double)c * (double)c > A) c--;
    while ((double)(c + 1) * (double)(c + 1) <= A) c++;
    return c;
}

/*
 * Equilibrium of one node (Sec. III.B).  Yn = [rho, rho*v_1..v_D, rho*E
 * (, rho*chi)] in lattice units (dx = dt = 1).
 */
int oc_levels_of(const oc_problem* P, const double* Yn, oc_levels* L)
{
    const int D = P->dim;
    memset(L, 0, sizeof(*L));
    L->rho = Yn[0];
    if (!(L->rho > 0.0)) {
        L->valid = 0;
        return 0;
    }
    L->valid = 1;
    /* flow velocity and total energy per unit mass (eq. 7) */
    for (int a = 0; a < D; ++a) L->v[a] = Yn[1 + a] / L->rho;
    L->E = Yn[1 + D] / L->rho;
    /* internal energy e = E - v^2/2 (below eq. 15) */
    double v2 = 0.0;
    for (int a = 0; a < D; ++a) v2 = v2 + L->v[a] * L->v[a];
    L->e = L->E - 0.5 * v2;
    if (L->e < 0.0) L->e = 0.0;
    /* non-translational energy (eq. 15) */
    /* the node's gas: one gamma, or the mixture of two by mass fraction */
    L->gm1 = P->gamma - 1.0;
    if (P->species) {
        double chi = Yn[D + 2] / L->rho;
        chi = chi < 0.0 ? 0.0 : (chi > 1.0 ? 1.0 : chi);
        L->chi = chi;
        L->gm1 = 1.0 / (chi / (P->gamma - 1.0) + (1.0 - chi) / (P->gamma2 - 1.0));
    }
    L->phi = (1.0 - ((double)D / 2.0) * L->gm1) * L->e;
    /* velocity set (Sec. IV): 1-D b0=1, b1=b2=2; square lattice b0=0, b1=b2=4
     * (dual level), or b0=1 with d0 = delta0 rho (triple level) */
    const int bdir = (D == 2 && P->hex) ? 6 : 2 * D; /* directions per level */
    if (D == 1) {
        L->b0 = 1; L->b1 = 2; L->b2 = 2;
        L->d0 = P->delta0 * L->rho;
    } else if (P->delta0 > 0.0) {
        L->b0 = 1; L->b1 = bdir; L->b2 = bdir;
        L->d0 = P->delta0 * L->rho;
    } else {
        L->b0 = 0; L->b1 = bdir; L->b2 = bdir;
        L->d0 = 0.0;
    }
    /* level speeds (eq. 26) */
    const double Dg1 = (double)D * L->gm1;
    L->A = Dg1 * L->e * L->rho / (L->rho - (double)L->b0 * L->d0);
    if (!(L->A >= 0.0)) L->A = 0.0;
    if (L->A > 1.0e6) L->A = 1.0e6; /* far beyond any admissible reach */
    L->c1 = oc_isqrt_floor(L->A);
    L->c2 = L->c1 + 1;
    /* level weights (eq. 24-25) */
    const double c1s = (double)L->c1 * (double)L->c1;
    const double c2s = (double)L->c2 * (double)L->c2;
    const double rest = L->rho - (double)L->b0 * L->d0;
    const double Dp = Dg1 * L->rho * L->e;
    L->d1 = (c2s * rest - Dp) / ((double)L->b1 * (c2s - c1s));
    L->d2 = (Dp - c1s * rest) / ((double)L->b1 * (c2s - c1s));
    /* nodes surrounding the end point of v (eq. 13, 28-29) */
    if (D == 2 && P->hex) {
        /* axial coordinates of v: v_y = b sqrt(3)/2, v_x = a + b/2 */
        const double b = 2.0 * L->v[1] / sqrt(3.0);
        const double a = L->v[0] - 0.5 * b;
        L->f[0] = (int)floor(a);
        L->f[1] = (int)floor(b);
        L->r[0] = a - (double)L->f[0];
        L->r[1] = b - (double)L->f[1];
        L->tri = L->r[0] + L->r[1] > 1.0 ? 1 : 0;
        return 1;
    }
    for (int a = 0; a < D; ++a) {
        L->f[a] = (int)floor(L->v[a]);
        L->vp0[a] = (double)L->f[a] - L->v[a];
        L->vp1[a] = ((double)L->f[a] + 1.0) - L->v[a];
    }
    return 1;
}

/*
 * All packets one node emits (eq. 19-23, 30-33): for each lane, for each
 * corner, the displacement (integer, per axis) and eta = {m, m xi, m zeta}.
 * Returns the number of packets (10 in 1-D, 32 in 2-D, 36 with the 2-D rest
 * level; 0 if rho <= 0).
 * off: [n][2] integer displacement; pay: [n][nf].
 */
/* Packets of one node of the hexagonal lattice (see oc_packets): lanes in
 * the order rest group, six directions at c'_1, six at c'_2; per lane the
 * three vertices of the triangle around the end point of v. */
static int oc_packets_hex(const oc_problem* P, const oc_levels* L, int* off, double* pay)
{
    const int nf = oc_nf(P);
    /* the six directions: axial steps and Cartesian unit vectors */
    const int dir[6][2] = {{1, 0}, {0, 1}, {-1, 1}, {-1, 0}, {0, -1}, {1, -1}};
    const double h = sqrt(3.0) / 2.0;
    const double unit[6][2] = {{1.0, 0.0}, {0.5, h}, {-0.5, h}, {-1.0, 0.0}, {-0.5, -h}, {0.5, -h}};
    /* triangle vertices relative to f and their barycentric weights */
    int vert[3][2];
    double alpha[3];
    const double ra = L->r[0], rb = L->r[1];
    if (L->tri == 0) {
        vert[0][0] = 0; vert[0][1] = 0; alpha[0] = (1.0 - ra) - rb;
    } else {
        vert[0][0] = 1; vert[0][1] = 1; alpha[0] = (ra + rb) - 1.0;
    }
    vert[1][0] = 1; vert[1][1] = 0; alpha[1] = L->tri == 0 ? ra : 1.0 - rb;
    vert[2][0] = 0; vert[2][1] = 1; alpha[2] = L->tri == 0 ? rb : 1.0 - ra;
    /* lanes: speed, direction (-1: rest) and weight d_v */
    int lane_s[13], lane_j[13];
    double lane_d[13];
    int nl = 0;
    if (L->b0 == 1) { lane_s[nl] = 0; lane_j[nl] = -1; lane_d[nl++] = L->d0; }
    for (int lev = 1; lev <= 2; ++lev)
        for (int j = 0; j < 6; ++j) {
            lane_s[nl] = lev == 1 ? L->c1 : L->c2;
            lane_j[nl] = j;
            lane_d[nl++] = lev == 1 ? L->d1 : L->d2;
        }
    int n = 0;
    for (int l = 0; l < nl; ++l) {
        const int c = lane_s[l], j = lane_j[l];
        /* molecular velocity v + c' (eq. 12) and zeta (eq. 14) */
        const double xi0 = L->v[0] + (j < 0 ? 0.0 : (double)c * unit[j][0]);
        const double xi1 = L->v[1] + (j < 0 ? 0.0 : (double)c * unit[j][1]);
        const double zeta = 0.5 * (xi0 * xi0 + xi1 * xi1) + L->phi;
        for (int t = 0; t < 3; ++t) {
            const double m = alpha[t] * lane_d[l]; /* eq. 23 */
            off[2 * n + 0] = L->f[0] + vert[t][0] + (j < 0 ? 0 : c * dir[j][0]);
            off[2 * n + 1] = L->f[1] + vert[t][1] + (j < 0 ? 0 : c * dir[j][1]);
            pay[nf * n + 0] = m;
            pay[nf * n + 1] = m * xi0;
            pay[nf * n + 2] = m * xi1;
            pay[nf * n + 3] = m * zeta;
            ++n;
        }
    }
    return n;
}

int oc_packets(const oc_problem* P, const double* Yn, int* off, double* pay)
{
    oc_levels L;
    const int D = P->dim, nf = oc_nf(P);
    if (!oc_levels_of(P, Yn, &L)) return 0;
    if (D == 2 && P->hex) return oc_packets_hex(P, &L, off, pay);
    /* lanes: c' per axis and weight d_v */
    int lane_c[9][2];
    double lane_d[9];
    int nl = 0;
    if (D == 1) {
        lane_c[nl][0] = 0;       lane_c[nl][1] = 0; lane_d[nl++] = L.d0;
        lane_c[nl][0] = +L.c1;   lane_c[nl][1] = 0; lane_d[nl++] = L.d1;
        lane_c[nl][0] = -L.c1;   lane_c[nl][1] = 0; lane_d[nl++] = L.d1;
        lane_c[nl][0] = +L.c2;   lane_c[nl][1] = 0; lane_d[nl++] = L.d2;
        lane_c[nl][0] = -L.c2;   lane_c[nl][1] = 0; lane_d[nl++] = L.d2;
    } else {
        if (L.b0 == 1) { /* rest level of the triple-level square set */
            lane_c[nl][0] = 0; lane_c[nl][1] = 0; lane_d[nl++] = L.d0;
        }
        for (int lev = 1; lev <= 2; ++lev) {
            const int c = lev == 1 ? L.c1 : L.c2;
            const double d = lev == 1 ? L.d1 : L.d2;
            lane_c[nl][0] = +c; lane_c[nl][1] = 0;  lane_d[nl++] = d;
            lane_c[nl][0] = -c; lane_c[nl][1] = 0;  lane_d[nl++] = d;
            lane_c[nl][0] = 0;  lane_c[nl][1] = +c; lane_d[nl++] = d;
            lane_c[nl][0] = 0;  lane_c[nl][1] = -c; lane_d[nl++] = d;
        }
    }
    const int ncorner = D == 1 ? 2 : 4;
    int n = 0;
    for (int l = 0; l < nl; ++l) {
        for (int k = 0; k < ncorner; ++k) {
            const int kx = k & 1, ky = (k >> 1) & 1;
            /* alpha_k = rho_k / rho: the length (eq. 28) or area (eq. 29)
             * between the end point of v and the node opposite to corner k */
            double alpha = fabs(kx ? L.vp0[0] : L.vp1[0]);
            if (D == 2) alpha = fabs((kx ? L.vp0[0] : L.vp1[0]) * (ky ? L.vp0[1] : L.vp1[1]));
            const double m = alpha * lane_d[l]; /* eq. 23 */
            double xi[2] = {0.0, 0.0};
            double xi2 = 0.0;
            for (int a = 0; a < D; ++a) {
                xi[a] = L.v[a] + (double)lane_c[l][a]; /* eq. 12, 21 */
                xi2 = xi2 + xi[a] * xi[a];
            }
            const double zeta = 0.5 * xi2 + L.phi; /* eq. 14, 21 */
            off[2 * n + 0] = L.f[0] + kx + lane_c[l][0];
            off[2 * n + 1] = D == 2 ? L.f[1] + ky + lane_c[l][1] : 0;
            pay[nf * n + 0] = m;
            for (int a = 0; a < D; ++a) pay[nf * n + 1 + a] = m * xi[a];
            pay[nf * n + 1 + D] = m * zeta;
            if (P->species) pay[nf * n + 2 + D] = m * L.chi; /* gas 1 moves with the mass */
            ++n;
        }
    }
    return n;
}

static long oc_clamp(long i, long n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }
static long oc_wrap(long i, long n) { long r = i % n; return r < 0 ? r + n : r; }

/* Specular reflection off the walls on the outer faces of nodes 0 and n - 1:
 * the landing index, reflected (again, should it cross the opposite wall)
 * until inside; *flips counts the reflections. */
static long oc_reflect(long i, long n, int* flips)
{
    while (i < 0 || i >= n) {
        i = i < 0 ? -1 - i : 2 * n - 1 - i;
        ++*flips;
    }
    return i;
}

/*
 * One step Y -> Ynew (SoA [nf][ny][nx], lattice units).  max_reach (may be
 * NULL) receives the largest |displacement| component of any packet of any
 * interior node.  Returns 0 on success, -1 on bad arguments, -4 when an
 * interior node has rho <= 0 or a non-finite moment.
 */
int oc_step(const oc_problem* P, const double* Y, double* Ynew, int* max_reach)
{
    const int D = P->dim, nf = oc_nf(P);
    const long nx = P->nx, ny = D == 2 ? P->ny : 1, nn = nx * ny;
    if (nx < 1 || ny < 1 || (D != 1 && D != 2)) return -1;
    int status = 0, reach = 0;
    for (long q = 0; q < (long)nf * nn; ++q)
        if (!isfinite(Y[q])) status = -4;
    for (long q = 0; q < nn; ++q)
        if (!(Y[q] > 0.0)) status = -4;
    memset(Ynew, 0, sizeof(double) * (size_t)nf * (size_t)nn);
    if (P->bc_x < 0 || P->bc_x > 2 || (D == 2 && (P->bc_y < 0 || P->bc_y > 2))) return -1;
    /* the hexagonal lattice has no walls (nor a second gas) */
    if (D == 2 && P->hex && (P->bc_x == 2 || P->bc_y == 2 || P->species)) return -1;
    /* source range: ghosts beyond transmissive ends only (Sec. V.B) */
    const long gx = P->bc_x == 0 ? OC_GHOSTS : 0;
    const long gy = (D == 2 && P->bc_y == 0) ? OC_GHOSTS : 0;
    int off[2 * OC_MAX_PACKETS];
    double pay[5 * OC_MAX_PACKETS];
    double Yn[5];
    for (long sj = -gy; sj < ny + gy; ++sj) {
        for (long si = -gx; si < nx + gx; ++si) {
            /* ghost nodes hold a copy of the nearest edge node */
            const long ci = oc_clamp(si, nx), cj = oc_clamp(sj, ny);
            for (int fld = 0; fld < nf; ++fld) Yn[fld] = Y[(long)fld * nn + cj * nx + ci];
            const int np = oc_packets(P, Yn, off, pay);
            const int interior = si >= 0 && si < nx && sj >= 0 && sj < ny;
            for (int p = 0; p < np; ++p) {
                if (interior) {
                    for (int a = 0; a < D; ++a) {
                        const int r = abs(off[2 * p + a]);
                        if (r > reach) reach = r;
                    }
                }
                long ti = si + off[2 * p + 0];
                long tj = sj + off[2 * p + 1];
                int flips[2] = {0, 0};
                if (P->bc_x == 1) ti = oc_wrap(ti, nx);
                else if (P->bc_x == 2) ti = oc_reflect(ti, nx, &flips[0]);
                else if (ti < 0 || ti >= nx) continue; /* leaves the tube */
                if (D == 2) {
                    if (P->bc_y == 1) tj = oc_wrap(tj, ny);
                    else if (P->bc_y == 2) tj = oc_reflect(tj, ny, &flips[1]);
                    else if (tj < 0 || tj >= ny) continue;
                }
                for (int fld = 0; fld < nf; ++fld) {
                    double q = pay[nf * p + fld];
                    /* a reflected packet's normal momentum changes sign */
                    if (fld >= 1 && fld <= D && (flips[fld - 1] & 1)) q = -q;
                    Ynew[(long)fld * nn + tj * nx + ti] += q;
                }
            }
        }
    }
    if (max_reach) *max_reach = reach;
    return status;
}

/* n steps in place; max_reach gets the largest reach over all steps. */
int oc_run(const oc_problem* P, double* Y, long nsteps, int* max_reach)
{
    const int nf = oc_nf(P);
    const long nn = P->nx * (P->dim == 2 ? P->ny : 1);
    double* T = (double*)malloc(sizeof(double) * (size_t)nf * (size_t)nn);
    if (!T) return -2;
    int status = 0, reach = 0;
    for (long s = 0; s < nsteps; ++s) {
        int r = 0;
        const int st = oc_step(P, Y, T, &r);
        if (st != 0) { status = st; break; }
        if (r > reach) reach = r;
        memcpy(Y, T, sizeof(double) * (size_t)nf * (size_t)nn);
    }
    free(T);
    if (max_reach) *max_reach = reach;
    return status;
}

/* Conservation totals over the interior: sum of each moment field. */
void oc_totals(const oc_problem* P, const double* Y, double* out)
{
    const int nf = oc_nf(P);
    const long nn = P->nx * (P->dim == 2 ? P->ny : 1);
    for (int fld = 0; fld < nf; ++fld) {
        double s = 0.0;
        for (long q = 0; q < nn; ++q) s += Y[(long)fld * nn + q];
        out[fld] = s;
    }
}

/* Per-node lanes (f per axis, c'_1) of a whole field, for index parity. */
void oc_lanes(const oc_problem* P, const double* Y, int* fx, int* fy, int* c1)
{
    const int D = P->dim, nf = oc_nf(P);
    const long nn = P->nx * (D == 2 ? P->ny : 1);
    double Yn[5];
    for (long q = 0; q < nn; ++q) {
        oc_levels L;
        for (int fld = 0; fld < nf; ++fld) Yn[fld] = Y[(long)fld * nn + q];
        oc_levels_of(P, Yn, &L);
        fx[q] = L.valid ? L.f[0] : 0;
        fy[q] = (L.valid && D == 2) ? L.f[1] : 0;
        c1[q] = L.valid ? L.c1 : 0;
    }
}
