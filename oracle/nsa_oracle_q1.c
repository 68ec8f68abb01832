/*
 * nsa_oracle_q1.c -- plain, slow, serial FP64 CPU oracle for the 2-D element family: bilinear
 * quadrilaterals (four nodes, two space dimensions), incompressible Navier-Stokes element assembly
 * into a block-CSR matrix with 3x3 blocks (dofs u, v, p per node) plus RHS.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or load this file: it is
 * used by the tests and by the CPU-baseline leg of the benchmark, and it shares no code, header,
 * table or constant with the HIP library.
 *
 * What it computes follows the paper (Brown, arXiv 2111.05651) as the tetrahedral oracle does:
 *   - Sec. II-A, Listing 1: per element, in this order, gather nodal data, form the Cartesian
 *     derivatives of the shape functions, the Gauss-point values, the stabilisation parameters,
 *     the element operators, the convective term with the RHS, the viscous term, then scatter.
 *     All arithmetic is double precision.
 *   - Table 2: the two 2-D benchmarks (Cylinder 2D, Venturi 2D) have about one element per nodal
 *     point and the kernel takes four nodes per element (Sec. II-A): bilinear quadrilaterals.
 *   - Sec. III-A, Listings 3/4: the velocity-velocity block is indexed by dofv = node*NUM_DIMS + dim,
 *     a common term for every (idime, jdime) pair and an extra term on the diagonal.
 * The formulation is the tetrahedral reading carried to two dimensions: Oseen-linearised
 * backward-Euler Navier-Stokes with SUPG/PSPG/grad-div stabilisation, the 2x2 Gauss-Legendre rule
 * (PGAUS = 4 as for the tetrahedra; the Jacobian varies over a general quadrilateral, so every term
 * is integrated point by point), element length h = sqrt(area), dof 3*node + c with pressure as
 * c = 2, rows = test functions, BSR-3 output.
 *
 * Compile together with nsa_oracle.c (whose oracle_pattern builds the node-graph pattern of any
 * four-node element): gcc -O2 -ffp-contract=off -fPIC -shared.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q1_OK 0
#define Q1_EINVAL (-1)
#define Q1_ERANGE (-2)
#define Q1_EDEGENERATE (-3)

#define PNODE 4   /* nodes per bilinear quadrilateral */
#define NDIME 2   /* space dimensions */
#define NDOFN 3   /* dofs per node: u, v, p */
#define NEVAT (PNODE * NDOFN)
#define MAXGP 9   /* up to a 3x3 rule (the method's is 2x2; 3x3 serves the pins) */

/* reference square [-1, 1]^2, vertices counter-clockwise */
static const double XI[PNODE] = {-1.0, 1.0, 1.0, -1.0};
static const double ETA[PNODE] = {-1.0, -1.0, 1.0, 1.0};

typedef struct {
    double elcod[PNODE][NDIME];
    double elvel[PNODE][NDIME];
    int ngaus;
    double shape[MAXGP][PNODE];         /* N_a at Gauss point g */
    double gpcar[MAXGP][PNODE][NDIME];  /* d N_a / d x_d at g */
    double gpvol[MAXGP];                /* Gauss weight times |det J(g)| */
    double area;
    double gpvel[MAXGP][NDIME];
    double agrau[MAXGP][PNODE];         /* a_g . grad N_a at g */
    double hleng;
    double abar[NDIME];
    double tau1, tau2;
    double wgrgr[MAXGP][PNODE][PNODE];  /* grad N_a . grad N_b at g */
    double elauu[NEVAT][NEVAT];         /* rows = test (a,c), cols = trial (b,c') */
    double elrhs[NEVAT];
} qelem_t;

/* Gather (calculate_transients, Listing 2): elvel(j,i) = veloc(j, lnods(e,i)), elcod likewise. */
static void calculate_transients(const int32_t *ln, const double *coord, const double *veloc,
                                 double elcod[PNODE][NDIME], double elvel[PNODE][NDIME])
{
    for (int i = 0; i < PNODE; i++) {
        int64_t ipoin = ln[i];
        for (int j = 0; j < NDIME; j++) {
            elvel[i][j] = veloc ? veloc[NDIME * ipoin + j] : 0.0;
            elcod[i][j] = coord[NDIME * ipoin + j];
        }
    }
}

/* n-point Gauss-Legendre abscissae and weights on [-1, 1] (n = 2 or 3). */
static void gauss_legendre(int n, double *x, double *w)
{
    if (n == 2) {
        x[0] = -1.0 / sqrt(3.0); x[1] = 1.0 / sqrt(3.0);
        w[0] = 1.0; w[1] = 1.0;
    } else {
        x[0] = -sqrt(0.6); x[1] = 0.0; x[2] = sqrt(0.6);
        w[0] = 5.0 / 9.0; w[1] = 8.0 / 9.0; w[2] = 5.0 / 9.0;
    }
}

/* Shape functions, the Jacobian of the bilinear map, its inverse and the Cartesian derivatives at
 * every Gauss point of the n x n rule (calculate_cartesian_derivatives). Returns 0 for a degenerate
 * element: det J zero or not finite at a Gauss point, or of different signs at two of them. */
static int calculate_cartesian_derivatives(qelem_t *E, int n)
{
    double x[3], w[3];
    gauss_legendre(n, x, w);
    E->ngaus = n * n;
    E->area = 0.0;
    double sign = 0.0;
    for (int gj = 0; gj < n; gj++)
        for (int gi = 0; gi < n; gi++) {
            const int g = gj * n + gi;
            const double xi = x[gi], eta = x[gj];
            double deriv[PNODE][NDIME];
            for (int a = 0; a < PNODE; a++) {
                E->shape[g][a] = 0.25 * (1.0 + XI[a] * xi) * (1.0 + ETA[a] * eta);
                deriv[a][0] = 0.25 * XI[a] * (1.0 + ETA[a] * eta);
                deriv[a][1] = 0.25 * ETA[a] * (1.0 + XI[a] * xi);
            }
            double J[NDIME][NDIME] = {{0.0, 0.0}, {0.0, 0.0}};  /* J[r][s] = d x_r / d xi_s */
            for (int r = 0; r < NDIME; r++)
                for (int s = 0; s < NDIME; s++)
                    for (int a = 0; a < PNODE; a++) J[r][s] += E->elcod[a][r] * deriv[a][s];
            const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
            if (!(det != 0.0) || !isfinite(det)) return 0;
            if (sign == 0.0) sign = det > 0.0 ? 1.0 : -1.0;
            else if ((det > 0.0 ? 1.0 : -1.0) != sign) return 0;
            /* (J^-1)[s][d] */
            const double jinv[NDIME][NDIME] = {{J[1][1] / det, -J[0][1] / det}, {-J[1][0] / det, J[0][0] / det}};
            for (int a = 0; a < PNODE; a++)
                for (int d = 0; d < NDIME; d++) {
                    double s = 0.0;
                    for (int k = 0; k < NDIME; k++) s += deriv[a][k] * jinv[k][d];
                    E->gpcar[g][a][d] = s;
                }
            E->gpvol[g] = w[gi] * w[gj] * fabs(det);
            E->area += E->gpvol[g];
        }
    return 1;
}

/* Velocity at the Gauss points (calculate_gauss_point_values). */
static void calculate_gauss_point_values(qelem_t *E)
{
    for (int g = 0; g < E->ngaus; g++)
        for (int c = 0; c < NDIME; c++) {
            double s = 0.0;
            for (int a = 0; a < PNODE; a++) s += E->shape[g][a] * E->elvel[a][c];
            E->gpvel[g][c] = s;
        }
}

/* Element length and stabilisation parameters (calculate_tau_and_tim). */
static void calculate_tau_and_tim(qelem_t *E, double rho, double mu, double dt)
{
    E->hleng = sqrt(E->area);
    double an2 = 0.0;
    for (int c = 0; c < NDIME; c++) {
        double s = 0.0;
        for (int a = 0; a < PNODE; a++) s += E->elvel[a][c];
        E->abar[c] = 0.25 * s;
        an2 += E->abar[c] * E->abar[c];
    }
    const double anorm = sqrt(an2), h = E->hleng;
    E->tau1 = 1.0 / (rho / dt + 4.0 * mu / (h * h) + 2.0 * rho * anorm / h);
    E->tau2 = mu + 0.5 * rho * anorm * h;
}

/* a . grad N and grad N . grad N at the Gauss points (calculate_element_matricies). */
static void calculate_element_matricies(qelem_t *E)
{
    for (int g = 0; g < E->ngaus; g++) {
        for (int a = 0; a < PNODE; a++) {
            double s = 0.0;
            for (int d = 0; d < NDIME; d++) s += E->gpvel[g][d] * E->gpcar[g][a][d];
            E->agrau[g][a] = s;
        }
        for (int a = 0; a < PNODE; a++)
            for (int b = 0; b < PNODE; b++) {
                double s = 0.0;
                for (int d = 0; d < NDIME; d++) s += E->gpcar[g][a][d] * E->gpcar[g][b][d];
                E->wgrgr[g][a][b] = s;
            }
    }
}

/* Time, convective, SUPG and pressure-coupling terms plus the RHS, Gauss point by Gauss point
 * (calculate_convective_term_and_RHS). dof index 3*node + c, c = 2 is pressure. */
static void calculate_convective_term_and_RHS(qelem_t *E, double rho, double dt)
{
    const double rdt = rho / dt, t1 = E->tau1;
    memset(E->elauu, 0, sizeof(E->elauu));
    memset(E->elrhs, 0, sizeof(E->elrhs));
    for (int g = 0; g < E->ngaus; g++) {
        const double w = E->gpvol[g];
        for (int a = 0; a < PNODE; a++) {
            const double Na = E->shape[g][a], aga = E->agrau[g][a];
            for (int b = 0; b < PNODE; b++) {
                const double Nb = E->shape[g][b], agb = E->agrau[g][b];
                const double tuu = rdt * Na * Nb + rho * Na * agb + t1 * rho * aga * (rho * agb + rdt * Nb);
                for (int c = 0; c < NDIME; c++) E->elauu[3 * a + c][3 * b + c] += w * tuu;
                for (int c = 0; c < NDIME; c++) {
                    E->elauu[3 * a + c][3 * b + 2] += w * (-Nb * E->gpcar[g][a][c] + t1 * rho * aga * E->gpcar[g][b][c]);
                    E->elauu[3 * a + 2][3 * b + c] += w * (Na * E->gpcar[g][b][c] + t1 * E->gpcar[g][a][c] * (rdt * Nb + rho * agb));
                }
            }
            for (int c = 0; c < NDIME; c++)
                E->elrhs[3 * a + c] += w * (rdt * E->gpvel[g][c] * Na + t1 * rho * rdt * aga * E->gpvel[g][c]);
            double gdu = 0.0;
            for (int d = 0; d < NDIME; d++) gdu += E->gpcar[g][a][d] * E->gpvel[g][d];
            E->elrhs[3 * a + 2] += w * t1 * rdt * gdu;
        }
    }
}

/* Viscous term mu (grad u + grad u^T) : grad v, grad-div tau2 (div u)(div v) and the PSPG pressure
 * Laplacian tau1 (grad q, grad p), Gauss point by Gauss point (calculate_viscous_term). */
static void calculate_viscous_term(qelem_t *E, double mu)
{
    for (int g = 0; g < E->ngaus; g++) {
        const double w = E->gpvol[g];
        for (int a = 0; a < PNODE; a++)
            for (int b = 0; b < PNODE; b++) {
                for (int c = 0; c < NDIME; c++)
                    for (int cp = 0; cp < NDIME; cp++) {
                        double v = mu * E->gpcar[g][a][cp] * E->gpcar[g][b][c] + E->tau2 * E->gpcar[g][a][c] * E->gpcar[g][b][cp];
                        if (c == cp) v += mu * E->wgrgr[g][a][b];
                        E->elauu[3 * a + c][3 * b + cp] += w * v;
                    }
                E->elauu[3 * a + 2][3 * b + 2] += w * E->tau1 * E->wgrgr[g][a][b];
            }
    }
}

static int element_pipeline(const double X[PNODE][NDIME], const double U[PNODE][NDIME], double rho, double mu,
                            double dt, int n, qelem_t *E)
{
    memcpy(E->elcod, X, sizeof(E->elcod));
    memcpy(E->elvel, U, sizeof(E->elvel));
    if (!calculate_cartesian_derivatives(E, n)) return Q1_EDEGENERATE;
    calculate_gauss_point_values(E);
    calculate_tau_and_tim(E, rho, mu, dt);
    calculate_element_matricies(E);
    calculate_convective_term_and_RHS(E, rho, dt);
    calculate_viscous_term(E, mu);
    return Q1_OK;
}

/* ---------------------------------------------------------------------------------------------- */

/* One element with the n x n Gauss rule (n = 2 is the method's; n = 3 for the pins): X, U are [4][2]
 * row-major, A is [12][12] row-major, b is [12]. */
int oracle_q1_element_rule(const double *X, const double *U, double rho, double mu, double dt, int n, double *A,
                           double *b)
{
    if (n != 2 && n != 3) return Q1_EINVAL;
    qelem_t E;
    int st = element_pipeline((const double(*)[NDIME])X, (const double(*)[NDIME])U, rho, mu, dt, n, &E);
    if (st != Q1_OK) return st;
    memcpy(A, E.elauu, sizeof(E.elauu));
    memcpy(b, E.elrhs, sizeof(E.elrhs));
    return Q1_OK;
}

int oracle_q1_element(const double *X, const double *U, double rho, double mu, double dt, double *A, double *b)
{
    return oracle_q1_element_rule(X, U, rho, mu, dt, 2, A, b);
}

/* Element intermediates for pinning the integration (2x2 rule): scal = area, h, tau1, tau2; the
 * integrals mass[a][b] = int N_a N_b, stiff[a][b] = int grad N_a . grad N_b,
 * conv[a][b] = int N_a (a . grad N_b), aa[a][b] = int (a . grad N_a)(a . grad N_b). */
int oracle_q1_element_integrals(const double *X, const double *U, double rho, double mu, double dt, double *scal,
                                double *mass, double *stiff, double *conv, double *aa)
{
    qelem_t E;
    int st = element_pipeline((const double(*)[NDIME])X, (const double(*)[NDIME])U, rho, mu, dt, 2, &E);
    if (st != Q1_OK) return st;
    scal[0] = E.area; scal[1] = E.hleng; scal[2] = E.tau1; scal[3] = E.tau2;
    for (int a = 0; a < PNODE; a++)
        for (int b = 0; b < PNODE; b++) {
            double m = 0.0, k = 0.0, cv = 0.0, q = 0.0;
            for (int g = 0; g < E.ngaus; g++) {
                const double w = E.gpvol[g];
                m += w * E.shape[g][a] * E.shape[g][b];
                k += w * E.wgrgr[g][a][b];
                cv += w * E.shape[g][a] * E.agrau[g][b];
                q += w * E.agrau[g][a] * E.agrau[g][b];
            }
            mass[4 * a + b] = m; stiff[4 * a + b] = k; conv[4 * a + b] = cv; aa[4 * a + b] = q;
        }
    return Q1_OK;
}

/* Validation: every node id in [0, npoin) (else Q1_ERANGE); det J non-zero and of one sign at the
 * four Gauss points of every element (else Q1_EDEGENERATE). *bad receives the first offending element. */
int oracle_q1_validate(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord, int64_t *bad)
{
    *bad = -1;
    if (npoin < 0 || nelem < 0) return Q1_EINVAL;
    for (int64_t e = 0; e < nelem; e++)
        for (int i = 0; i < PNODE; i++)
            if (lnods[4 * e + i] < 0 || lnods[4 * e + i] >= npoin) { *bad = e; return Q1_ERANGE; }
    for (int64_t e = 0; e < nelem; e++) {
        qelem_t E;
        calculate_transients(lnods + 4 * e, coord, NULL, E.elcod, E.elvel);
        if (!calculate_cartesian_derivatives(&E, 2)) { *bad = e; return Q1_EDEGENERATE; }
    }
    return Q1_OK;
}

/* Global assembly (perform_assembly_in_global_system with the block CSR matrix as the target):
 * values [nnzb][3][3] and rhs [npoin][3] are zeroed, then every element adds its 12x12 matrix block
 * by block and its RHS node by node, elements in ascending order; emap [nelem][4][4] is the block
 * index of each element node pair (oracle_pattern). */
int oracle_q1_assemble(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord, const double *veloc,
                       double rho, double mu, double dt, int64_t nnzb, const int32_t *emap, double *values,
                       double *rhs)
{
    memset(values, 0, sizeof(double) * 9 * (size_t)nnzb);
    memset(rhs, 0, sizeof(double) * 3 * (size_t)npoin);
    for (int64_t e = 0; e < nelem; e++) {
        qelem_t E;
        double X[PNODE][NDIME], U[PNODE][NDIME];
        calculate_transients(lnods + 4 * e, coord, veloc, X, U);
        int st = element_pipeline(X, U, rho, mu, dt, 2, &E);
        if (st != Q1_OK) return st;
        for (int a = 0; a < PNODE; a++) {
            for (int b = 0; b < PNODE; b++) {
                double *blk = values + 9 * (size_t)emap[16 * e + 4 * a + b];
                for (int c = 0; c < NDOFN; c++)
                    for (int cp = 0; cp < NDOFN; cp++) blk[3 * c + cp] += E.elauu[3 * a + c][3 * b + cp];
            }
            double *r = rhs + 3 * (size_t)lnods[4 * e + a];
            for (int c = 0; c < NDOFN; c++) r[c] += E.elrhs[3 * a + c];
        }
    }
    return Q1_OK;
}
