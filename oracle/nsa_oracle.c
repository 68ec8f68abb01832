/*
 * nsa_oracle.c -- plain, slow, serial FP64 CPU oracle for P1-tetrahedron incompressible
 * Navier-Stokes element assembly into a block-CSR (BSR, 4x4 blocks) matrix plus RHS.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or load this file:
 * it is used by the tests, by the package's smoke check and by the CPU-baseline leg of the
 * benchmark, and it shares no code, header, table or constant with the HIP library.
 *
 * What it computes follows the paper (Brown, "Porting incompressible flow matrix assembly to
 * FPGAs...", arXiv 2111.05651):
 *   - Sec. II-A, Listing 1: per element, in this order, gather nodal data, form the Cartesian
 *     derivatives of the shape functions, the Gauss-point values, the stabilisation parameters,
 *     the element operators, the convective term with the RHS, the viscous term, and finally
 *     scatter into the global system.  All arithmetic is double precision.
 *   - Sec. II-A, Listing 2: elvel(j,i) = veloc(j, lnods(e,i)), elcod likewise (4 nodes, 3 dims);
 *     the assembly accumulates through the same lnods map.
 *   - Sec. III-A, Listings 3/4: the velocity-velocity block elauu is indexed by
 *     dofv = node*NUM_DIMS + dim and every (idime, jdime) pair receives a common term, with an
 *     extra term on the diagonal jdime == idime.
 * The paper prints no equations. The formulation here (Oseen-linearised backward-Euler
 * Navier-Stokes with SUPG/PSPG/grad-div stabilisation, 4-point Gauss rule, dof 4*node + c with
 * pressure as c = 3, rows = test functions, BSR-4 output) is the documented reading of the paper;
 * each such reading is listed with the design notes of the repository.
 *
 * Compile: gcc -O2 -ffp-contract=off -fPIC -shared -o liboracle.so nsa_oracle.c -lm
 * (no FMA contraction, IEEE round-to-nearest; loops run in ascending index order). That serial build
 * is the oracle the tests pin and compare against. The same source built with -fopenmp runs the
 * element loops of oracle_assemble and oracle_residual on all host threads with atomic adds into the
 * global arrays (sums in a run-dependent order); it only times the CPU baseline.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ERANGE (-2)
#define OR_EDEGENERATE (-3)
#define OR_ENOMEM (-4)

#define PNODE 4 /* nodes per linear tetrahedron (Sec. II-A) */
#define NDIME 3 /* space dimensions (Sec. II-A) */
#define PGAUS 4 /* Gauss points: 4-point degree-2 rule (reading of PGAUS_SIZE) */
#define NDOFN 4 /* dofs per node: u, v, w, p */
#define NEVAT (PNODE * NDOFN)

/* Per-element intermediate values, named after the paper's temporaries (Sec. II-A). */
typedef struct {
    double elcod[PNODE][NDIME]; /* nodal coordinates */
    double elvel[PNODE][NDIME]; /* nodal velocities */
    double jac[NDIME][NDIME];   /* jac[r][s] = d x_r / d xi_s */
    double detjac;
    double gpcar[PNODE][NDIME]; /* d N_a / d x_d, constant over a linear tet */
    double vol;                 /* element volume |det J| / 6 */
    double gpvol[PGAUS];        /* Gauss weight times |det J| */
    double shape[PGAUS][PNODE]; /* N_a at Gauss point g */
    double gpvel[PGAUS][NDIME]; /* velocity (advection and previous step) at Gauss point g */
    double agrau[PGAUS][PNODE]; /* a_g . grad N_a */
    double hleng;               /* element length */
    double abar[NDIME];         /* element-mean velocity */
    double tau1, tau2;          /* momentum/continuity and grad-div stabilisation */
    double wgrgr[PNODE][PNODE]; /* grad N_a . grad N_b */
    double elauu[NEVAT][NEVAT]; /* element matrix, rows = test (a,c), cols = trial (b,c') */
    double elrhs[NEVAT];        /* element right-hand side */
} element_t;

/* Gather (calculate_transients, Listing 2): elvel(j,i) = veloc(j, lnods(e,i)), elcod likewise.
 * veloc may be NULL (coordinates only). */
static void calculate_transients(const int32_t *ln, const double *coord, const double *veloc,
                                 double elcod[PNODE][NDIME], double elvel[PNODE][NDIME])
{
    for (int i = 0; i < PNODE; i++) {
        int64_t ipoin = ln[i];
        for (int j = 0; j < NDIME; j++) {
            elvel[i][j] = veloc ? veloc[3 * ipoin + j] : 0.0;
            elcod[i][j] = coord[3 * ipoin + j];
        }
    }
}

/* Jacobian of the affine map from the reference tet (0, e1, e2, e3), its inverse, and the
 * Cartesian shape-function derivatives (calculate_cartesian_derivatives). Returns 0 if the
 * element is degenerate (det J == 0). */
static int calculate_cartesian_derivatives(element_t *E)
{
    double (*J)[NDIME] = E->jac;
    for (int r = 0; r < NDIME; r++)
        for (int s = 0; s < NDIME; s++)
            J[r][s] = E->elcod[s + 1][r] - E->elcod[0][r];
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    E->detjac = det;
    if (!(det != 0.0) || !isfinite(det)) return 0;
    /* cofactor matrix; inverse = transpose(cofactor) / det */
    double cof[NDIME][NDIME];
    cof[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    cof[0][1] = -(J[1][0] * J[2][2] - J[1][2] * J[2][0]);
    cof[0][2] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    cof[1][0] = -(J[0][1] * J[2][2] - J[0][2] * J[2][1]);
    cof[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    cof[1][2] = -(J[0][0] * J[2][1] - J[0][1] * J[2][0]);
    cof[2][0] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    cof[2][1] = -(J[0][0] * J[1][2] - J[0][2] * J[1][0]);
    cof[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    double jinv[NDIME][NDIME];
    for (int s = 0; s < NDIME; s++)
        for (int d = 0; d < NDIME; d++)
            jinv[s][d] = cof[d][s] / det;
    /* N_{s+1} = xi_s, N_0 = 1 - xi_1 - xi_2 - xi_3: grad N_{s+1} = row s of J^{-1} */
    for (int d = 0; d < NDIME; d++) {
        E->gpcar[0][d] = 0.0;
        for (int s = 0; s < NDIME; s++) {
            E->gpcar[s + 1][d] = jinv[s][d];
            E->gpcar[0][d] -= jinv[s][d];
        }
    }
    E->vol = fabs(det) / 6.0;
    /* 4-point rule on the tet: point g sits at barycentric weight alpha on node g and beta on
     * the other three, weight 1/4 of the volume each. */
    const double sq5 = sqrt(5.0);
    const double alpha = (5.0 + 3.0 * sq5) / 20.0;
    const double beta = (5.0 - sq5) / 20.0;
    for (int g = 0; g < PGAUS; g++) {
        E->gpvol[g] = 0.25 * E->vol;
        for (int a = 0; a < PNODE; a++) E->shape[g][a] = (a == g) ? alpha : beta;
    }
    return 1;
}

/* Velocity at the Gauss points and its projection on the shape-function gradients
 * (calculate_gauss_point_values). */
static void calculate_gauss_point_values(element_t *E)
{
    for (int g = 0; g < PGAUS; g++) {
        for (int c = 0; c < NDIME; c++) {
            double s = 0.0;
            for (int a = 0; a < PNODE; a++) s += E->shape[g][a] * E->elvel[a][c];
            E->gpvel[g][c] = s;
        }
    }
}

/* Element length and stabilisation parameters (calculate_tau_and_tim). */
static void calculate_tau_and_tim(element_t *E, double rho, double mu, double dt)
{
    E->hleng = cbrt(6.0 * E->vol);
    double an2 = 0.0;
    for (int c = 0; c < NDIME; c++) {
        double s = 0.0;
        for (int a = 0; a < PNODE; a++) s += E->elvel[a][c];
        E->abar[c] = 0.25 * s;
        an2 += E->abar[c] * E->abar[c];
    }
    double anorm = sqrt(an2);
    double h = E->hleng;
    E->tau1 = 1.0 / (rho / dt + 4.0 * mu / (h * h) + 2.0 * rho * anorm / h);
    E->tau2 = mu + 0.5 * rho * anorm * h;
}

/* a . grad N at the Gauss points and grad N . grad N (calculate_element_matricies). */
static void calculate_element_matricies(element_t *E)
{
    for (int g = 0; g < PGAUS; g++)
        for (int a = 0; a < PNODE; a++) {
            double s = 0.0;
            for (int d = 0; d < NDIME; d++) s += E->gpvel[g][d] * E->gpcar[a][d];
            E->agrau[g][a] = s;
        }
    for (int a = 0; a < PNODE; a++)
        for (int b = 0; b < PNODE; b++) {
            double s = 0.0;
            for (int d = 0; d < NDIME; d++) s += E->gpcar[a][d] * E->gpcar[b][d];
            E->wgrgr[a][b] = s;
        }
}

/* Time, convective, SUPG and pressure-coupling terms plus the RHS, integrated Gauss point by
 * Gauss point (calculate_convective_term_and_RHS). Rows are test functions (a,c), columns
 * trial functions (b,c'); dof index 4*node + c, c = 3 is pressure. */
static void calculate_convective_term_and_RHS(element_t *E, double rho, double dt)
{
    const double rdt = rho / dt;
    const double t1 = E->tau1;
    memset(E->elauu, 0, sizeof(E->elauu));
    memset(E->elrhs, 0, sizeof(E->elrhs));
    for (int g = 0; g < PGAUS; g++) {
        const double w = E->gpvol[g];
        for (int a = 0; a < PNODE; a++) {
            const double Na = E->shape[g][a];
            const double aga = E->agrau[g][a];
            for (int b = 0; b < PNODE; b++) {
                const double Nb = E->shape[g][b];
                const double agb = E->agrau[g][b];
                /* momentum, same component: mass/dt + Galerkin convection + SUPG on both */
                const double tuu = rdt * Na * Nb + rho * Na * agb + t1 * rho * aga * (rho * agb + rdt * Nb);
                for (int c = 0; c < NDIME; c++)
                    E->elauu[4 * a + c][4 * b + c] += w * tuu;
                for (int c = 0; c < NDIME; c++) {
                    /* velocity test, pressure trial: -(p, div v) + SUPG (rho a.grad v, grad p) */
                    E->elauu[4 * a + c][4 * b + 3] += w * (-Nb * E->gpcar[a][c] + t1 * rho * aga * E->gpcar[b][c]);
                    /* pressure test, velocity trial: (q, div u) + PSPG (grad q, rho u/dt + rho a.grad u) */
                    E->elauu[4 * a + 3][4 * b + c] += w * (Na * E->gpcar[b][c] + t1 * E->gpcar[a][c] * (rdt * Nb + rho * agb));
                }
            }
            /* RHS: (rho/dt) u^n tested with the Galerkin and SUPG weights; PSPG for pressure */
            for (int c = 0; c < NDIME; c++)
                E->elrhs[4 * a + c] += w * (rdt * E->gpvel[g][c] * Na + t1 * rho * rdt * aga * E->gpvel[g][c]);
            double gdu = 0.0;
            for (int d = 0; d < NDIME; d++) gdu += E->gpcar[a][d] * E->gpvel[g][d];
            E->elrhs[4 * a + 3] += w * t1 * rdt * gdu;
        }
    }
}

/* Viscous term mu (grad u + grad u^T) : grad v, grad-div tau2 (div u)(div v) and the PSPG
 * pressure Laplacian tau1 (grad q, grad p) (calculate_viscous_term). */
static void calculate_viscous_term(element_t *E, double mu)
{
    const double V = E->vol;
    for (int a = 0; a < PNODE; a++)
        for (int b = 0; b < PNODE; b++) {
            for (int c = 0; c < NDIME; c++)
                for (int cp = 0; cp < NDIME; cp++) {
                    double v = mu * V * E->gpcar[a][cp] * E->gpcar[b][c]
                             + E->tau2 * V * E->gpcar[a][c] * E->gpcar[b][cp];
                    if (c == cp) v += mu * V * E->wgrgr[a][b];
                    E->elauu[4 * a + c][4 * b + cp] += v;
                }
            E->elauu[4 * a + 3][4 * b + 3] += E->tau1 * V * E->wgrgr[a][b];
        }
}

/* Full element pipeline of Listing 1 for one element, coordinates and velocities given. */
static int element_pipeline(const double X[PNODE][NDIME], const double U[PNODE][NDIME], double rho,
                            double mu, double dt, element_t *E)
{
    memcpy(E->elcod, X, sizeof(E->elcod));
    memcpy(E->elvel, U, sizeof(E->elvel));
    if (!calculate_cartesian_derivatives(E)) return OR_EDEGENERATE;
    calculate_gauss_point_values(E);
    calculate_tau_and_tim(E, rho, mu, dt);
    calculate_element_matricies(E);
    calculate_convective_term_and_RHS(E, rho, dt);
    calculate_viscous_term(E, mu);
    return OR_OK;
}

/* ------------------------------------------------------------------------------------------ */
/* Exported entry points                                                                       */
/* ------------------------------------------------------------------------------------------ */

/* One element: X, U are [4][3] row-major, A is [16][16] row-major, b is [16]. */
int oracle_element(const double *X, const double *U, double rho, double mu, double dt, double *A,
                   double *b)
{
    element_t E;
    int st = element_pipeline((const double(*)[NDIME])X, (const double(*)[NDIME])U, rho, mu, dt, &E);
    if (st != OR_OK) return st;
    memcpy(A, E.elauu, sizeof(E.elauu));
    memcpy(b, E.elrhs, sizeof(E.elrhs));
    return OR_OK;
}

/* Element intermediates exposed for pinning the integration: out[0..3] V, h, tau1, tau2;
 * gpcar [4][3]; then the Gauss-rule integrals
 *   mass[a][b] = int N_a N_b, conv[a][b] = int N_a (a.grad N_b), aa[a][b] = int (a.grad N_a)(a.grad N_b),
 *   iag[a] = int a.grad N_a, un[a][c] = int u_c N_a, au[a][c] = int (a.grad N_a) u_c. */
int oracle_element_integrals(const double *X, const double *U, double rho, double mu, double dt,
                             double *scal, double *gpcar, double *mass, double *conv, double *aa,
                             double *iag, double *un, double *au)
{
    element_t E;
    int st = element_pipeline((const double(*)[NDIME])X, (const double(*)[NDIME])U, rho, mu, dt, &E);
    if (st != OR_OK) return st;
    scal[0] = E.vol; scal[1] = E.hleng; scal[2] = E.tau1; scal[3] = E.tau2;
    memcpy(gpcar, E.gpcar, sizeof(E.gpcar));
    for (int a = 0; a < PNODE; a++) {
        iag[a] = 0.0;
        for (int b = 0; b < PNODE; b++) { mass[4 * a + b] = 0.0; conv[4 * a + b] = 0.0; aa[4 * a + b] = 0.0; }
        for (int c = 0; c < NDIME; c++) { un[3 * a + c] = 0.0; au[3 * a + c] = 0.0; }
    }
    for (int g = 0; g < PGAUS; g++) {
        double w = E.gpvol[g];
        for (int a = 0; a < PNODE; a++) {
            iag[a] += w * E.agrau[g][a];
            for (int b = 0; b < PNODE; b++) {
                mass[4 * a + b] += w * E.shape[g][a] * E.shape[g][b];
                conv[4 * a + b] += w * E.shape[g][a] * E.agrau[g][b];
                aa[4 * a + b] += w * E.agrau[g][a] * E.agrau[g][b];
            }
            for (int c = 0; c < NDIME; c++) {
                un[3 * a + c] += w * E.gpvel[g][c] * E.shape[g][a];
                au[3 * a + c] += w * E.agrau[g][a] * E.gpvel[g][c];
            }
        }
    }
    return OR_OK;
}

/* Validation: every node id in [0, npoin) (else OR_ERANGE), every element with det J != 0
 * (else OR_EDEGENERATE). *bad receives the first offending element, or -1. */
int oracle_validate(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord, int64_t *bad)
{
    *bad = -1;
    if (npoin < 0 || nelem < 0) return OR_EINVAL;
    for (int64_t e = 0; e < nelem; e++)
        for (int i = 0; i < PNODE; i++)
            if (lnods[4 * e + i] < 0 || lnods[4 * e + i] >= npoin) { *bad = e; return OR_ERANGE; }
    for (int64_t e = 0; e < nelem; e++) {
        element_t E;
        calculate_transients(lnods + 4 * e, coord, NULL, E.elcod, E.elvel);
        if (!calculate_cartesian_derivatives(&E)) { *bad = e; return OR_EDEGENERATE; }
    }
    return OR_OK;
}

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/* Sparsity pattern of the node graph as block CSR: row i holds every node j that shares an
 * element with i (diagonal included), columns strictly ascending. bptr has npoin+1 entries,
 * bcol must hold 16*nelem entries (an upper bound), emap[e][a][b] receives the block index of
 * the node pair (lnods[e][a], lnods[e][b]). Returns nnzb, or a negative status. */
int64_t oracle_pattern(int64_t npoin, int64_t nelem, const int32_t *lnods, int64_t *bptr,
                       int32_t *bcol, int32_t *emap)
{
    /* Step 1: every (row, col) pair of every element, duplicates kept, bucketed by row. */
    int64_t *cnt = calloc((size_t)npoin + 1, sizeof(int64_t));
    if (!cnt) return OR_ENOMEM;
    for (int64_t e = 0; e < nelem; e++)
        for (int a = 0; a < PNODE; a++) cnt[lnods[4 * e + a] + 1] += PNODE;
    for (int64_t i = 0; i < npoin; i++) cnt[i + 1] += cnt[i];
    int32_t *pairs = malloc(sizeof(int32_t) * (size_t)(cnt[npoin] > 0 ? cnt[npoin] : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(npoin > 0 ? npoin : 1));
    if (!pairs || !fill) { free(cnt); free(pairs); free(fill); return OR_ENOMEM; }
    for (int64_t i = 0; i < npoin; i++) fill[i] = cnt[i];
    for (int64_t e = 0; e < nelem; e++)
        for (int a = 0; a < PNODE; a++)
            for (int b = 0; b < PNODE; b++) pairs[fill[lnods[4 * e + a]]++] = lnods[4 * e + b];
    /* Step 2: each row sorted, duplicates dropped. */
    int64_t nnzb = 0;
    bptr[0] = 0;
    for (int64_t i = 0; i < npoin; i++) {
        int64_t lo = cnt[i], hi = cnt[i + 1];
        qsort(pairs + lo, (size_t)(hi - lo), sizeof(int32_t), cmp_i32);
        for (int64_t k = lo; k < hi; k++)
            if (k == lo || pairs[k] != pairs[k - 1]) bcol[nnzb++] = pairs[k];
        bptr[i + 1] = nnzb;
    }
    free(pairs); free(fill); free(cnt);
    /* Step 3: block index of each element node pair, by binary search in its row. */
    for (int64_t e = 0; e < nelem; e++)
        for (int a = 0; a < PNODE; a++) {
            int64_t row = lnods[4 * e + a];
            for (int b = 0; b < PNODE; b++) {
                int32_t col = lnods[4 * e + b];
                int64_t lo = bptr[row], hi = bptr[row + 1] - 1;
                while (lo < hi) {
                    int64_t mid = (lo + hi) / 2;
                    if (bcol[mid] < col) lo = mid + 1; else hi = mid;
                }
                emap[16 * e + 4 * a + b] = (int32_t)lo;
            }
        }
    return nnzb;
}

/* Global assembly (perform_assembly_in_global_system, Listing 2, with the block CSR matrix
 * as the target): values [nnzb][4][4] and rhs [npoin][4] are zeroed, then every element adds
 * its 16x16 matrix block by block and its RHS node by node, elements in ascending order. */
int oracle_assemble(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord,
                    const double *veloc, double rho, double mu, double dt, int64_t nnzb,
                    const int32_t *emap, double *values, double *rhs)
{
    memset(values, 0, sizeof(double) * 16 * (size_t)nnzb);
    memset(rhs, 0, sizeof(double) * 4 * (size_t)npoin);
    int status = OR_OK;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nelem; e++) {
        element_t E;
        double X[PNODE][NDIME], U[PNODE][NDIME];
        calculate_transients(lnods + 4 * e, coord, veloc, X, U);
        int st = element_pipeline(X, U, rho, mu, dt, &E);
        if (st != OR_OK) {
#pragma omp atomic write
            status = st;
            continue;
        }
        for (int a = 0; a < PNODE; a++) {
            for (int b = 0; b < PNODE; b++) {
                double *blk = values + 16 * (size_t)emap[16 * e + 4 * a + b];
                for (int c = 0; c < NDOFN; c++)
                    for (int cp = 0; cp < NDOFN; cp++) {
#pragma omp atomic
                        blk[4 * c + cp] += E.elauu[4 * a + c][4 * b + cp];
                    }
            }
            double *r = rhs + 4 * (size_t)lnods[4 * e + a];
            for (int c = 0; c < NDOFN; c++) {
#pragma omp atomic
                r[c] += E.elrhs[4 * a + c];
            }
        }
    }
    return status;
}

/* Threads the element loops use: 1 in the serial build. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Explicit-residual assembly: the outputs of Listing 2 (rhsid, dt_rho_nsi, mass_rho_nsi) instead
 * of a matrix. Per element, after the pipeline of Listing 1:
 *   elrbu(c, a)  = elrhs[4a+c] - sum_b sum_c' elauu[4a+c][4b+c'] * elvel[b][c']   (c, c' < 3)
 *                  (the momentum residual of the element with the nodal velocities as the trial
 *                  field; the pressure is not an input of Listing 2 and enters as zero);
 *   eldtrho(a)   = sum_g gpvol[g] * shape[g][a] * tau1   (tau-weighted lumped mass), and
 *   elmurho(a)   = sum_g gpvol[g] * shape[g][a] * rho    (rho-weighted lumped mass),
 * the two per-node quantities calculate_tau_and_tim hands to the scatter (a reading: the paper does
 * not define them). rhsid [npoin][3], dt_rho [npoin] and mass_rho [npoin] are zeroed, then every
 * element adds into the rows of its nodes through lnods, elements in ascending order. */
int oracle_residual(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord,
                    const double *veloc, double rho, double mu, double dt, double *rhsid,
                    double *dt_rho, double *mass_rho)
{
    memset(rhsid, 0, sizeof(double) * 3 * (size_t)npoin);
    memset(dt_rho, 0, sizeof(double) * (size_t)npoin);
    memset(mass_rho, 0, sizeof(double) * (size_t)npoin);
    int status = OR_OK;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nelem; e++) {
        element_t E;
        double X[PNODE][NDIME], U[PNODE][NDIME];
        calculate_transients(lnods + 4 * e, coord, veloc, X, U);
        int st = element_pipeline(X, U, rho, mu, dt, &E);
        if (st != OR_OK) {
#pragma omp atomic write
            status = st;
            continue;
        }
        for (int a = 0; a < PNODE; a++) {
            int64_t ipoin = lnods[4 * e + a];
            for (int c = 0; c < NDIME; c++) {
                double r = E.elrhs[4 * a + c];
                for (int b = 0; b < PNODE; b++)
                    for (int cp = 0; cp < NDIME; cp++) r -= E.elauu[4 * a + c][4 * b + cp] * E.elvel[b][cp];
#pragma omp atomic
                rhsid[3 * ipoin + c] += r;
            }
            double lump = 0.0;
            for (int g = 0; g < PGAUS; g++) lump += E.gpvol[g] * E.shape[g][a];
            const double dtr = lump * E.tau1, mr = lump * rho;
#pragma omp atomic
            dt_rho[ipoin] += dtr;
#pragma omp atomic
            mass_rho[ipoin] += mr;
        }
    }
    return status;
}

/* Assembly restricted to a sample of rows, for checking large meshes one row at a time.
 * rowslot[i] is the position of node i in the sample (or -1). For sampled row s, its pattern
 * is rebuilt from the elements that touch it: cols[s*maxdeg + k] (ascending, -1 padded),
 * deg[s], vals[(s*maxdeg + k)*16 + 4c + c'] and rhs_s[4s + c]. Returns OR_OK, or OR_ENOMEM if
 * a sampled row has more than maxdeg distinct columns. */
int oracle_assemble_rows(int64_t npoin, int64_t nelem, const int32_t *lnods, const double *coord,
                         const double *veloc, double rho, double mu, double dt, int64_t nsample,
                         const int64_t *rowslot, int32_t maxdeg, int32_t *cols, int32_t *deg,
                         double *vals, double *rhs_s)
{
    (void)npoin;
    for (int64_t s = 0; s < nsample; s++) {
        deg[s] = 0;
        for (int k = 0; k < maxdeg; k++) cols[s * maxdeg + k] = -1;
    }
    memset(vals, 0, sizeof(double) * 16 * (size_t)nsample * (size_t)maxdeg);
    memset(rhs_s, 0, sizeof(double) * 4 * (size_t)nsample);
    /* pass 1: column sets */
    for (int64_t e = 0; e < nelem; e++)
        for (int a = 0; a < PNODE; a++) {
            int64_t s = rowslot[lnods[4 * e + a]];
            if (s < 0) continue;
            for (int b = 0; b < PNODE; b++) {
                int32_t col = lnods[4 * e + b], *row = cols + s * maxdeg;
                int k = 0;
                while (k < deg[s] && row[k] < col) k++;
                if (k < deg[s] && row[k] == col) continue;
                if (deg[s] >= maxdeg) return OR_ENOMEM;
                memmove(row + k + 1, row + k, sizeof(int32_t) * (size_t)(deg[s] - k));
                row[k] = col;
                deg[s]++;
            }
        }
    /* pass 2: values */
    for (int64_t e = 0; e < nelem; e++) {
        int touched = 0;
        for (int a = 0; a < PNODE; a++) touched |= rowslot[lnods[4 * e + a]] >= 0;
        if (!touched) continue;
        element_t E;
        double X[PNODE][NDIME], U[PNODE][NDIME];
        calculate_transients(lnods + 4 * e, coord, veloc, X, U);
        int st = element_pipeline(X, U, rho, mu, dt, &E);
        if (st != OR_OK) return st;
        for (int a = 0; a < PNODE; a++) {
            int64_t s = rowslot[lnods[4 * e + a]];
            if (s < 0) continue;
            for (int b = 0; b < PNODE; b++) {
                int32_t col = lnods[4 * e + b], *row = cols + s * maxdeg;
                int k = 0;
                while (row[k] != col) k++;
                double *blk = vals + 16 * ((size_t)s * maxdeg + k);
                for (int c = 0; c < NDOFN; c++)
                    for (int cp = 0; cp < NDOFN; cp++) blk[4 * c + cp] += E.elauu[4 * a + c][4 * b + cp];
            }
            for (int c = 0; c < NDOFN; c++) rhs_s[4 * s + c] += E.elrhs[4 * a + c];
        }
    }
    return OR_OK;
}
