/*
 * oracle.c -- plain FP64 CPU oracle for the assembled spectral-element
 * screened-Poisson operator and the conjugate-gradient loop around it
 * (Chalmers, Karakus, Austin, Swirydowicz, Warburton: "hipBone", arXiv:2202.12477).
 *
 * TEST INFRASTRUCTURE ONLY.  The product library never includes, links or calls
 * this file; only the test-suite, the smoke check and the benchmark's CPU
 * baseline do.  It shares no source with the GPU path (its own GLL nodes,
 * derivative matrix, mesh, geometry, random generator and arithmetic).
 *
 * It is written to be checked by eye against the paper, not to be fast:
 *   - every loop is the definition, no blocking or fusion beyond what the paper
 *     states (sum factorisation IS the paper's definition of the gradient:
 *     the Kronecker form of the 3D derivative in the NekBone section);
 *   - built with gcc -O2 -ffp-contract=off, so no FMA contraction happens.
 * A second build of this file (-O3 -march=native -fopenmp, still without
 * contraction) is the benchmark's CPU baseline: there the vector loops run on
 * several threads and oracle_ax_classes / oracle_cg_classes sweep the elements
 * class by class (elements of one class share no node); the parity tests use
 * the single-threaded build.
 *
 * Notation (NekBone section): E elements, degree N, Np = (N+1)^3 local nodes per
 * element, N_L = E*Np, N_G assembled DOFs.  Local node (a,b,c) of an element has
 * index a + (N+1)*(b + (N+1)*c); element (ex,ey,ez) of an nx*ny*nz box has index
 * ex + nx*(ey + ny*ez); global node (I,J,K) has index I + gx*(J + gy*K) with
 * gx = nx*N+1, gy = ny*N+1.  No boundary nodes are masked.
 *
 * Parity-pinned by tests/test_oracle_*.py: GLL closed forms, quadrature
 * exactness, derivative closed forms, dense brute force built by a different
 * route (numpy Legendre + Kronecker products), the Kronecker closed form of an
 * affine box, symmetry, constants, volume and polynomial exactness, a tiny CG
 * against a dense solve, and a manufactured-solution convergence trend.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Counter-based random numbers: splitmix64 (Steele, Lea & Flood, "Fast      */
/* splittable pseudorandom number generators", OOPSLA 2014).  The generator  */
/* state advances by the golden-ratio increment gamma; each output is the    */
/* state passed through the published 64-bit finaliser.  Output number i     */
/* (i = 0, 1, ...) of the sequence started at state s is mix(s + (i+1)gamma). */
/* The paper only says the forcing is pseudo-random (HipBone section); both  */
/* sides of the parity tests implement this generator independently.        */
/* ------------------------------------------------------------------------ */
static const uint64_t SM64_GAMMA = 0x9E3779B97F4A7C15ULL;

static uint64_t sm64_finalise(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Output number i of splitmix64 started from state s. */
uint64_t oracle_splitmix64(uint64_t s, uint64_t i)
{
    return sm64_finalise(s + (i + 1) * SM64_GAMMA);
}

/* Uniform [0,1) double for (seed, stream, index): the stream's own start state
 * is output number `stream` of the sequence started at `seed`; the value is the
 * top 53 bits of output number `index` of that stream, times 2^-53. */
double oracle_uniform(uint64_t seed, uint64_t stream, uint64_t index)
{
    uint64_t start = oracle_splitmix64(seed, stream);
    uint64_t bits = oracle_splitmix64(start, index);
    return (double)(bits >> 11) * (1.0 / 9007199254740992.0);
}

/* Forcing vector b_g = 2U - 1 in [-1, 1), stream 0 (HipBone section: the RHS
 * is filled once by a pseudo-random kernel). */
void oracle_rhs(int64_t n, uint64_t seed, double *b)
{
    for (int64_t g = 0; g < n; ++g)
        b[g] = 2.0 * oracle_uniform(seed, 0, (uint64_t)g) - 1.0;
}

/* ------------------------------------------------------------------------ */
/* Legendre polynomials, GLL nodes/weights, 1D derivative matrix.            */
/* (NekBone section: tensor-product Lagrange bases on GLL points; the 1D SEM  */
/* derivative operator D.  Formulas from Canuto et al. / Deville, Fischer &  */
/* Mund, which the paper cites for the operators.)                          */
/* ------------------------------------------------------------------------ */

/* P_n(x) by Bonnet's recurrence (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}. */
static double legendre_p(int n, double x)
{
    double pm1 = 1.0, p = x;
    if (n == 0) return 1.0;
    for (int k = 1; k < n; ++k) {
        double pp1 = ((2.0 * k + 1.0) * x * p - k * pm1) / (k + 1.0);
        pm1 = p;
        p = pp1;
    }
    return p;
}

/* P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1) inside (-1,1). */
static double legendre_dp(int n, double x)
{
    if (n == 0) return 0.0;
    return n * (x * legendre_p(n, x) - legendre_p(n - 1, x)) / (x * x - 1.0);
}

/* GLL nodes xi[0..N] (ascending; xi_0 = -1, xi_N = 1, interior nodes are the
 * roots of P_N') and weights w_i = 2 / (N (N+1) P_N(xi_i)^2).  The interior
 * roots are found by Newton's method on P_N', with P_N'' taken from Legendre's
 * equation (1-x^2) P'' - 2x P' + N(N+1) P = 0, started from the
 * Chebyshev-Lobatto points -cos(pi i / N).  Returns 0, or -1 if N < 1. */
int oracle_gll(int N, double *xi, double *w)
{
    if (N < 1) return -1;
    xi[0] = -1.0;
    xi[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = -cos(M_PI * i / N);
        for (int it = 0; it < 100; ++it) {
            double p = legendre_p(N, x);
            double dp = legendre_dp(N, x);
            double d2p = (2.0 * x * dp - N * (N + 1.0) * p) / (1.0 - x * x);
            double dx = dp / d2p;
            x -= dx;
            if (fabs(dx) < 1e-15) break;
        }
        xi[i] = x;
    }
    for (int i = 0; i <= N; ++i) {
        double p = legendre_p(N, xi[i]);
        w[i] = 2.0 / (N * (N + 1.0) * p * p);
    }
    return 0;
}

/* D[i][j] = l_j'(xi_i) (row-major, (N+1)x(N+1)) by the closed form for GLL
 * Lagrange bases: P_N(xi_i) / (P_N(xi_j) (xi_i - xi_j)) off the diagonal,
 * -N(N+1)/4 at (0,0), +N(N+1)/4 at (N,N), zero elsewhere on the diagonal. */
int oracle_deriv(int N, const double *xi, double *D)
{
    if (N < 1) return -1;
    int n1 = N + 1;
    for (int i = 0; i <= N; ++i)
        for (int j = 0; j <= N; ++j) {
            double v;
            if (i != j)
                v = legendre_p(N, xi[i]) / (legendre_p(N, xi[j]) * (xi[i] - xi[j]));
            else if (i == 0)
                v = -N * (N + 1.0) / 4.0;
            else if (i == N)
                v = N * (N + 1.0) / 4.0;
            else
                v = 0.0;
            D[i * n1 + j] = v;
        }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Box mesh (NekBone section: a regular mesh of E hexahedra).                */
/* ------------------------------------------------------------------------ */

/* Vertex coordinates V[v][3], v = i + (nx+1)*(j + (ny+1)*k), on [0,1]^3.
 * Reading of the jittered configurations: only vertices strictly inside the
 * box move, each coordinate d by h_d * jitter * (2U - 1), U from stream d+1 of
 * `seed` at index v, so the domain stays exactly the unit cube and the mesh
 * stays conforming (the jitter is keyed by the global vertex). */
int oracle_vertices(int nx, int ny, int nz, double jitter, uint64_t seed, double *V)
{
    if (nx < 1 || ny < 1 || nz < 1) return -1;
    const int n[3] = {nx, ny, nz};
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                int64_t v = i + (int64_t)(nx + 1) * (j + (int64_t)(ny + 1) * k);
                int ijk[3] = {i, j, k};
                int interior = (i > 0 && i < nx && j > 0 && j < ny && k > 0 && k < nz);
                for (int d = 0; d < 3; ++d) {
                    double h = 1.0 / n[d];
                    double c = (double)ijk[d] / n[d];
                    if (interior && jitter != 0.0)
                        c += h * jitter * (2.0 * oracle_uniform(seed, (uint64_t)d + 1, (uint64_t)v) - 1.0);
                    V[3 * v + d] = c;
                }
            }
    return 0;
}

/* Rows of the scatter matrix Z (eq. stiffness): map[e*Np + n] = global index
 * of local node n of element e. */
void oracle_map(int nx, int ny, int nz, int N, int64_t *map)
{
    int n1 = N + 1;
    int64_t Np = (int64_t)n1 * n1 * n1;
    int64_t gx = (int64_t)nx * N + 1, gy = (int64_t)ny * N + 1;
    for (int ez = 0; ez < nz; ++ez)
        for (int ey = 0; ey < ny; ++ey)
            for (int ex = 0; ex < nx; ++ex) {
                int64_t e = ex + (int64_t)nx * (ey + (int64_t)ny * ez);
                for (int c = 0; c <= N; ++c)
                    for (int b = 0; b <= N; ++b)
                        for (int a = 0; a <= N; ++a) {
                            int64_t I = (int64_t)ex * N + a;
                            int64_t J = (int64_t)ey * N + b;
                            int64_t K = (int64_t)ez * N + c;
                            map[e * Np + a + n1 * (b + n1 * c)] = I + gx * (J + gy * K);
                        }
            }
}

/* The same rows for the box with homogeneous Dirichlet conditions on the
 * boundary of [0,1]^3, as in the paper's experiments (their DOF counts are
 * (nN-1)^3): a node on the boundary carries no DOF (map entry -1) and the
 * interior nodes are numbered lexicographically,
 * (I-1) + (gx-2)((J-1) + (gy-2)(K-1)). */
void oracle_map_dirichlet(int nx, int ny, int nz, int N, int64_t *map)
{
    int n1 = N + 1;
    int64_t Np = (int64_t)n1 * n1 * n1;
    int64_t gx = (int64_t)nx * N + 1, gy = (int64_t)ny * N + 1, gz = (int64_t)nz * N + 1;
    for (int ez = 0; ez < nz; ++ez)
        for (int ey = 0; ey < ny; ++ey)
            for (int ex = 0; ex < nx; ++ex) {
                int64_t e = ex + (int64_t)nx * (ey + (int64_t)ny * ez);
                for (int c = 0; c <= N; ++c)
                    for (int b = 0; b <= N; ++b)
                        for (int a = 0; a <= N; ++a) {
                            int64_t I = (int64_t)ex * N + a;
                            int64_t J = (int64_t)ey * N + b;
                            int64_t K = (int64_t)ez * N + c;
                            int boundary = I == 0 || J == 0 || K == 0 || I == gx - 1 || J == gy - 1 || K == gz - 1;
                            map[e * Np + a + n1 * (b + n1 * c)] =
                                boundary ? -1 : (I - 1) + (gx - 2) * ((J - 1) + (gy - 2) * (K - 1));
                        }
            }
}

/* ------------------------------------------------------------------------ */
/* Geometric factors (NekBone section: G^e is the symmetric 3x3 block of     */
/* diagonal matrices holding the metric tensor combined with GLL weights).   */
/* Reading: G_dd' = w_a w_b w_c J sum_i (d xi_d / d x_i)(d xi_d' / d x_i),    */
/* the standard variational form, with the Jacobian of the trilinear map     */
/* taken analytically.  The 7th per-node value is the mass coefficient c:    */
/* mass_kind 0: c = w_a w_b w_c J (A = S + lambda M);                        */
/* mass_kind 1: c = 1 / multiplicity of the node's global DOF, the inverse   */
/* degree weights W of the Poisson Operator section (Z^T W Z = I), which     */
/* makes A = S + lambda I as in eq. poisson.                                 */
/* Layout: geo[(e*7 + f)*Np + n], f = rr, rs, rt, ss, st, tt, c.             */
/* Returns 0, -1 on bad arguments, -2 if some Jacobian is not positive.      */
/* ------------------------------------------------------------------------ */
int oracle_geometry(int nx, int ny, int nz, int N, const double *V, int mass_kind, double *geo)
{
    if (nx < 1 || ny < 1 || nz < 1 || N < 1 || (mass_kind != 0 && mass_kind != 1)) return -1;
    int n1 = N + 1;
    int64_t Np = (int64_t)n1 * n1 * n1;
    double *xi = malloc(sizeof(double) * n1), *w = malloc(sizeof(double) * n1);
    oracle_gll(N, xi, w);
    int status = 0;

    int64_t *mult = NULL;
    int64_t *map = NULL;
    int64_t E = (int64_t)nx * ny * nz;
    if (mass_kind == 1) {
        int64_t NG = ((int64_t)nx * N + 1) * ((int64_t)ny * N + 1) * ((int64_t)nz * N + 1);
        map = malloc(sizeof(int64_t) * E * Np);
        mult = calloc((size_t)NG, sizeof(int64_t));
        oracle_map(nx, ny, nz, N, map);
        for (int64_t m = 0; m < E * Np; ++m) mult[map[m]] += 1;
    }

    for (int ez = 0; ez < nz; ++ez)
        for (int ey = 0; ey < ny; ++ey)
            for (int ex = 0; ex < nx; ++ex) {
                int64_t e = ex + (int64_t)nx * (ey + (int64_t)ny * ez);
                /* the 8 vertices, corner (dx,dy,dz) in {0,1}^3 */
                double X[2][2][2][3];
                for (int dz = 0; dz < 2; ++dz)
                    for (int dy = 0; dy < 2; ++dy)
                        for (int dx = 0; dx < 2; ++dx) {
                            int64_t v = (ex + dx) + (int64_t)(nx + 1) * ((ey + dy) + (int64_t)(ny + 1) * (ez + dz));
                            for (int d = 0; d < 3; ++d) X[dz][dy][dx][d] = V[3 * v + d];
                        }
                for (int c = 0; c <= N; ++c)
                    for (int b = 0; b <= N; ++b)
                        for (int a = 0; a <= N; ++a) {
                            double r[3] = {xi[a], xi[b], xi[c]};
                            /* Jm[i][d] = d x_i / d xi_d of
                             * x(r) = sum_corners X * prod_d (1 + s_d r_d)/2, s_d = 2*corner_d - 1 */
                            double Jm[3][3] = {{0}};
                            for (int dz = 0; dz < 2; ++dz)
                                for (int dy = 0; dy < 2; ++dy)
                                    for (int dx = 0; dx < 2; ++dx) {
                                        double s[3] = {2.0 * dx - 1.0, 2.0 * dy - 1.0, 2.0 * dz - 1.0};
                                        double phi[3] = {(1.0 + s[0] * r[0]) / 2.0, (1.0 + s[1] * r[1]) / 2.0,
                                                         (1.0 + s[2] * r[2]) / 2.0};
                                        double dphi[3] = {s[0] / 2.0 * phi[1] * phi[2],
                                                          phi[0] * s[1] / 2.0 * phi[2],
                                                          phi[0] * phi[1] * s[2] / 2.0};
                                        for (int i = 0; i < 3; ++i)
                                            for (int d = 0; d < 3; ++d)
                                                Jm[i][d] += X[dz][dy][dx][i] * dphi[d];
                                    }
                            double J = Jm[0][0] * (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1])
                                     - Jm[0][1] * (Jm[1][0] * Jm[2][2] - Jm[1][2] * Jm[2][0])
                                     + Jm[0][2] * (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]);
                            if (!(J > 0.0)) status = -2;
                            /* R = Jm^{-1}: R[d][i] = d xi_d / d x_i, by cofactors */
                            double R[3][3];
                            R[0][0] = (Jm[1][1] * Jm[2][2] - Jm[1][2] * Jm[2][1]) / J;
                            R[0][1] = (Jm[0][2] * Jm[2][1] - Jm[0][1] * Jm[2][2]) / J;
                            R[0][2] = (Jm[0][1] * Jm[1][2] - Jm[0][2] * Jm[1][1]) / J;
                            R[1][0] = (Jm[1][2] * Jm[2][0] - Jm[1][0] * Jm[2][2]) / J;
                            R[1][1] = (Jm[0][0] * Jm[2][2] - Jm[0][2] * Jm[2][0]) / J;
                            R[1][2] = (Jm[0][2] * Jm[1][0] - Jm[0][0] * Jm[1][2]) / J;
                            R[2][0] = (Jm[1][0] * Jm[2][1] - Jm[1][1] * Jm[2][0]) / J;
                            R[2][1] = (Jm[0][1] * Jm[2][0] - Jm[0][0] * Jm[2][1]) / J;
                            R[2][2] = (Jm[0][0] * Jm[1][1] - Jm[0][1] * Jm[1][0]) / J;
                            double wJ = w[a] * w[b] * w[c] * J;
                            const int pd[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
                            int64_t n = a + (int64_t)n1 * (b + (int64_t)n1 * c);
                            for (int f = 0; f < 6; ++f) {
                                double g = 0.0;
                                for (int i = 0; i < 3; ++i) g += R[pd[f][0]][i] * R[pd[f][1]][i];
                                geo[(e * 7 + f) * Np + n] = wJ * g;
                            }
                            geo[(e * 7 + 6) * Np + n] = (mass_kind == 0) ? wJ : 1.0 / (double)mult[map[e * Np + n]];
                        }
            }
    free(xi);
    free(w);
    free(mult);
    free(map);
    return status;
}

/* ------------------------------------------------------------------------ */
/* The screened Poisson operator, eq. poisson / eq. stiffness:               */
/*   y = A x = Z^T (S_L + lambda C) Z x,  S_L^e = D^T G^e D,                  */
/* with the gradient D = [D (x) I (x) I; I (x) D (x) I; I (x) I (x) D] acting on */
/* the element's (N+1)^3 nodal values (r along a, s along b, t along c).      */
/* C is diagonal with the 7th geometric value c (see oracle_geometry).        */
/* A map entry -1 (a Dirichlet boundary node) has no DOF: Z puts 0 there and  */
/* Z^T drops its value.                                                       */
/* ------------------------------------------------------------------------ */
/* Work arrays of one element's operator application, (N+1)^3 doubles each. */
typedef struct {
    double *q, *qr, *qs, *qt, *fr, *fs, *ft, *ye;
} ax_work;

static void ax_work_alloc(ax_work *w, int64_t Np)
{
    w->q = malloc(sizeof(double) * Np);
    w->qr = malloc(sizeof(double) * Np); w->qs = malloc(sizeof(double) * Np); w->qt = malloc(sizeof(double) * Np);
    w->fr = malloc(sizeof(double) * Np); w->fs = malloc(sizeof(double) * Np); w->ft = malloc(sizeof(double) * Np);
    w->ye = malloc(sizeof(double) * Np);
}

static void ax_work_free(ax_work *w)
{
    free(w->q); free(w->qr); free(w->qs); free(w->qt); free(w->fr); free(w->fs); free(w->ft); free(w->ye);
}

/* Element e's share of the operator: y += Z_e^T (D^T G^e D + lambda C^e) Z_e x. */
static void ax_element(int64_t e, int N, const double *D, const double *geo, const int64_t *map, double lambda,
                       const double *x, double *y, ax_work *w)
{
    int n1 = N + 1;
    int64_t Np = (int64_t)n1 * n1 * n1;
    double *q = w->q, *qr = w->qr, *qs = w->qs, *qt = w->qt, *fr = w->fr, *fs = w->fs, *ft = w->ft, *ye = w->ye;
#define IDX(a, b, c) ((a) + n1 * ((b) + n1 * (c)))
    const int64_t *me = map + e * Np;
    const double *ge = geo + e * 7 * Np;
    /* Z: gather the element's nodal values from the assembled vector */
    for (int64_t n = 0; n < Np; ++n) q[n] = me[n] >= 0 ? x[me[n]] : 0.0;
    /* D: reference gradient */
    for (int c = 0; c <= N; ++c)
        for (int b = 0; b <= N; ++b)
            for (int a = 0; a <= N; ++a) {
                double sr = 0.0, ss = 0.0, st = 0.0;
                for (int m = 0; m <= N; ++m) {
                    sr += D[a * n1 + m] * q[IDX(m, b, c)];
                    ss += D[b * n1 + m] * q[IDX(a, m, c)];
                    st += D[c * n1 + m] * q[IDX(a, b, m)];
                }
                qr[IDX(a, b, c)] = sr;
                qs[IDX(a, b, c)] = ss;
                qt[IDX(a, b, c)] = st;
            }
    /* G^e: pointwise symmetric metric */
    for (int64_t n = 0; n < Np; ++n) {
        double Grr = ge[0 * Np + n], Grs = ge[1 * Np + n], Grt = ge[2 * Np + n];
        double Gss = ge[3 * Np + n], Gst = ge[4 * Np + n], Gtt = ge[5 * Np + n];
        fr[n] = Grr * qr[n] + Grs * qs[n] + Grt * qt[n];
        fs[n] = Grs * qr[n] + Gss * qs[n] + Gst * qt[n];
        ft[n] = Grt * qr[n] + Gst * qs[n] + Gtt * qt[n];
    }
    /* D^T: divergence, plus the lambda-weighted mass term */
    for (int c = 0; c <= N; ++c)
        for (int b = 0; b <= N; ++b)
            for (int a = 0; a <= N; ++a) {
                double s = 0.0;
                for (int m = 0; m <= N; ++m) {
                    s += D[m * n1 + a] * fr[IDX(m, b, c)];
                    s += D[m * n1 + b] * fs[IDX(a, m, c)];
                    s += D[m * n1 + c] * ft[IDX(a, b, m)];
                }
                int64_t n = IDX(a, b, c);
                ye[n] = s + lambda * ge[6 * Np + n] * q[n];
            }
    /* Z^T: assemble (gather-sum) into the global vector */
    for (int64_t n = 0; n < Np; ++n)
        if (me[n] >= 0) y[me[n]] += ye[n];
#undef IDX
}

/* Element classes for a parallel sweep: the elements order[cls[k] .. cls[k+1])
 * form class k, and no two elements of one class share a global node (on a box:
 * the 8 classes of (ex mod 2, ey mod 2, ez mod 2)).  A NULL class list means
 * every element in index order, one at a time. */
typedef struct {
    const int64_t *order;
    const int64_t *cls;
    int ncls;
} elem_classes;

static void ax_apply(int64_t E, int N, const double *D, const double *geo, const int64_t *map, int64_t NG,
                     double lambda, const double *x, double *y, const elem_classes *ec)
{
    int n1 = N + 1;
    int64_t Np = (int64_t)n1 * n1 * n1;
#pragma omp parallel for schedule(static) if (NG >= 65536)
    for (int64_t g = 0; g < NG; ++g) y[g] = 0.0;
    if (!ec) {
        ax_work w;
        ax_work_alloc(&w, Np);
        for (int64_t e = 0; e < E; ++e) ax_element(e, N, D, geo, map, lambda, x, y, &w);
        ax_work_free(&w);
        return;
    }
    /* the timing build (OpenMP): threads share the elements of one class, which
     * write disjoint entries of y; the classes follow each other */
#pragma omp parallel
    {
        ax_work w;
        ax_work_alloc(&w, Np);
        for (int k = 0; k < ec->ncls; ++k) {
#pragma omp for schedule(static)
            for (int64_t i = ec->cls[k]; i < ec->cls[k + 1]; ++i)
                ax_element(ec->order[i], N, D, geo, map, lambda, x, y, &w);
        }
        ax_work_free(&w);
    }
}

void oracle_ax(int64_t E, int N, const double *D, const double *geo, const int64_t *map, int64_t NG,
               double lambda, const double *x, double *y)
{
    ax_apply(E, N, D, geo, map, NG, lambda, x, y, NULL);
}

/* The same operator with the elements swept class by class (see elem_classes):
 * the CPU baseline's multi-threaded timing; the parity tests use oracle_ax. */
void oracle_ax_classes(int64_t E, int N, const double *D, const double *geo, const int64_t *map, int64_t NG,
                       double lambda, const double *x, double *y, const int64_t *order, const int64_t *cls, int ncls)
{
    elem_classes ec = {order, cls, ncls};
    ax_apply(E, N, D, geo, map, NG, lambda, x, y, &ec);
}

/* The diagonal of the assembled operator, for the Jacobi preconditioner (a
 * NekBone option the paper leaves out): diag(A)_g = sum over the local nodes i
 * of g of (D^T G D + lambda C)_ii, with, at node i = (a,b,c),
 *   (D^T G D)_ii = sum_m D[m][a]^2 G_rr(m,b,c) + sum_m D[m][b]^2 G_ss(a,m,c)
 *                + sum_m D[m][c]^2 G_tt(a,b,m)
 *                + 2 D[a][a] D[b][b] G_rs(i) + 2 D[a][a] D[c][c] G_rt(i)
 *                + 2 D[b][b] D[c][c] G_st(i)
 * (the r-derivative of q at node n depends on q_i only when n shares b and c
 * with i, so the cross terms meet only at n = i). */
void oracle_diag(int64_t E, int N, const double *D, const double *geo, const int64_t *map, int64_t NG,
                 double lambda, double *diag)
{
    int n1 = N + 1;
    int64_t Np = (int64_t)n1 * n1 * n1;
#define IDX(a, b, c) ((a) + n1 * ((b) + n1 * (c)))
    for (int64_t g = 0; g < NG; ++g) diag[g] = 0.0;
    for (int64_t e = 0; e < E; ++e) {
        const int64_t *me = map + e * Np;
        const double *ge = geo + e * 7 * Np;
        for (int c = 0; c <= N; ++c)
            for (int b = 0; b <= N; ++b)
                for (int a = 0; a <= N; ++a) {
                    int64_t i = IDX(a, b, c);
                    if (me[i] < 0) continue;
                    double s = 0.0;
                    for (int m = 0; m <= N; ++m) {
                        s += D[m * n1 + a] * D[m * n1 + a] * ge[0 * Np + IDX(m, b, c)];
                        s += D[m * n1 + b] * D[m * n1 + b] * ge[3 * Np + IDX(a, m, c)];
                        s += D[m * n1 + c] * D[m * n1 + c] * ge[5 * Np + IDX(a, b, m)];
                    }
                    double Daa = D[a * n1 + a], Dbb = D[b * n1 + b], Dcc = D[c * n1 + c];
                    s += 2.0 * Daa * Dbb * ge[1 * Np + i] + 2.0 * Daa * Dcc * ge[2 * Np + i] +
                         2.0 * Dbb * Dcc * ge[4 * Np + i];
                    diag[me[i]] += s + lambda * ge[6 * Np + i];
                }
    }
#undef IDX
}

/* ------------------------------------------------------------------------ */
/* Conjugate gradient, Algorithm 1.                                          */
/* ------------------------------------------------------------------------ */

/* Dot product; compensated (Neumaier) when `compensated` is set, else plain
 * left-to-right.  The paper leaves the summation order open. */
static double dot_serial(int64_t n, const double *u, const double *v, int compensated)
{
    double s = 0.0, comp = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double t = u[i] * v[i];
        if (!compensated) { s += t; continue; }
        double sum = s + t;
        if (fabs(s) >= fabs(t)) comp += (s - sum) + t;
        else comp += (t - sum) + s;
        s = sum;
    }
    return s + comp;
}

static double dot(int64_t n, const double *u, const double *v, int compensated)
{
#ifdef _OPENMP
    /* the timing build with several threads: each thread sums one contiguous
     * block as above, and the block sums are added in block order */
    int nt = omp_get_max_threads();
    if (nt > 1 && n >= 65536) {
        double part[256];
        if (nt > 256) nt = 256;
#pragma omp parallel for num_threads(nt) schedule(static, 1)
        for (int k = 0; k < nt; ++k) {
            int64_t lo = n * k / nt, hi = n * (k + 1) / nt;
            part[k] = dot_serial(hi - lo, u + lo, v + lo, compensated);
        }
        double s = 0.0;
        for (int k = 0; k < nt; ++k) s += part[k];
        return s;
    }
#endif
    return dot_serial(n, u, v, compensated);
}

/*
 * Algorithm 1 with x given on entry as the initial guess.  Before the loop:
 * r_0 = b - A x, p = r_0, rho_0 = r_0.r_0.  Each iteration: Ap = A p;
 * alpha = rho_j / p.Ap; x += alpha p; r -= alpha Ap; rho_{j+1} = r.r;
 * beta = rho_{j+1} / rho_j; p = r + beta p.
 *
 * Stopping (the paper's loop test compares r.r to an absolute epsilon; the
 * benchmark itself runs a fixed 100 iterations):
 *   fixed_iters > 0: run exactly fixed_iters iterations;
 *   otherwise stop once sqrt(rho_j) <= rtol * ||b||, at most max_iter iterations.
 * In both modes stop early if rho_j == 0 (exact solution) or p.Ap <= 0
 * (breakdown).  Histories (length >= iterations+1 for res, >= iterations for
 * alpha/beta/pap) may be NULL: res[j] = sqrt(rho_j).
 * Returns 0 converged / fixed count done, 1 not converged, 2 breakdown.
 */
static int cg_run(int64_t E, int N, const double *D, const double *geo, const int64_t *map, int64_t NG,
                  double lambda, const double *b, double *x, int max_iter, int fixed_iters, double rtol,
                  int compensated, double *res, double *alpha_h, double *beta_h, double *pap_h, int *iters,
                  const elem_classes *ec)
{
    double *r = malloc(sizeof(double) * NG), *p = malloc(sizeof(double) * NG), *Ap = malloc(sizeof(double) * NG);
    ax_apply(E, N, D, geo, map, NG, lambda, x, Ap, ec);
#pragma omp parallel for schedule(static) if (NG >= 65536)
    for (int64_t g = 0; g < NG; ++g) {
        r[g] = b[g] - Ap[g];
        p[g] = r[g];
    }
    double rho = dot(NG, r, r, compensated);
    double bnorm = sqrt(dot(NG, b, b, compensated));
    if (res) res[0] = sqrt(rho);
    int limit = fixed_iters > 0 ? fixed_iters : max_iter;
    int status = 1, j = 0;
    if (fixed_iters <= 0 && sqrt(rho) <= rtol * bnorm) status = 0;
    while (status == 1 && j < limit) {
        if (rho == 0.0) { status = 0; break; }
        ax_apply(E, N, D, geo, map, NG, lambda, p, Ap, ec);
        double pAp = dot(NG, p, Ap, compensated);
        if (pap_h) pap_h[j] = pAp;
        if (!(pAp > 0.0)) { status = 2; break; }
        double alpha = rho / pAp;
#pragma omp parallel for schedule(static) if (NG >= 65536)
        for (int64_t g = 0; g < NG; ++g) x[g] = x[g] + alpha * p[g];
#pragma omp parallel for schedule(static) if (NG >= 65536)
        for (int64_t g = 0; g < NG; ++g) r[g] = r[g] - alpha * Ap[g];
        double rho_new = dot(NG, r, r, compensated);
        double beta = rho_new / rho;
#pragma omp parallel for schedule(static) if (NG >= 65536)
        for (int64_t g = 0; g < NG; ++g) p[g] = r[g] + beta * p[g];
        if (alpha_h) alpha_h[j] = alpha;
        if (beta_h) beta_h[j] = beta;
        rho = rho_new;
        ++j;
        if (res) res[j] = sqrt(rho);
        if (fixed_iters <= 0 && sqrt(rho) <= rtol * bnorm) status = 0;
    }
    if (fixed_iters > 0 && status == 1 && j == limit) status = 0;
    if (iters) *iters = j;
    free(r); free(p); free(Ap);
    return status;
}

int oracle_cg(int64_t E, int N, const double *D, const double *geo, const int64_t *map, int64_t NG,
              double lambda, const double *b, double *x, int max_iter, int fixed_iters, double rtol,
              int compensated, double *res, double *alpha_h, double *beta_h, double *pap_h, int *iters)
{
    return cg_run(E, N, D, geo, map, NG, lambda, b, x, max_iter, fixed_iters, rtol, compensated, res, alpha_h,
                  beta_h, pap_h, iters, NULL);
}

/* Algorithm 1 as oracle_cg, with the operator swept class by class
 * (oracle_ax_classes): the CPU baseline's multi-threaded timing. */
int oracle_cg_classes(int64_t E, int N, const double *D, const double *geo, const int64_t *map, int64_t NG,
                      double lambda, const double *b, double *x, int max_iter, int fixed_iters, double rtol,
                      int compensated, double *res, int *iters, const int64_t *order, const int64_t *cls,
                      int ncls)
{
    elem_classes ec = {order, cls, ncls};
    return cg_run(E, N, D, geo, map, NG, lambda, b, x, max_iter, fixed_iters, rtol, compensated, res, NULL, NULL,
                  NULL, iters, &ec);
}

/* Threads of the timing build (OpenMP); the parity build is single-threaded
 * and reports 1. */
int oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/*
 * Algorithm 1 with the Jacobi preconditioner M = diag(A) (inv = 1/diag(A)):
 * z = M^{-1} r takes the place of r in the direction update and in rho,
 *   r_0 = b - A x, z_0 = M^{-1} r_0, p = z_0, rho_0 = r_0.z_0; each iteration:
 *   Ap = A p; alpha = rho_j / p.Ap; x += alpha p; r -= alpha Ap;
 *   z = M^{-1} r; rho_{j+1} = r.z; beta = rho_{j+1} / rho_j; p = z + beta p.
 * res[j] = ||r_j|| (the unpreconditioned residual, also the stopping test);
 * stopping, histories and return values as oracle_cg.
 */
int oracle_pcg(int64_t E, int N, const double *D, const double *geo, const int64_t *map, int64_t NG,
               double lambda, const double *inv, const double *b, double *x, int max_iter, int fixed_iters,
               double rtol, int compensated, double *res, int *iters)
{
    double *r = malloc(sizeof(double) * NG), *z = malloc(sizeof(double) * NG), *p = malloc(sizeof(double) * NG),
           *Ap = malloc(sizeof(double) * NG);
    oracle_ax(E, N, D, geo, map, NG, lambda, x, Ap);
    for (int64_t g = 0; g < NG; ++g) {
        r[g] = b[g] - Ap[g];
        z[g] = inv[g] * r[g];
        p[g] = z[g];
    }
    double rho = dot(NG, r, z, compensated);
    double rr = dot(NG, r, r, compensated);
    double bnorm = sqrt(dot(NG, b, b, compensated));
    if (res) res[0] = sqrt(rr);
    int limit = fixed_iters > 0 ? fixed_iters : max_iter;
    int status = 1, j = 0;
    if (fixed_iters <= 0 && sqrt(rr) <= rtol * bnorm) status = 0;
    while (status == 1 && j < limit) {
        if (rho == 0.0) { status = 0; break; }
        oracle_ax(E, N, D, geo, map, NG, lambda, p, Ap);
        double pAp = dot(NG, p, Ap, compensated);
        if (!(pAp > 0.0)) { status = 2; break; }
        double alpha = rho / pAp;
        for (int64_t g = 0; g < NG; ++g) x[g] = x[g] + alpha * p[g];
        for (int64_t g = 0; g < NG; ++g) r[g] = r[g] - alpha * Ap[g];
        for (int64_t g = 0; g < NG; ++g) z[g] = inv[g] * r[g];
        double rho_new = dot(NG, r, z, compensated);
        rr = dot(NG, r, r, compensated);
        double beta = rho_new / rho;
        for (int64_t g = 0; g < NG; ++g) p[g] = z[g] + beta * p[g];
        rho = rho_new;
        ++j;
        if (res) res[j] = sqrt(rr);
        if (fixed_iters <= 0 && sqrt(rr) <= rtol * bnorm) status = 0;
    }
    if (fixed_iters > 0 && status == 1 && j == limit) status = 0;
    if (iters) *iters = j;
    free(r); free(z); free(p); free(Ap);
    return status;
}
