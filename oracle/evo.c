/*
 * evo.c -- plain FP64 CPU oracle of the explicit Enskog-Vlasov lattice
 * Boltzmann step of Karlin & Hosseini, "Practical Kinetic Models for Dense
 * Fluids" (arXiv 2508.00577).
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists so that the tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the HIP library
 * against the paper.  It shares no code, header, table or helper with the HIP
 * path and the product never links it.
 *
 * Style: every stage of the update is a separate loop over the whole lattice,
 * in the order in which the paper introduces the quantities, writing a full
 * field; nothing is fused, blocked or reordered.  Arithmetic is FP64 and the
 * library is built with -ffp-contract=off.
 *
 * Readings of the paper taken here where it is silent (each one is listed
 * with its reason in the design notes of the repository):
 *   - 2D runs use D2Q9, the z-summed form of the paper's D3Q27 product
 *     equilibria; the thermodynamics stay three-dimensional ((3/2) rho R T).
 *   - Gradients and the Laplacian are the isotropic lattice-weighted stencils
 *     d_a phi = 3 sum_i w_i c_ia phi(x+c_i),
 *     lap phi = 6 sum_i w_i (phi(x+c_i) - phi(x)).
 *   - The mean-field force is written in conservative form a grad(rho^2).
 *   - The sign in front of the first term of the diagonal correction
 *     Phi_aa (eq. correction_u) is a parameter s_phi; the tests decide it from
 *     the hydrodynamic limit the paper states (eq. viscosity, zero bulk
 *     viscosity).
 *   - f* takes the unshifted P0/rho as printed in eq. f_star; g* is
 *     g^eq(u*, RT*) with P0/rho evaluated at RT* (eq. gstar).
 *   - The energy half-step uses the total energy of g:
 *     rho E = sum g + (dt/2)(u.F + Qtilde), which equals eq. T_shift.
 *   - Enskog's pressure P_E = rho R T (1 + b rho chi) with the contact value
 *     chi of the pair distribution: the van der Waals form the paper uses,
 *     chi = 1/(1 - b rho), or Carnahan-Starling's hard-sphere value
 *     chi = (1 - eta/2)/(1 - eta)^3 with eta = b rho/4 (Carnahan & Starling,
 *     J. Chem. Phys. 51, 635 (1969)).  Either way P_E = rho R T Z(rho) and
 *     gamma_0 of eq. gamma follows from Z.
 *   - Prandtl number (optional; the concluding paragraph names a
 *     quasi-equilibrium relaxation of g as the way to lift Pr = 1, the paper
 *     gives no scheme).  g relaxes with beta_g = 1/(2 tau_g + 1), tau_g =
 *     tau/Pr, in both terms of eq. pre_LBM, and the part of its energy flux
 *     that carries the viscous heating, u . Pi^neq with Pi^neq the second
 *     moment of fh - f^eq, keeps f's beta through the quasi-equilibrium term
 *     2 (beta_g - beta) dg, dg_i = (1/2) c_i . (u . Pi^neq) on the axis
 *     directions (zero mass and energy, flux u . Pi^neq).  Pr = 1 is the
 *     paper's scheme exactly; k = (5/2) R mu/Pr.
 *   - Walls (the thermal Couette flow after eq. P0E, Fig. 2; optional, normal
 *     to x at x = -1/2 and x = nx - 1/2, the second moving with U_w along y,
 *     both at T_w): diffuse reflection.  A population entering the fluid from
 *     a wall is the wall's equilibrium f^eq(u_w, P0/rho at T_w), g^eq alike,
 *     times the density that makes the mass entering the cell equal the mass
 *     its populations send into the wall in the same step.  Stencils read a
 *     field beyond a wall from its linear extrapolation through the two
 *     nearest cells.
 *
 * Lattice units: dt = dx = 1, particle mass m = 1 so rho = n.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 27

typedef struct {
    int D, Q, nx, ny, nz;
    long N;
    int c[QMAX][3];
    double w[QMAX];
    /* model parameters */
    double R, a, b, kappa, tau, lambda, sphi;
    double prandtl; /* tau/tau_g of the energy populations (1: the paper's scheme) */
    int eos; /* 0: van der Waals contact factor, 1: Carnahan-Starling */
    int walls;       /* 1: diffuse walls normal to x (see the header) */
    double Tw, Uw;   /* wall temperature, speed of the wall at x = nx - 1/2 (along y) */
    /* state S_n: post-collision, pre-stream populations, layout [i][cell] */
    double *f, *g;
    /* work fields, one value (or D values, layout [alpha][cell]) per cell */
    double *fh, *gh;
    double *rho, *j, *e, *rho2, *lap, *F;
    double *u, *rhoE, *RT, *Th, *P0;
    double *divu, *M, *Phi, *tdiff, *qp, *Phip;
    double *us, *RTs, *Ths;
    long step;
} evo_t;

/* ------------------------------------------------------------------ lattice */

/* Velocity index i = sum_a (c_ia + 1) 3^a; the opposite direction is Q-1-i.
 * Weights are the product of the 1D weights 2/3 (c = 0) and 1/6 (c = +-1),
 * which is the rest equilibrium at P0/rho = 1/3. */
static void lattice_tables(int D, int c[QMAX][3], double w[QMAX], int *Qout)
{
    int Q = (D == 2) ? 9 : 27;
    for (int i = 0; i < Q; i++) {
        int r = i;
        double wi = 1.0;
        for (int a = 0; a < 3; a++) {
            if (a < D) {
                c[i][a] = (r % 3) - 1;
                r /= 3;
                wi *= (c[i][a] == 0) ? (2.0 / 3.0) : (1.0 / 6.0);
            } else {
                c[i][a] = 0;
            }
        }
        w[i] = wi;
    }
    *Qout = Q;
}

static long cell_index(const evo_t *h, int x, int y, int z)
{
    return (long)x + (long)h->nx * ((long)y + (long)h->ny * (long)z);
}

static long neighbour(const evo_t *h, long cell, int dx, int dy, int dz)
{
    int x = (int)(cell % h->nx);
    int y = (int)((cell / h->nx) % h->ny);
    int z = (int)(cell / ((long)h->nx * h->ny));
    x = ((x + dx) % h->nx + h->nx) % h->nx;
    y = ((y + dy) % h->ny + h->ny) % h->ny;
    z = ((z + dz) % h->nz + h->nz) % h->nz;
    return cell_index(h, x, y, z);
}

/* ----------------------------------------------------- Enskog pressure */

/* Compressibility factor Z = P_E/(rho R T) of Enskog's pressure
 * P_E = rho R T (1 + b rho chi), and its logarithmic density derivative
 * d ln Z/d ln rho (both independent of T).
 *   van der Waals: chi = 1/(1 - b rho), so Z = 1/(1 - b rho) and
 *     d ln Z/d ln rho = b rho/(1 - b rho);
 *   Carnahan-Starling: chi = (1 - eta/2)/(1 - eta)^3, eta = b rho/4, so
 *     Z = 1 + 4 eta chi = (1 + eta + eta^2 - eta^3)/(1 - eta)^3 and
 *     d ln Z/d ln rho = eta (1 + 2 eta - 3 eta^2)/(1 + eta + eta^2 - eta^3)
 *                       + 3 eta/(1 - eta).
 * Returns 0 outside the physical range (b rho >= 1, resp. eta >= 1). */
static int enskog_factor(const evo_t *h, double rho, double *Z, double *dlnZ)
{
    double b = h->b;
    if (h->eos == 1) {
        double eta = 0.25 * b * rho;
        if (!(eta < 1.0)) return 0;
        double num = 1.0 + eta + eta * eta - eta * eta * eta;
        double den = (1.0 - eta) * (1.0 - eta) * (1.0 - eta);
        *Z = num / den;
        if (dlnZ) *dlnZ = eta * (1.0 + 2.0 * eta - 3.0 * eta * eta) / num + 3.0 * eta / (1.0 - eta);
        return 1;
    }
    if (!(1.0 - b * rho > 0.0)) return 0;
    *Z = 1.0 / (1.0 - b * rho);
    if (dlnZ) *dlnZ = b * rho / (1.0 - b * rho);
    return 1;
}

/* ------------------------------------------------------------- stencils */

/* Value of field phi at the cell displaced by (dx, dy, dz): periodic, or with
 * walls, beyond them in x the linear extrapolation through the two cells
 * next to the wall, phi(e) + k (phi(e) - phi(e -+ 1)) at distance k. */
static double field_at(const evo_t *h, const double *phi, long cell, int dx, int dy, int dz)
{
    int x = (int)(cell % h->nx);
    if (h->walls && (x + dx < 0 || x + dx >= h->nx)) {
        int e = (x + dx < 0) ? 0 : h->nx - 1;        /* the cell next to the wall */
        int in = (x + dx < 0) ? 1 : h->nx - 2;       /* its inner neighbour */
        int k = (x + dx < 0) ? -(x + dx) : x + dx - (h->nx - 1);
        long ce = neighbour(h, cell, e - x, dy, dz), ci = neighbour(h, cell, in - x, dy, dz);
        return phi[ce] + (double)k * (phi[ce] - phi[ci]);
    }
    return phi[neighbour(h, cell, dx, dy, dz)];
}

static double grad_at(const evo_t *h, const double *phi, int a, long cell)
{
    double s = 0.0;
    for (int i = 0; i < h->Q; i++) {
        if (h->c[i][a] == 0) continue;
        s += h->w[i] * (double)h->c[i][a] * field_at(h, phi, cell, h->c[i][0], h->c[i][1], h->c[i][2]);
    }
    return 3.0 * s;
}

static double lap_at(const evo_t *h, const double *phi, long cell)
{
    double s = 0.0;
    for (int i = 0; i < h->Q; i++)
        s += h->w[i] * (field_at(h, phi, cell, h->c[i][0], h->c[i][1], h->c[i][2]) - phi[cell]);
    return 6.0 * s;
}

/* ------------------------------------------------------- equilibria */

/* Per-axis generating function of eq. phi:
 * Psi(xi, zeta) = 1 - c^2 + (1/2)[(3c^2 - 2) zeta + c xi]. */
double evo_psi(int c, double xi, double zeta)
{
    double c2 = (double)(c * c);
    return 1.0 - c2 + 0.5 * ((3.0 * c2 - 2.0) * zeta + (double)c * xi);
}

/* f_i = rho prod_a Psi(c_ia; xi_a, zeta_a) (eq. feq, eq. f_star). */
static double product_population(const evo_t *h, int i, double rho,
                                 const double *xi, const double *zeta)
{
    double p = rho;
    for (int a = 0; a < h->D; a++) p *= evo_psi(h->c[i][a], xi[a], zeta[a]);
    return p;
}

/* Univariate polynomial in one velocity component u_a, used to apply the
 * operator O_a = (P0/rho) d/du_a + u_a of the energy equilibrium literally. */
#define PDEG 9
typedef struct { double k[PDEG]; } poly_t;

static poly_t poly_O(poly_t p, double theta)
{
    poly_t r;
    for (int n = 0; n < PDEG; n++) {
        double v = 0.0;
        if (n + 1 < PDEG) v += theta * (double)(n + 1) * p.k[n + 1];
        if (n >= 1) v += p.k[n - 1];
        r.k[n] = v;
    }
    return r;
}

/* Psi(O, O^2) applied to p: the symbols xi -> O and zeta -> O^2 of eq. phi,
 * the constant term acting as the identity. */
static poly_t poly_Psi(int c, poly_t p, double theta)
{
    poly_t Op = poly_O(p, theta);
    poly_t OOp = poly_O(Op, theta);
    double c2 = (double)(c * c);
    poly_t r;
    for (int n = 0; n < PDEG; n++)
        r.k[n] = (1.0 - c2) * p.k[n] + 0.5 * ((3.0 * c2 - 2.0) * OOp.k[n] + (double)c * Op.k[n]);
    return r;
}

static double poly_eval(poly_t p, double u)
{
    double s = 0.0;
    for (int n = PDEG - 1; n >= 0; n--) s = s * u + p.k[n];
    return s;
}

/* Energy equilibrium g_i^eq(u, RT) = rho prod_a Psi_ia(O_a, O_a^2) E(u, RT),
 * eq. geq, with E = (3/2) RT + (1/2)|u|^2 and theta = P0/rho.
 * O_a acts on u_a only, so the product operator acts factor by factor on
 * each term of E: the constant (3/2)RT and the terms u_b^2/2, which depend
 * on a single component each. */
static double energy_population(const evo_t *h, int i, double rho,
                                const double *u, double RT, double theta)
{
    poly_t one = {{0}};
    one.k[0] = 1.0;
    poly_t half_sq = {{0}};
    half_sq.k[2] = 0.5;
    double on_one[3], on_sq[3];
    for (int a = 0; a < h->D; a++) {
        on_one[a] = poly_eval(poly_Psi(h->c[i][a], one, theta), u[a]);
        on_sq[a] = poly_eval(poly_Psi(h->c[i][a], half_sq, theta), u[a]);
    }
    double prod_all = 1.0;
    for (int a = 0; a < h->D; a++) prod_all *= on_one[a];
    double s = 1.5 * RT * prod_all;
    for (int b = 0; b < h->D; b++) {
        double t = on_sq[b];
        for (int a = 0; a < h->D; a++)
            if (a != b) t *= on_one[a];
        s += t;
    }
    return rho * s;
}

/* --------------------------------------------------------- lifecycle */

static double *alloc_field(long n)
{
    double *p = (double *)calloc((size_t)n, sizeof(double));
    return p;
}

evo_t *evo_create(int D, int nx, int ny, int nz)
{
    if (!(D == 2 || D == 3) || nx <= 0 || ny <= 0 || nz <= 0) return NULL;
    if (D == 2 && nz != 1) return NULL;
    evo_t *h = (evo_t *)calloc(1, sizeof(evo_t));
    h->D = D;
    h->nx = nx;
    h->ny = ny;
    h->nz = nz;
    h->N = (long)nx * ny * nz;
    lattice_tables(D, h->c, h->w, &h->Q);
    h->R = 1.0;
    h->tau = 1.0;
    h->lambda = 1.0;
    h->sphi = -1.0;
    h->prandtl = 1.0;
    long N = h->N, Q = h->Q;
    h->f = alloc_field(Q * N);
    h->g = alloc_field(Q * N);
    h->fh = alloc_field(Q * N);
    h->gh = alloc_field(Q * N);
    h->rho = alloc_field(N);
    h->j = alloc_field(3 * N);
    h->e = alloc_field(N);
    h->rho2 = alloc_field(N);
    h->lap = alloc_field(N);
    h->F = alloc_field(3 * N);
    h->u = alloc_field(3 * N);
    h->rhoE = alloc_field(N);
    h->RT = alloc_field(N);
    h->Th = alloc_field(N);
    h->P0 = alloc_field(N);
    h->divu = alloc_field(N);
    h->M = alloc_field(3 * N);
    h->Phi = alloc_field(3 * N);
    h->tdiff = alloc_field(N);
    h->qp = alloc_field(3 * N);
    h->Phip = alloc_field(N);
    h->us = alloc_field(3 * N);
    h->RTs = alloc_field(N);
    h->Ths = alloc_field(N);
    return h;
}

void evo_destroy(evo_t *h)
{
    if (!h) return;
    double *fields[] = {h->f, h->g, h->fh, h->gh, h->rho, h->j, h->e, h->rho2,
                        h->lap, h->F, h->u, h->rhoE, h->RT, h->Th, h->P0,
                        h->divu, h->M, h->Phi, h->tdiff, h->qp, h->Phip,
                        h->us, h->RTs, h->Ths};
    for (size_t k = 0; k < sizeof(fields) / sizeof(fields[0]); k++) free(fields[k]);
    free(h);
}

int evo_Q(const evo_t *h) { return h->Q; }
long evo_N(const evo_t *h) { return h->N; }
long evo_step_count(const evo_t *h) { return h->step; }

void evo_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int evo_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* EOS P_E = rho R T/(1 - b rho), P_V = -a rho^2, capillarity kappa
 * (eq. EVforce1 and the text after it); relaxation tau, lambda (eq. beta). */
int evo_set_params(evo_t *h, double R, double a, double b, double kappa,
                   double tau, double lambda, double sphi)
{
    if (R <= 0 || a < 0 || b < 0 || kappa < 0 || tau <= 0 || lambda <= 0 || tau > lambda)
        return -1;
    h->R = R;
    h->a = a;
    h->b = b;
    h->kappa = kappa;
    h->tau = tau;
    h->lambda = lambda;
    h->sphi = sphi;
    return 0;
}

/* Prandtl number Pr = tau/tau_g of the energy populations (see the header). */
int evo_set_prandtl(evo_t *h, double Pr)
{
    if (!(Pr > 0)) return -1;
    h->prandtl = Pr;
    return 0;
}

/* Contact factor of Enskog's pressure: 0 van der Waals, 1 Carnahan-Starling. */
int evo_set_eos(evo_t *h, int kind)
{
    if (kind != 0 && kind != 1) return -1;
    h->eos = kind;
    return 0;
}

/* Diffuse walls normal to x (see the header): enable, wall temperature T_w,
 * speed U_w of the wall at x = nx - 1/2 along y (the other is at rest). */
int evo_set_walls(evo_t *h, int enable, double Tw, double Uw)
{
    if (enable && (h->nx < 2 || !(Tw > 0))) return -1;
    h->walls = enable ? 1 : 0;
    h->Tw = Tw;
    h->Uw = Uw;
    return 0;
}

/* Initial state: f = f^eq(rho0, u0, P0/rho), g = g^eq(rho0, u0, RT0), stored
 * as the post-collision state S_0. */
int evo_init(evo_t *h, const double *rho0, const double *u0, const double *T0)
{
    for (long x = 0; x < h->N; x++) {
        double r = rho0[x], RT = h->R * T0[x], Z;
        if (!(r > 0) || !(RT > 0) || !enskog_factor(h, r, &Z, NULL)) return -1;
    }
#pragma omp parallel for schedule(static)
    for (long x = 0; x < h->N; x++) {
        double r = rho0[x], RT = h->R * T0[x], Z;
        double uu[3] = {0, 0, 0};
        if (u0)
            for (int a = 0; a < h->D; a++) uu[a] = u0[a * h->N + x];
        enskog_factor(h, r, &Z, NULL);
        double theta = RT * Z;
        double zeta[3];
        for (int a = 0; a < h->D; a++) zeta[a] = theta + uu[a] * uu[a];
        for (int i = 0; i < h->Q; i++) {
            h->f[i * h->N + x] = product_population(h, i, r, uu, zeta);
            h->g[i * h->N + x] = energy_population(h, i, r, uu, RT, theta);
        }
    }
    h->step = 0;
    return 0;
}

void evo_get_pops(const evo_t *h, double *f, double *g)
{
    memcpy(f, h->f, sizeof(double) * h->Q * h->N);
    memcpy(g, h->g, sizeof(double) * h->Q * h->N);
}

void evo_set_pops(evo_t *h, const double *f, const double *g)
{
    memcpy(h->f, f, sizeof(double) * h->Q * h->N);
    memcpy(h->g, g, sizeof(double) * h->Q * h->N);
}

/* ---------------------------------------------------------- the step */

/* Diffuse re-emission at a wall for cell x next to it: side = -1 (wall at
 * x = -1/2, at rest) or +1 (wall at x = nx - 1/2, moving with U_w along y).
 * The populations entering the cell from the wall (c_x = -side) become
 * rho_w f^eq_i(1, u_w, theta_w) and rho_w g^eq_i(1, u_w, R T_w, theta_w), with
 * theta_w = R T_w Z(rho) at the cell's stored density and rho_w such that they
 * carry the mass of the cell's populations heading into the wall (c_x = side). */
static void wall_emission(evo_t *h, long x, int side)
{
    long N = h->N;
    double rho = 0.0, out = 0.0, in = 0.0, Z = 1.0;
    for (int i = 0; i < h->Q; i++) {
        rho += h->f[i * N + x];
        if (h->c[i][0] == side) out += h->f[i * N + x];
    }
    enskog_factor(h, rho, &Z, NULL);
    double RTw = h->R * h->Tw, theta = RTw * Z;
    double uw[3] = {0.0, side > 0 ? h->Uw : 0.0, 0.0}, zeta[3];
    for (int a = 0; a < h->D; a++) zeta[a] = theta + uw[a] * uw[a];
    for (int i = 0; i < h->Q; i++)
        if (h->c[i][0] == -side) in += product_population(h, i, 1.0, uw, zeta);
    double rho_w = out / in;
    for (int i = 0; i < h->Q; i++)
        if (h->c[i][0] == -side) {
            h->fh[i * N + x] = rho_w * product_population(h, i, 1.0, uw, zeta);
            h->gh[i * N + x] = rho_w * energy_population(h, i, 1.0, uw, RTw, theta);
        }
}

/* Exact on-lattice propagation (pull form): fh_i(x) = f_i(x - c_i); with
 * walls, the populations whose source lies beyond a wall come from it. */
static void stage_stream(evo_t *h)
{
    long N = h->N;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        int xc = (int)(x % h->nx);
        for (int i = 0; i < h->Q; i++) {
            if (h->walls && (xc - h->c[i][0] < 0 || xc - h->c[i][0] >= h->nx)) continue;
            long src = neighbour(h, x, -h->c[i][0], -h->c[i][1], -h->c[i][2]);
            h->fh[i * N + x] = h->f[i * N + src];
            h->gh[i * N + x] = h->g[i * N + src];
        }
        if (h->walls && xc == 0) wall_emission(h, x, -1);
        if (h->walls && xc == h->nx - 1) wall_emission(h, x, +1);
    }
}

/* Raw moments: rho = sum fh, j = sum c fh, e = sum gh. */
static void stage_moments(evo_t *h)
{
    long N = h->N;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double r = 0, e = 0, jj[3] = {0, 0, 0};
        for (int i = 0; i < h->Q; i++) {
            r += h->fh[i * N + x];
            e += h->gh[i * N + x];
            for (int a = 0; a < h->D; a++) jj[a] += (double)h->c[i][a] * h->fh[i * N + x];
        }
        h->rho[x] = r;
        h->e[x] = e;
        for (int a = 0; a < 3; a++) h->j[a * N + x] = (a < h->D) ? jj[a] : 0.0;
    }
}

/* Non-local force in the Enskog gauge P0 = P_E (eq. P0E): the -grad(P_E - P0)
 * term vanishes and F = -grad P_V + kappa rho grad(lap rho) with
 * P_V = -a rho^2 (eq. EVforce1).  The compression work Qtilde vanishes. */
static void stage_force(evo_t *h)
{
    long N = h->N;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) h->rho2[x] = h->rho[x] * h->rho[x];
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) h->lap[x] = lap_at(h, h->rho, x);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++)
        for (int a = 0; a < 3; a++) {
            double Fa = 0.0;
            if (a < h->D)
                Fa = h->a * grad_at(h, h->rho2, a, x) + h->kappa * h->rho[x] * grad_at(h, h->lap, a, x);
            h->F[a * N + x] = Fa;
        }
}

/* Half-step shifted fields (eq. u_shift, eq. T_shift), Qtilde = 0:
 * rho u = j + F/2, rho E = e + u.F/2, (3/2) rho RT = rho E - rho |u|^2/2,
 * P0 = P_E = rho RT Z(rho) (Z = 1/(1 - b rho) for van der Waals). */
static void stage_fields(evo_t *h)
{
    long N = h->N;
    const double Qtilde = 0.0;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double r = h->rho[x];
        double uF = 0.0, u2 = 0.0;
        for (int a = 0; a < 3; a++) {
            double ua = (h->j[a * N + x] + 0.5 * h->F[a * N + x]) / r;
            h->u[a * N + x] = ua;
            uF += ua * h->F[a * N + x];
            u2 += ua * ua;
        }
        double rhoE = h->e[x] + 0.5 * (uF + Qtilde);
        h->rhoE[x] = rhoE;
        double RT = (2.0 / 3.0) * (rhoE / r - 0.5 * u2);
        h->RT[x] = RT;
        double Z = NAN;
        enskog_factor(h, r, &Z, NULL); /* NAN outside the physical range: caught by fields_physical */
        double PE = r * RT * Z;
        h->P0[x] = PE;
        h->Th[x] = PE / r;
    }
}

/* Corrections: Phi_aa (eq. correction_u), Phi' (eq. correction_gamma) with
 * gamma_0 of eq. gamma, and q'_a (eq. correction_q). */
static void stage_corrections(evo_t *h)
{
    long N = h->N;
    const double varsigma2 = 1.0 / 3.0;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double r = h->rho[x];
        for (int a = 0; a < 3; a++) {
            double ua = h->u[a * N + x];
            h->M[a * N + x] = r * ua * (ua * ua + 3.0 * h->P0[x] / r - 3.0 * varsigma2);
        }
        h->tdiff[x] = h->P0[x] / r - h->RT[x];
    }
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double d = 0.0;
        for (int a = 0; a < h->D; a++) d += grad_at(h, h->u + a * N, a, x);
        h->divu[x] = d;
    }
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double r = h->rho[x];
        double Z, dlnZ;
        enskog_factor(h, r, &Z, &dlnZ);
        /* P0 = P_E = rho R T Z(rho):
         * (d ln P0/d ln rho)_T = 1 + d ln Z/d ln rho, (d ln P0/d ln T)_rho = 1,
         * P_E/(rho R T) = Z (van der Waals: 1/(1 - b rho), 1, 1/(1 - b rho)). */
        double dlnP_dlnrho = 1.0 + dlnZ;
        double dlnP_dlnT = 1.0;
        double PE_over_rhoRT = Z;
        double gamma0 = dlnP_dlnrho + (2.0 / 3.0) * PE_over_rhoRT * dlnP_dlnT;
        double Phip = h->P0[x] * (5.0 / 3.0 - gamma0) * h->divu[x];
        h->Phip[x] = Phip;
        for (int a = 0; a < 3; a++) {
            double Pa = 0.0, qa = 0.0;
            if (a < h->D) {
                Pa = h->sphi * grad_at(h, h->M + a * N, a, x) + Phip;
                qa = h->lambda * h->P0[x] * grad_at(h, h->tdiff, a, x) + h->lambda * h->u[a * N + x] * Phip;
            }
            h->Phi[a * N + x] = Pa;
            h->qp[a * N + x] = qa;
        }
    }
}

/* Shifted velocity and temperature (eq. def_ustar), Qtilde = 0. */
static void stage_shift(evo_t *h)
{
    long N = h->N;
    const double Qtilde = 0.0;
    double lam = h->lambda;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double r = h->rho[x], F2 = 0.0;
        for (int a = 0; a < 3; a++) {
            h->us[a * N + x] = h->u[a * N + x] + lam * h->F[a * N + x] / r;
            F2 += h->F[a * N + x] * h->F[a * N + x];
        }
        double RTs = h->RT[x] + 2.0 * lam * Qtilde / (3.0 * r) - lam * lam * F2 / (3.0 * r * r);
        double Z;
        enskog_factor(h, r, &Z, NULL);
        h->RTs[x] = RTs;
        h->Ths[x] = RTs * Z;
    }
}

/* Equilibria and the update of eq. pre_LBM:
 * f <- fh + 2 beta (f^eq - fh) + (dt/lambda)(1 - beta)(f* - f^eq), the same
 * for g, beta = dt/(2 tau + dt).  diag (optional) receives per-cell sums for
 * the conservation checks. */
static void stage_collide(evo_t *h, double *diag)
{
    long N = h->N;
    int D = h->D;
    double beta = 1.0 / (2.0 * h->tau + 1.0);
    double wstar = (1.0 / h->lambda) * (1.0 - beta);
    double beta_g = 1.0 / (2.0 * (h->tau / h->prandtl) + 1.0);
    double wstar_g = (1.0 / h->lambda) * (1.0 - beta_g);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < N; x++) {
        double r = h->rho[x];
        double u[3], us[3], zeq[3], zst[3];
        for (int a = 0; a < 3; a++) {
            u[a] = h->u[a * N + x];
            us[a] = h->us[a * N + x];
        }
        for (int a = 0; a < D; a++) {
            zeq[a] = h->Th[x] + u[a] * u[a];
            zst[a] = h->Th[x] + us[a] * us[a] + h->lambda * h->Phi[a * N + x] / r;
        }
        double sf = 0, sg = 0, scf[3] = {0, 0, 0};
        /* u . Pi^neq with Pi^neq = sum_i c_i c_i (fh_i - f^eq_i) (quasi-equilibrium flux) */
        double upi[3] = {0, 0, 0};
        for (int i = 0; i < h->Q; i++) {
            double d = h->fh[i * N + x] - product_population(h, i, r, u, zeq);
            double cu = 0.0;
            for (int a = 0; a < D; a++) cu += (double)h->c[i][a] * u[a];
            for (int a = 0; a < D; a++) upi[a] += (double)h->c[i][a] * cu * d;
        }
        for (int i = 0; i < h->Q; i++) {
            double feq = product_population(h, i, r, u, zeq);
            double fst = product_population(h, i, r, us, zst);
            double geq = energy_population(h, i, r, u, h->RT[x], h->Th[x]);
            double gst = energy_population(h, i, r, us, h->RTs[x], h->Ths[x]);
            int c2 = 0;
            for (int a = 0; a < D; a++) c2 += h->c[i][a] * h->c[i][a];
            if (c2 == 1) {
                double cq = 0.0;
                for (int a = 0; a < D; a++) cq += (double)h->c[i][a] * h->qp[a * N + x];
                gst += 0.5 * cq;
            }
            double fh = h->fh[i * N + x], gh = h->gh[i * N + x];
            double dg = 0.0;
            if (c2 == 1)
                for (int a = 0; a < D; a++) dg += 0.5 * (double)h->c[i][a] * upi[a];
            double fn = fh + 2.0 * beta * (feq - fh) + wstar * (fst - feq);
            double gn = gh + 2.0 * beta_g * (geq - gh) + wstar_g * (gst - geq) + 2.0 * (beta_g - beta) * dg;
            h->f[i * N + x] = fn;
            h->g[i * N + x] = gn;
            if (diag) {
                sf += fn;
                sg += gn;
                for (int a = 0; a < D; a++) scf[a] += (double)h->c[i][a] * fn;
            }
        }
        if (diag) {
            double uF = 0.0;
            for (int a = 0; a < D; a++) uF += u[a] * h->F[a * N + x];
            int k = 0;
            diag[(k++) * N + x] = r;
            diag[(k++) * N + x] = sf;
            for (int a = 0; a < D; a++) diag[(k++) * N + x] = h->j[a * N + x];
            for (int a = 0; a < D; a++) diag[(k++) * N + x] = scf[a];
            for (int a = 0; a < D; a++) diag[(k++) * N + x] = h->F[a * N + x];
            diag[(k++) * N + x] = h->e[x];
            diag[(k++) * N + x] = sg;
            diag[(k++) * N + x] = uF;
        }
    }
}

static int fields_physical(const evo_t *h)
{
    for (long x = 0; x < h->N; x++) {
        double Z;
        if (!(h->rho[x] > 0) || !enskog_factor(h, h->rho[x], &Z, NULL) || !(h->RT[x] > 0)) return 0;
    }
    return 1;
}

static void analyse(evo_t *h)
{
    stage_stream(h);
    stage_moments(h);
    stage_force(h);
    stage_fields(h);
}

/* Advance nsteps.  Returns 0, or -2 when a non-physical state (rho <= 0,
 * b rho >= 1, RT <= 0 or a non-finite value) is met. */
int evo_step(evo_t *h, long nsteps, double *diag)
{
    for (long s = 0; s < nsteps; s++) {
        analyse(h);
        if (!fields_physical(h)) return -2;
        stage_corrections(h);
        stage_shift(h);
        stage_collide(h, (s == nsteps - 1) ? diag : NULL);
        h->step++;
    }
    return 0;
}

/* Readout of S_n: pull, raw moments, force and half-step fields.
 * rho[N], u[D*N] (layout [alpha][cell]), T[N] = RT/R.  Any pointer may be
 * NULL.  F (D*N) optional. */
void evo_moments(evo_t *h, double *rho, double *u, double *T, double *F)
{
    analyse(h);
    long N = h->N;
    for (long x = 0; x < N; x++) {
        if (rho) rho[x] = h->rho[x];
        if (T) T[x] = h->RT[x] / h->R;
        for (int a = 0; a < h->D; a++) {
            if (u) u[a * N + x] = h->u[a * N + x];
            if (F) F[a * N + x] = h->F[a * N + x];
        }
    }
}

/* Correction fields of the current state (for tests): Phi[D*N], qp[D*N],
 * Phip[N]. */
void evo_corrections(evo_t *h, double *Phi, double *qp, double *Phip)
{
    analyse(h);
    stage_corrections(h);
    long N = h->N;
    for (long x = 0; x < N; x++) {
        if (Phip) Phip[x] = h->Phip[x];
        for (int a = 0; a < h->D; a++) {
            if (Phi) Phi[a * N + x] = h->Phi[a * N + x];
            if (qp) qp[a * N + x] = h->qp[a * N + x];
        }
    }
}

/* Global FP64 sums of the readout at S_n:
 * out[0] = sum rho, out[1..3] = sum rho u, out[4] = sum rho E,
 * out[5] = sum [rho E - a rho^2 + (kappa/2)|grad rho|^2],
 * out[6] = max |u|, out[7] = min fh. */
void evo_global_sums(evo_t *h, double *out)
{
    analyse(h);
    long N = h->N;
    double m = 0, p[3] = {0, 0, 0}, E = 0, Et = 0, umax = 0, fmin = 1e300;
    for (long x = 0; x < N; x++) {
        double r = h->rho[x], u2 = 0, g2 = 0;
        m += r;
        for (int a = 0; a < h->D; a++) {
            double ua = h->u[a * N + x];
            p[a] += r * ua;
            u2 += ua * ua;
            double gr = grad_at(h, h->rho, a, x);
            g2 += gr * gr;
        }
        E += h->rhoE[x];
        Et += h->rhoE[x] - h->a * r * r + 0.5 * h->kappa * g2;
        if (sqrt(u2) > umax) umax = sqrt(u2);
        for (int i = 0; i < h->Q; i++)
            if (h->fh[i * N + x] < fmin) fmin = h->fh[i * N + x];
    }
    out[0] = m;
    out[1] = p[0];
    out[2] = p[1];
    out[3] = p[2];
    out[4] = E;
    out[5] = Et;
    out[6] = umax;
    out[7] = fmin;
}

/* --------------------------------------------- single-cell helpers */

static evo_t *cell_lattice(int D)
{
    static evo_t L2, L3;
    evo_t *L = (D == 2) ? &L2 : &L3;
    if (L->Q == 0) {
        L->D = D;
        lattice_tables(D, L->c, L->w, &L->Q);
    }
    return L;
}

/* Lattice tables: c[Q*3], w[Q]. */
int evo_lattice(int D, int *c, double *w)
{
    evo_t *L = cell_lattice(D);
    for (int i = 0; i < L->Q; i++) {
        for (int a = 0; a < 3; a++) c[3 * i + a] = L->c[i][a];
        w[i] = L->w[i];
    }
    return L->Q;
}

/* f_i = rho prod_a Psi(c_ia; xi_a, zeta_a) for given xi, zeta. */
void evo_product_cell(int D, double rho, const double *xi, const double *zeta, double *out)
{
    evo_t *L = cell_lattice(D);
    for (int i = 0; i < L->Q; i++) out[i] = product_population(L, i, rho, xi, zeta);
}

/* g_i^eq(u, RT) with P0/rho = theta (eq. geq). */
void evo_geq_cell(int D, double rho, const double *u, double RT, double theta, double *out)
{
    evo_t *L = cell_lattice(D);
    for (int i = 0; i < L->Q; i++) out[i] = energy_population(L, i, rho, u, RT, theta);
}

/* The nonlinear operator of eq. K for one cell, with the lattice Maxwellian
 * f^eq(u, RT) = rho prod Psi(u_a, RT + u_a^2) of the kinetic theory (P0 =
 * rho R T there):  F = sum c J, Qt = sum (c - u)^2/2 J (eq. defF, defQ),
 * u* = u + lambda F/rho, RT* = RT + 2 lambda Qt/(3 rho) - lambda^2 F.F/(3 rho^2),
 * K = [f^eq(u*, RT*) - f^eq(u, RT)]/lambda.
 * Returns -1 when RT* <= 0. */
int evo_kop(int D, double rho, const double *u, double RT, const double *J,
            double lambda, double *out)
{
    evo_t *L = cell_lattice(D);
    double F[3] = {0, 0, 0}, Qt = 0.0;
    for (int i = 0; i < L->Q; i++) {
        double cu2 = 0.0;
        for (int a = 0; a < D; a++) {
            F[a] += (double)L->c[i][a] * J[i];
            double d = (double)L->c[i][a] - u[a];
            cu2 += d * d;
        }
        Qt += 0.5 * cu2 * J[i];
    }
    double us[3], F2 = 0.0;
    for (int a = 0; a < D; a++) {
        us[a] = u[a] + lambda * F[a] / rho;
        F2 += F[a] * F[a];
    }
    double RTs = RT + 2.0 * lambda * Qt / (3.0 * rho) - lambda * lambda * F2 / (3.0 * rho * rho);
    if (!(RTs > 0)) return -1;
    double z0[3], zs[3];
    for (int a = 0; a < D; a++) {
        z0[a] = RT + u[a] * u[a];
        zs[a] = RTs + us[a] * us[a];
    }
    for (int i = 0; i < L->Q; i++)
        out[i] = (product_population(L, i, rho, us, zs) - product_population(L, i, rho, u, z0)) / lambda;
    return 0;
}

/* Isotropic stencils on a periodic scalar field (for their own tests):
 * grad[D*N] (layout [alpha][cell]) and lap[N]. */
void evo_stencils(int D, int nx, int ny, int nz, const double *phi, double *grad, double *lap)
{
    evo_t h;
    memset(&h, 0, sizeof(h));
    h.D = D;
    h.nx = nx;
    h.ny = ny;
    h.nz = nz;
    h.N = (long)nx * ny * nz;
    lattice_tables(D, h.c, h.w, &h.Q);
    for (long x = 0; x < h.N; x++) {
        if (lap) lap[x] = lap_at(&h, phi, x);
        if (grad)
            for (int a = 0; a < D; a++) grad[a * h.N + x] = grad_at(&h, phi, a, x);
    }
}
