/*
 * FP64 reference solver for the D3Q19 BGK lattice Boltzmann update.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares
 * no code, header, table or constant with the HIP library: its velocity set,
 * weights, indexing and arithmetic are written out here on their own.
 *
 * What it computes (paper, Section 2 "Lattice Boltzmann Method", Eq. 1-3, and
 * Section 3.1 "Computational Description"):
 *
 *   Eq. 1  f_i(x + c_i, t + 1) = f_i(x, t) - omega (f_i(x, t) - f_i^eq(x, t)) + S_i
 *   Eq. 2  f_i^eq = w_i rho (1 + u_i + q_i)
 *   Eq. 3  u_i = 3 (u . c_i),  q_i = (9/2)(u . c_i)^2 - (3/2) u . u
 *
 * Eq. 3 is printed with the sound speed c_s mixed into it; the reading used
 * here is the standard second-order expansion with c_s^2 = 1/3 substituted,
 * which gives the coefficients 3, 9/2 and 3/2.  The moment identities of
 * f^eq pin that reading in the tests.
 *
 * Section 3.1 describes the fused scheme: two population arrays, a scattered
 * read from the pre-collision array, collision, a write into the other array,
 * and a swap.  The state kept between steps is the post-collision array S:
 *
 *   one step, for every fluid site x:
 *     1. gather  f_i = S_i(x - c_i)        (pull streaming, periodic wrap)
 *                f_i = S_opp(i)(x)          if the site x - c_i is solid
 *                                           (halfway bounce-back, no-slip wall)
 *     2. moments rho = sum_i f_i,  u = (sum_i c_i f_i + F/2) / rho
 *     3. f_i^eq  from Eq. 2-3
 *     4. source  S_i^F = (1 - omega/2) w_i [3 (c_i - u) + 9 (c_i . u) c_i] . F
 *                (the paper names a source term S_i without a formula; the
 *                 reading taken is Guo's forcing scheme with the half-force
 *                 velocity shift of step 2)
 *     5. relax   S'_i(x) = f_i - omega (f_i - f_i^eq) + S_i^F     (Eq. 1)
 *   then S <- S'.  Solid sites are never written and never read as state.
 *
 * The velocity set is D3Q19 (the paper's mini-app is D2Q9; its parent
 * application and its stated future work are three-dimensional).  Ordering:
 * rest, the six axis directions as (+,-) pairs, then the twelve face
 * diagonals grouped by plane (xy, xz, yz); see LATTICE_C.
 *
 * Populations are stored unshifted, in FP64, structure-of-arrays: population
 * i of site s = x + nx (y + ny z) lives at S[i * N + s] with N = nx ny nz
 * (Section 3.1: one unit-stride vector per population).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

/* D3Q19 velocities. */
static const int LATTICE_C[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
    {1, 1, 0},   {1, -1, 0},  {-1, 1, 0},  {-1, -1, 0},
    {1, 0, 1},   {1, 0, -1},  {-1, 0, 1},  {-1, 0, -1},
    {0, 1, 1},   {0, 1, -1},  {0, -1, 1},  {0, -1, -1},
};

/* Weight of direction i from its speed: |c|^2 = 0 -> 1/3, 1 -> 1/18, 2 -> 1/36. */
static double lattice_w(int i)
{
    int c2 = LATTICE_C[i][0] * LATTICE_C[i][0] + LATTICE_C[i][1] * LATTICE_C[i][1] +
             LATTICE_C[i][2] * LATTICE_C[i][2];
    if (c2 == 0) return 1.0 / 3.0;
    if (c2 == 1) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* Opposite direction: found by search, so it cannot disagree with LATTICE_C. */
static int lattice_opp(int i)
{
    for (int j = 0; j < Q; ++j)
        if (LATTICE_C[j][0] == -LATTICE_C[i][0] && LATTICE_C[j][1] == -LATTICE_C[i][1] &&
            LATTICE_C[j][2] == -LATTICE_C[i][2])
            return j;
    return -1;
}

static int wrap(int a, int n)
{
    a %= n;
    return a < 0 ? a + n : a;
}

int oracle_q(void) { return Q; }

/* Export the velocity set, weights and opposites (c: 3*Q ints, w: Q, opp: Q). */
void oracle_lattice(int *c, double *w, int *opp)
{
    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = LATTICE_C[i][a];
        w[i] = lattice_w(i);
        opp[i] = lattice_opp(i);
    }
}

/* Eq. 2-3: f_i^eq = w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u). */
void oracle_feq(double rho, const double *u, double *feq)
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double cu = LATTICE_C[i][0] * u[0] + LATTICE_C[i][1] * u[1] + LATTICE_C[i][2] * u[2];
        feq[i] = lattice_w(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* Guo source term (reading of Eq. 1's S_i): (1 - omega/2) w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F */
void oracle_source(double omega, const double *u, const double *F, double *src)
{
    for (int i = 0; i < Q; ++i) {
        double cu = LATTICE_C[i][0] * u[0] + LATTICE_C[i][1] * u[1] + LATTICE_C[i][2] * u[2];
        double acc = 0.0;
        for (int a = 0; a < 3; ++a)
            acc += (3.0 * (LATTICE_C[i][a] - u[a]) + 9.0 * cu * LATTICE_C[i][a]) * F[a];
        src[i] = (1.0 - 0.5 * omega) * lattice_w(i) * acc;
    }
}

/*
 * Initial state S_0 = f^eq(rho, u) at fluid sites, the rest state f_i = w_i at
 * solid sites.  rho: N values (NULL means 1); u: 3N values, component-major
 * (all u_x, then all u_y, then all u_z; NULL means 0).  flags: N bytes,
 * 0 fluid, 1 solid (NULL means all fluid).
 */
void oracle_init(int nx, int ny, int nz, const uint8_t *flags, const double *rho,
                 const double *u, double *S)
{
    size_t N = (size_t)nx * ny * nz;
    for (size_t s = 0; s < N; ++s) {
        double feq[Q];
        if (flags && flags[s]) {
            for (int i = 0; i < Q; ++i) feq[i] = lattice_w(i);
        } else {
            double r = rho ? rho[s] : 1.0;
            double v[3] = {u ? u[s] : 0.0, u ? u[N + s] : 0.0, u ? u[2 * N + s] : 0.0};
            oracle_feq(r, v, feq);
        }
        for (int i = 0; i < Q; ++i) S[(size_t)i * N + s] = feq[i];
    }
}

/*
 * One fused step S_in -> S_out (steps 1-5 above).  omega = 1/tau.
 * F: uniform force density (3 values) or NULL; Fx_field: optional per-site
 * x-force added to F[0] (N values) or NULL.  rho_pre / u_pre, when not NULL,
 * receive the pre-collision moments of step 2 (u with the half-force shift).
 * Solid sites of S_out are copied from S_in; their moments are set to 0.
 */
void oracle_step(int nx, int ny, int nz, const uint8_t *flags, double omega, const double *F,
                 const double *Fx_field, const double *S_in, double *S_out, double *rho_pre,
                 double *u_pre)
{
    size_t N = (size_t)nx * ny * nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t s = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
                if (flags && flags[s]) {
                    for (int i = 0; i < Q; ++i) S_out[(size_t)i * N + s] = S_in[(size_t)i * N + s];
                    if (rho_pre) rho_pre[s] = 0.0;
                    if (u_pre) u_pre[s] = u_pre[N + s] = u_pre[2 * N + s] = 0.0;
                    continue;
                }
                /* 1. gather */
                double f[Q];
                for (int i = 0; i < Q; ++i) {
                    int xs = wrap(x - LATTICE_C[i][0], nx);
                    int ys = wrap(y - LATTICE_C[i][1], ny);
                    int zs = wrap(z - LATTICE_C[i][2], nz);
                    size_t src = (size_t)xs + (size_t)nx * ((size_t)ys + (size_t)ny * zs);
                    if (flags && flags[src])
                        f[i] = S_in[(size_t)lattice_opp(i) * N + s];
                    else
                        f[i] = S_in[(size_t)i * N + src];
                }
                /* 2. moments */
                double force[3] = {F ? F[0] : 0.0, F ? F[1] : 0.0, F ? F[2] : 0.0};
                if (Fx_field) force[0] += Fx_field[s];
                double rho = 0.0, mom[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i < Q; ++i) {
                    rho += f[i];
                    for (int a = 0; a < 3; ++a) mom[a] += LATTICE_C[i][a] * f[i];
                }
                double u[3];
                for (int a = 0; a < 3; ++a) u[a] = (mom[a] + 0.5 * force[a]) / rho;
                if (rho_pre) rho_pre[s] = rho;
                if (u_pre)
                    for (int a = 0; a < 3; ++a) u_pre[(size_t)a * N + s] = u[a];
                /* 3-5. equilibrium, source, relaxation */
                double feq[Q], src[Q];
                oracle_feq(rho, u, feq);
                oracle_source(omega, u, force, src);
                for (int i = 0; i < Q; ++i)
                    S_out[(size_t)i * N + s] = f[i] - omega * (f[i] - feq[i]) + src[i];
            }
}

/* n steps in place on S (the result ends in S).  Returns 0, or -1 on allocation failure. */
int oracle_run(int nx, int ny, int nz, const uint8_t *flags, double omega, const double *F,
               const double *Fx_field, double *S, int nsteps)
{
    if (nsteps <= 0) return 0;
    size_t bytes = (size_t)Q * nx * ny * nz * sizeof(double);
    double *T = (double *)malloc(bytes);
    if (!T) return -1;
    double *a = S, *b = T;
    for (int t = 0; t < nsteps; ++t) {
        oracle_step(nx, ny, nz, flags, omega, F, Fx_field, a, b, NULL, NULL);
        double *tmp = a;
        a = b;
        b = tmp;
    }
    if (a != S) memcpy(S, a, bytes);
    free(T);
    return 0;
}

/*
 * Macroscopic fields of a stored post-collision state S_n:
 *   rho = sum_i S_i,  u = (sum_i c_i S_i - F/2) / rho.
 * Collision conserves mass and the Guo source adds exactly F to the momentum,
 * so these equal the pre-collision moments of step n (for n >= 1).  Solid
 * sites give rho = 0, u = 0.
 */
void oracle_macros(int nx, int ny, int nz, const uint8_t *flags, const double *F,
                   const double *Fx_field, const double *S, double *rho, double *u)
{
    size_t N = (size_t)nx * ny * nz;
    for (size_t s = 0; s < N; ++s) {
        if (flags && flags[s]) {
            rho[s] = 0.0;
            u[s] = u[N + s] = u[2 * N + s] = 0.0;
            continue;
        }
        double force[3] = {F ? F[0] : 0.0, F ? F[1] : 0.0, F ? F[2] : 0.0};
        if (Fx_field) force[0] += Fx_field[s];
        double r = 0.0, m[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            double v = S[(size_t)i * N + s];
            r += v;
            for (int a = 0; a < 3; ++a) m[a] += LATTICE_C[i][a] * v;
        }
        rho[s] = r;
        for (int a = 0; a < 3; ++a) u[(size_t)a * N + s] = (m[a] - 0.5 * force[a]) / r;
    }
}

/* Conserved totals over fluid sites: out = {sum S, sum c_x S, sum c_y S, sum c_z S}. */
void oracle_sums(int nx, int ny, int nz, const uint8_t *flags, const double *S, double *out)
{
    size_t N = (size_t)nx * ny * nz;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (size_t s = 0; s < N; ++s) {
        if (flags && flags[s]) continue;
        for (int i = 0; i < Q; ++i) {
            double v = S[(size_t)i * N + s];
            acc[0] += v;
            for (int a = 0; a < 3; ++a) acc[1 + a] += LATTICE_C[i][a] * v;
        }
    }
    for (int k = 0; k < 4; ++k) out[k] = acc[k];
}

/* ------------------------------------------------------------------------- *
 * Adjoint of the fused step (reverse-mode derivative).
 *
 * One step maps the stored state S_n to S_{n+1} = C(P S_n, F): P is the pull
 * streaming with halfway bounce-back (step 1 above), C the per-site
 * collision with the Guo source (steps 2-5).  For an objective J(S_N) the
 * adjoint state lam_n = dJ/dS_n obeys
 *     lam_n = P^T ( (dC/df)^T lam_{n+1} ),
 * and the force enters every step through C, so
 *     dJ/dF_x(x) = sum_n (dC/dF_x)(x)^T lam_{n+1}(x)   (+ any direct term of J).
 *
 * dC/df at one site, with rho = sum f, u = (sum c f + F/2) / rho:
 *   dC_i/df_j = (1 - omega) delta_ij
 *             + omega [ dfeq_i/drho + sum_a dfeq_i/du_a (c_ja - u_a) / rho ]
 *             + sum_a dS_i/du_a (c_ja - u_a) / rho
 *   dfeq_i/drho = w_i (1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u)
 *   dfeq_i/du_a = w_i rho (3 c_ia + 9 (c_i.u) c_ia - 3 u_a)
 *   dS_i/du_a   = (1 - omega/2) w_i (9 (c_i.F) c_ia - 3 F_a)
 * and, since du_x/dF_x = 1 / (2 rho),
 *   dC_i/dF_x = [omega dfeq_i/du_x + dS_i/du_x] / (2 rho)
 *             + (1 - omega/2) w_i (3 (c_ix - u_x) + 9 (c_i.u) c_ix).
 *
 * P^T: P reads S_k(y) exactly once, at site y + c_k for direction k when
 * that site is fluid, else at site y itself for direction opp(k) (bounce-back
 * at the solid y + c_k).  So, for a fluid site y,
 *     (P^T m)_k(y) = m_k(y + c_k)     if y + c_k is fluid,
 *                  = m_opp(k)(y)      otherwise.
 * ------------------------------------------------------------------------- */

/*
 * Jacobian of the collision at one site: J[i*Q + j] = dC_i/df_j for the
 * pre-collision populations f (unshifted) and force density F (3 values);
 * dFx[i] = dC_i/dF_x.
 */
void oracle_collision_jacobian(double omega, const double *f, const double *F, double *J, double *dFx)
{
    double rho = 0.0, mom[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        rho += f[i];
        for (int a = 0; a < 3; ++a) mom[a] += LATTICE_C[i][a] * f[i];
    }
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = (mom[a] + 0.5 * F[a]) / rho;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; ++i) {
        double w = lattice_w(i);
        double cu = LATTICE_C[i][0] * u[0] + LATTICE_C[i][1] * u[1] + LATTICE_C[i][2] * u[2];
        double cF = LATTICE_C[i][0] * F[0] + LATTICE_C[i][1] * F[1] + LATTICE_C[i][2] * F[2];
        double dfeq_drho = w * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        double dfeq_du[3], dS_du[3];
        for (int a = 0; a < 3; ++a) {
            dfeq_du[a] = w * rho * (3.0 * LATTICE_C[i][a] + 9.0 * cu * LATTICE_C[i][a] - 3.0 * u[a]);
            dS_du[a] = (1.0 - 0.5 * omega) * w * (9.0 * cF * LATTICE_C[i][a] - 3.0 * F[a]);
        }
        for (int j = 0; j < Q; ++j) {
            double v = (i == j ? 1.0 - omega : 0.0) + omega * dfeq_drho;
            for (int a = 0; a < 3; ++a) {
                double du = (LATTICE_C[j][a] - u[a]) / rho;
                v += (omega * dfeq_du[a] + dS_du[a]) * du;
            }
            J[i * Q + j] = v;
        }
        dFx[i] = (omega * dfeq_du[0] + dS_du[0]) / (2.0 * rho)
                 + (1.0 - 0.5 * omega) * w * (3.0 * (LATTICE_C[i][0] - u[0]) + 9.0 * cu * LATTICE_C[i][0]);
    }
}

/*
 * Adjoint of one step taken from S_n: lam_out = dJ/dS_n from lam_next =
 * dJ/dS_{n+1} (both 19N, same layout as S; solid sites of lam_out are 0),
 * and grad_fx[s] += dJ/dF_x(s) through this step (N values, fluid sites).
 * F / Fx_field as in oracle_step.  Returns 0, or -1 on allocation failure.
 */
int oracle_adjoint_step(int nx, int ny, int nz, const uint8_t *flags, double omega, const double *F,
                        const double *Fx_field, const double *S_n, const double *lam_next, double *lam_out,
                        double *grad_fx)
{
    size_t N = (size_t)nx * ny * nz;
    double *m = (double *)calloc((size_t)Q * N, sizeof(double));
    if (!m) return -1;
    /* m = (dC/df)^T lam_next at every fluid site */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t s = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
                if (flags && flags[s]) continue;
                double f[Q];
                for (int i = 0; i < Q; ++i) {
                    int xs = wrap(x - LATTICE_C[i][0], nx);
                    int ys = wrap(y - LATTICE_C[i][1], ny);
                    int zs = wrap(z - LATTICE_C[i][2], nz);
                    size_t src = (size_t)xs + (size_t)nx * ((size_t)ys + (size_t)ny * zs);
                    if (flags && flags[src])
                        f[i] = S_n[(size_t)lattice_opp(i) * N + s];
                    else
                        f[i] = S_n[(size_t)i * N + src];
                }
                double force[3] = {F ? F[0] : 0.0, F ? F[1] : 0.0, F ? F[2] : 0.0};
                if (Fx_field) force[0] += Fx_field[s];
                double J[Q * Q], dFx[Q];
                oracle_collision_jacobian(omega, f, force, J, dFx);
                double g = 0.0;
                for (int j = 0; j < Q; ++j) {
                    double acc = 0.0;
                    for (int i = 0; i < Q; ++i) acc += lam_next[(size_t)i * N + s] * J[i * Q + j];
                    m[(size_t)j * N + s] = acc;
                }
                for (int i = 0; i < Q; ++i) g += lam_next[(size_t)i * N + s] * dFx[i];
                if (grad_fx) grad_fx[s] += g;
            }
    /* lam_out = P^T m */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t s = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
                for (int k = 0; k < Q; ++k) {
                    if (flags && flags[s]) {
                        lam_out[(size_t)k * N + s] = 0.0;
                        continue;
                    }
                    int xt = wrap(x + LATTICE_C[k][0], nx);
                    int yt = wrap(y + LATTICE_C[k][1], ny);
                    int zt = wrap(z + LATTICE_C[k][2], nz);
                    size_t t = (size_t)xt + (size_t)nx * ((size_t)yt + (size_t)ny * zt);
                    if (flags && flags[t])
                        lam_out[(size_t)k * N + s] = m[(size_t)lattice_opp(k) * N + s];
                    else
                        lam_out[(size_t)k * N + s] = m[(size_t)k * N + t];
                }
            }
    free(m);
    return 0;
}
