/*
 * Driver for a sanitizer build of the oracle (test infrastructure).
 *
 * Built by tests/test_sanitizers.py with gcc -fsanitize=address,undefined
 * together with d3q19_oracle.c and d2q9_oracle.c, it calls every exported
 * oracle function on small lattices with random solid flags, so that
 * AddressSanitizer and UndefinedBehaviorSanitizer see every index path
 * (periodic wraps on 1-, 2- and 3-site axes, bounce-back next to solids,
 * the transposed streaming of the adjoint).  It also checks two exact
 * properties on the way, so a build that runs is also a build that computes:
 * mass is conserved to rounding by the fused step (Eq. 1 with halfway
 * bounce-back; Section 2), and the rest state f = w is a fixed point.
 * Prints "sanitize_check ok" and exits 0, or prints the failure and exits 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* D3Q19 oracle (d3q19_oracle.c) */
int oracle_q(void);
void oracle_lattice(int *c, double *w, int *opp);
void oracle_feq(double rho, const double *u, double *feq);
void oracle_source(double omega, const double *u, const double *F, double *src);
void oracle_init(int nx, int ny, int nz, const uint8_t *flags, const double *rho, const double *u, double *S);
void oracle_step(int nx, int ny, int nz, const uint8_t *flags, double omega, const double *F,
                 const double *Fx_field, const double *S_in, double *S_out, double *rho_pre, double *u_pre);
int oracle_run(int nx, int ny, int nz, const uint8_t *flags, double omega, const double *F,
               const double *Fx_field, double *S, int nsteps);
void oracle_macros(int nx, int ny, int nz, const uint8_t *flags, const double *F, const double *Fx_field,
                   const double *S, double *rho, double *u);
void oracle_sums(int nx, int ny, int nz, const uint8_t *flags, const double *S, double *out);
void oracle_collision_jacobian(double omega, const double *f, const double *F, double *J, double *dFx);
int oracle_adjoint_step(int nx, int ny, int nz, const uint8_t *flags, double omega, const double *F,
                        const double *Fx_field, const double *S_n, const double *lam_next, double *lam_out,
                        double *grad_fx);
/* D2Q9 oracle (d2q9_oracle.c) */
void oracle2_lattice(int *c, double *w, int *opp);
void oracle2_feq(double rho, const double *u, double *feq);
void oracle2_init(int nx, int ny, const uint8_t *flags, const double *rho, const double *u, double *S);
void oracle2_step(int nx, int ny, const uint8_t *flags, double omega, const double *lid, const double *S_in,
                  double *S_out);
int oracle2_run(int nx, int ny, const uint8_t *flags, double omega, const double *lid, double *S, int nsteps);
void oracle2_macros(int nx, int ny, const uint8_t *flags, const double *S, double *rho, double *u);
void oracle2_sums(int nx, int ny, const uint8_t *flags, const double *S, double *out);

static int failures = 0;

static void expect(int ok, const char *what, double a, double b)
{
    if (!ok) {
        printf("FAIL %s: %.17g vs %.17g\n", what, a, b);
        ++failures;
    }
}

/* xorshift64: a small deterministic generator for the test inputs */
static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double urand(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static void check_d3q19(int nx, int ny, int nz, double solid_fraction, double tau, int steps)
{
    const int Q = oracle_q();
    const size_t N = (size_t)nx * ny * nz;
    uint8_t *flags = malloc(N);
    double *rho = malloc(N * sizeof(double)), *u = malloc(3 * N * sizeof(double));
    double *S = malloc(Q * N * sizeof(double)), *T = malloc(Q * N * sizeof(double));
    double *rho_pre = malloc(N * sizeof(double)), *u_pre = malloc(3 * N * sizeof(double));
    double *fx = malloc(N * sizeof(double)), *lam = malloc(Q * N * sizeof(double));
    double *lam2 = malloc(Q * N * sizeof(double)), *grad = calloc(N, sizeof(double));
    if (!flags || !rho || !u || !S || !T || !rho_pre || !u_pre || !fx || !lam || !lam2 || !grad) {
        printf("FAIL allocation\n");
        exit(1);
    }
    size_t nfluid = 0;
    for (size_t s = 0; s < N; ++s) {
        flags[s] = urand() < solid_fraction;
        nfluid += !flags[s];
        rho[s] = 1.0 + 1e-3 * (urand() - 0.5);
        for (int a = 0; a < 3; ++a) u[a * N + s] = 0.02 * (urand() - 0.5);
        fx[s] = 1e-5 * urand();
    }
    const double F[3] = {1e-5, -2e-6, 3e-6};
    const double omega = 1.0 / tau;
    double before[4], after[4];

    /* mass conservation of the fused step with walls and forces */
    oracle_init(nx, ny, nz, flags, rho, u, S);
    oracle_sums(nx, ny, nz, flags, S, before);
    oracle_step(nx, ny, nz, flags, omega, F, fx, S, T, rho_pre, u_pre);
    if (oracle_run(nx, ny, nz, flags, omega, F, fx, T, steps) != 0) ++failures;
    oracle_sums(nx, ny, nz, flags, T, after);
    expect(fabs(after[0] - before[0]) <= 1e-12 * (double)nfluid, "d3q19 mass", after[0], before[0]);
    oracle_macros(nx, ny, nz, flags, F, fx, T, rho_pre, u_pre);

    /* rest state is a fixed point without force */
    oracle_init(nx, ny, nz, flags, NULL, NULL, S);
    if (oracle_run(nx, ny, nz, flags, omega, NULL, NULL, S, steps) != 0) ++failures;
    double w[19];
    int c[57], opp[19];
    oracle_lattice(c, w, opp);
    double dmax = 0.0;
    for (int i = 0; i < Q; ++i)
        for (size_t s = 0; s < N; ++s)
            if (!flags[s]) dmax = fmax(dmax, fabs(S[(size_t)i * N + s] - w[i]));
    expect(dmax <= 1e-15, "d3q19 rest state", dmax, 0.0);

    /* the adjoint step and the pieces it is built from */
    double f[19], feq[19], src[19], J[19 * 19], dFx[19];
    oracle_feq(1.01, F, feq);
    oracle_source(omega, F, F, src);
    for (int i = 0; i < Q; ++i) f[i] = feq[i] + 1e-4 * (urand() - 0.5);
    oracle_collision_jacobian(omega, f, F, J, dFx);
    oracle_init(nx, ny, nz, flags, rho, u, S);
    for (size_t k = 0; k < (size_t)Q * N; ++k) lam[k] = urand() - 0.5;
    if (oracle_adjoint_step(nx, ny, nz, flags, omega, F, fx, S, lam, lam2, grad) != 0) ++failures;
    for (size_t s = 0; s < N; ++s) {
        if (!isfinite(grad[s])) expect(0, "d3q19 adjoint gradient finite", grad[s], 0.0);
        if (flags[s])
            for (int k = 0; k < Q; ++k)
                if (lam2[(size_t)k * N + s] != 0.0) expect(0, "d3q19 adjoint solid site", lam2[(size_t)k * N + s], 0.0);
    }
    free(flags), free(rho), free(u), free(S), free(T), free(rho_pre), free(u_pre);
    free(fx), free(lam), free(lam2), free(grad);
}

static void check_d2q9(int nx, int ny, double tau, int steps)
{
    const size_t N = (size_t)nx * ny;
    uint8_t *flags = malloc(N);
    double *rho = malloc(N * sizeof(double)), *u = malloc(2 * N * sizeof(double));
    double *S = malloc(9 * N * sizeof(double)), *T = malloc(9 * N * sizeof(double));
    if (!flags || !rho || !u || !S || !T) {
        printf("FAIL allocation\n");
        exit(1);
    }
    /* a cavity: solid frame, with the top row the moving lid's wall */
    size_t nfluid = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const size_t s = (size_t)x + (size_t)nx * y;
            flags[s] = (x == 0 || y == 0 || x == nx - 1 || y == ny - 1);
            nfluid += !flags[s];
            rho[s] = 1.0;
            u[s] = u[N + s] = 0.0;
        }
    const double lid[2] = {0.05, 0.0};
    double before[3], after[3], w[9], feq[9];
    int c[18], opp[9];
    oracle2_lattice(c, w, opp);
    oracle2_feq(1.0, lid, feq);
    oracle2_init(nx, ny, flags, rho, u, S);
    oracle2_sums(nx, ny, flags, S, before);
    oracle2_step(nx, ny, flags, 1.0 / tau, lid, S, T);
    if (oracle2_run(nx, ny, flags, 1.0 / tau, lid, T, steps) != 0) ++failures;
    oracle2_sums(nx, ny, flags, T, after);
    /* the moving wall transfers momentum, not mass */
    expect(fabs(after[0] - before[0]) <= 1e-12 * (double)nfluid, "d2q9 mass", after[0], before[0]);
    oracle2_macros(nx, ny, flags, T, rho, u);
    free(flags), free(rho), free(u), free(S), free(T);
}

int main(void)
{
    check_d3q19(7, 5, 3, 0.2, 0.6, 12);
    check_d3q19(1, 1, 1, 0.0, 1.0, 3);   /* every neighbour is the site itself */
    check_d3q19(2, 1, 4, 0.0, 0.55, 5);
    check_d3q19(6, 6, 6, 0.35, 0.9, 8);
    check_d2q9(9, 7, 0.6, 20);
    check_d2q9(3, 3, 1.0, 4);             /* one fluid site */
    if (failures) {
        printf("sanitize_check: %d failure(s)\n", failures);
        return 1;
    }
    printf("sanitize_check ok\n");
    return 0;
}
