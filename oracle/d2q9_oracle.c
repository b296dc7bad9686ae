/*
 * FP64 reference solver for the two-dimensional D2Q9 BGK update with a
 * moving lid (the paper's own mini-app workload, the lid-driven cavity).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU leg may load it.  It shares no code, header, table or
 * constant with the HIP library (nor with the D3Q19 oracle beside it).
 *
 * What it computes: the lattice Boltzmann equation (paper Eq. 1) with the
 * second-order equilibrium (Eq. 2-3, sound speed squared 1/3) on the nine
 * velocities of the paper's D2Q9 lattice (Section 2), fused as in Section 3.1
 * (pull from the post-collision array, collide, write, swap).  The stored
 * state S is the post-collision array.  One step, for every fluid site x:
 *   1. gather  f_i = S_i(x - c_i)                         (periodic wrap)
 *              f_i = S_opp(i)(x)                           x - c_i is a wall
 *              f_i = S_opp(i)(x) + 6 w_i (c_i . u_lid)     x - c_i is the lid
 *      (halfway bounce-back; the lid, a wall moving with velocity u_lid,
 *       adds the momentum term of Ladd's moving-wall rule with wall density
 *       1: the paper states no-slip walls and a lid moving at constant
 *       tangential velocity but no formula)
 *   2. moments rho = sum f,  u = sum c f / rho
 *   3. f^eq_i = w_i rho (1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u)
 *   4. S'_i(x) = f_i - omega (f_i - f^eq_i)
 * Flags: 0 fluid, 1 wall, 2 lid.  Solid sites are never read as state.
 * Storage: S[i * N + s], s = x + nx y, unshifted FP64.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q2 9

/* D2Q9 velocities: rest, the four axis directions as (+,-) pairs, the diagonals. */
static const int C2[Q2][2] = {{0, 0}, {1, 0}, {-1, 0}, {0, 1}, {0, -1}, {1, 1}, {1, -1}, {-1, 1}, {-1, -1}};

/* Weight from the speed: |c|^2 = 0 -> 4/9, 1 -> 1/9, 2 -> 1/36. */
static double w2(int i)
{
    int c2 = C2[i][0] * C2[i][0] + C2[i][1] * C2[i][1];
    return c2 == 0 ? 4.0 / 9.0 : (c2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
}

static int opp2(int i)
{
    for (int j = 0; j < Q2; ++j)
        if (C2[j][0] == -C2[i][0] && C2[j][1] == -C2[i][1]) return j;
    return -1;
}

static int wrap2(int a, int n)
{
    a %= n;
    return a < 0 ? a + n : a;
}

void oracle2_lattice(int *c, double *w, int *opp)
{
    for (int i = 0; i < Q2; ++i) {
        c[2 * i] = C2[i][0];
        c[2 * i + 1] = C2[i][1];
        w[i] = w2(i);
        opp[i] = opp2(i);
    }
}

void oracle2_feq(double rho, const double *u, double *feq)
{
    double uu = u[0] * u[0] + u[1] * u[1];
    for (int i = 0; i < Q2; ++i) {
        double cu = C2[i][0] * u[0] + C2[i][1] * u[1];
        feq[i] = w2(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
}

/* S_0 = f^eq(rho, u) at fluid sites, f = w at solid ones (rho: N or NULL, u: 2N or NULL). */
void oracle2_init(int nx, int ny, const uint8_t *flags, const double *rho, const double *u, double *S)
{
    size_t N = (size_t)nx * ny;
    for (size_t s = 0; s < N; ++s) {
        double feq[Q2];
        if (flags && flags[s]) {
            for (int i = 0; i < Q2; ++i) feq[i] = w2(i);
        } else {
            double v[2] = {u ? u[s] : 0.0, u ? u[N + s] : 0.0};
            oracle2_feq(rho ? rho[s] : 1.0, v, feq);
        }
        for (int i = 0; i < Q2; ++i) S[(size_t)i * N + s] = feq[i];
    }
}

/* One step S_in -> S_out (solid sites copied).  lid: u_lid (2 values). */
void oracle2_step(int nx, int ny, const uint8_t *flags, double omega, const double *lid, const double *S_in,
                  double *S_out)
{
    size_t N = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t s = (size_t)x + (size_t)nx * y;
            if (flags && flags[s]) {
                for (int i = 0; i < Q2; ++i) S_out[(size_t)i * N + s] = S_in[(size_t)i * N + s];
                continue;
            }
            double f[Q2];
            for (int i = 0; i < Q2; ++i) {
                size_t src = (size_t)wrap2(x - C2[i][0], nx) + (size_t)nx * wrap2(y - C2[i][1], ny);
                int fl = flags ? flags[src] : 0;
                if (fl == 0)
                    f[i] = S_in[(size_t)i * N + src];
                else {
                    f[i] = S_in[(size_t)opp2(i) * N + s];
                    if (fl == 2) f[i] += 6.0 * w2(i) * (C2[i][0] * lid[0] + C2[i][1] * lid[1]);
                }
            }
            double rho = 0.0, m[2] = {0.0, 0.0};
            for (int i = 0; i < Q2; ++i) {
                rho += f[i];
                m[0] += C2[i][0] * f[i];
                m[1] += C2[i][1] * f[i];
            }
            double u[2] = {m[0] / rho, m[1] / rho}, feq[Q2];
            oracle2_feq(rho, u, feq);
            for (int i = 0; i < Q2; ++i) S_out[(size_t)i * N + s] = f[i] - omega * (f[i] - feq[i]);
        }
}

int oracle2_run(int nx, int ny, const uint8_t *flags, double omega, const double *lid, double *S, int nsteps)
{
    if (nsteps <= 0) return 0;
    size_t bytes = (size_t)Q2 * nx * ny * sizeof(double);
    double *T = (double *)malloc(bytes);
    if (!T) return -1;
    double *a = S, *b = T;
    for (int t = 0; t < nsteps; ++t) {
        oracle2_step(nx, ny, flags, omega, lid, a, b);
        double *tmp = a;
        a = b;
        b = tmp;
    }
    if (a != S) memcpy(S, a, bytes);
    free(T);
    return 0;
}

/* rho = sum S, u = sum c S / rho of a stored state; solid sites 0. */
void oracle2_macros(int nx, int ny, const uint8_t *flags, const double *S, double *rho, double *u)
{
    size_t N = (size_t)nx * ny;
    for (size_t s = 0; s < N; ++s) {
        if (flags && flags[s]) {
            rho[s] = u[s] = u[N + s] = 0.0;
            continue;
        }
        double r = 0.0, m0 = 0.0, m1 = 0.0;
        for (int i = 0; i < Q2; ++i) {
            double v = S[(size_t)i * N + s];
            r += v;
            m0 += C2[i][0] * v;
            m1 += C2[i][1] * v;
        }
        rho[s] = r;
        u[s] = m0 / r;
        u[N + s] = m1 / r;
    }
}

/* {sum S, sum c_x S, sum c_y S} over fluid sites. */
void oracle2_sums(int nx, int ny, const uint8_t *flags, const double *S, double *out)
{
    size_t N = (size_t)nx * ny;
    double a[3] = {0.0, 0.0, 0.0};
    for (size_t s = 0; s < N; ++s) {
        if (flags && flags[s]) continue;
        for (int i = 0; i < Q2; ++i) {
            double v = S[(size_t)i * N + s];
            a[0] += v;
            a[1] += C2[i][0] * v;
            a[2] += C2[i][1] * v;
        }
    }
    memcpy(out, a, sizeof a);
}
