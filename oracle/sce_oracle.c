/*
 * sce_oracle.c -- plain FP64 CPU oracle for the spectral canonical
 * electrostatic method (Webb, "A Spectral Canonical Electrostatic Algorithm",
 * arXiv:1508.07344).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * definition that the HIP library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or constant with the HIP library.
 *
 * Every sum here is the plain definition: one cos/sin per (particle, mode)
 * pair, accumulated in index order in double precision with compensated
 * (Neumaier) summation, so the reference stays accurate to a few ulps of the
 * largest partial sum however many particles are summed.  No separable phase
 * tables, no blocking, no reordering.  OpenMP only splits independent outputs
 * (modes for the deposit, particles for the force) across threads; each
 * output's own sum runs serially in index order, so results do not depend on
 * the thread count.
 *
 * Notation (periodic box [0, L)^3, volume V = L^3):
 *   modes      n in Z^3, max_i |n_i| <= n_max, n != 0, wave vector k = 2 pi n / L
 *              (Section 8: spacing 2 pi / L keeps the box periodic).
 *   half space H = { n : n_x > 0, or n_x = 0 and n_y > 0, or n_x = n_y = 0 and
 *              n_z > 0 }; every mode pairs with its negative (Section 4: the
 *              -k partner keeps the potential real), so H holds one of each pair.
 *   shape      S(k) is the particle shape's Fourier transform normalised to
 *              S(0) = 1 (Section 3, the particle-shape transform): Gaussian
 *              exp(-|k|^2 a^2 / 2), point (delta) 1, or tent prod_d sinc^2(k_d a / 2).
 *   deposit    rho_n = S(k_n) sum_j q_j exp(-i k_n . x_j)       (Poisson right-hand side, eq. del_2)
 *   solve      phi_n = rho_n / (eps0 |k_n|^2);  psi_n = S(k_n) phi_n / V
 *              (delta field shape: the k-squared matrix is diagonal, Section 4)
 *   force      F_j = 2 q_j sum_{n in H} k_n Im(psi_n exp(i k_n . x_j))   (kick, eq. del_1)
 *   energy     W = (1 / (eps0 V)) sum_{n in H} |rho_n|^2 / |k_n|^2,
 *              Phi_j = 2 sum_{n in H} Re(psi_n exp(i k_n . x_j)), sum_j q_j Phi_j = 2 W.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

static const double TWO_PI = 6.283185307179586476925286766559;

enum { SHAPE_DELTA = 0, SHAPE_GAUSSIAN = 1, SHAPE_TENT = 2 };

static int in_half_space(int nx, int ny, int nz)
{
    return nx > 0 || (nx == 0 && (ny > 0 || (ny == 0 && nz > 0)));
}

/* Half-space modes in canonical order: n_x = 0..n_max outermost, then
 * n_y = -n_max..n_max, then n_z = -n_max..n_max, keeping those in H.
 * Writes 3 ints per mode to out (if non-NULL); returns the count. */
int64_t sce_oracle_half_modes(int32_t n_max, int32_t *out)
{
    int64_t c = 0;
    for (int nx = 0; nx <= n_max; ++nx)
        for (int ny = -n_max; ny <= n_max; ++ny)
            for (int nz = -n_max; nz <= n_max; ++nz) {
                if (!in_half_space(nx, ny, nz)) continue;
                if (out) { out[3 * c] = nx; out[3 * c + 1] = ny; out[3 * c + 2] = nz; }
                ++c;
            }
    return c;
}

/* All modes of the cube except n = 0, lexicographic from (-n_max,-n_max,-n_max). */
int64_t sce_oracle_cube_modes(int32_t n_max, int32_t *out)
{
    int64_t c = 0;
    for (int nx = -n_max; nx <= n_max; ++nx)
        for (int ny = -n_max; ny <= n_max; ++ny)
            for (int nz = -n_max; nz <= n_max; ++nz) {
                if (nx == 0 && ny == 0 && nz == 0) continue;
                if (out) { out[3 * c] = nx; out[3 * c + 1] = ny; out[3 * c + 2] = nz; }
                ++c;
            }
    return c;
}

static double sinc(double u) { return u == 0.0 ? 1.0 : sin(u) / u; }

/* Shape factor S(k) for wave vector k (Section 3, particle-shape transform). */
double sce_oracle_shape(int32_t kind, double a, double kx, double ky, double kz)
{
    switch (kind) {
    case SHAPE_DELTA: return 1.0;
    case SHAPE_GAUSSIAN: return exp(-0.5 * (kx * kx + ky * ky + kz * kz) * a * a);
    case SHAPE_TENT: {
        double sx = sinc(0.5 * kx * a), sy = sinc(0.5 * ky * a), sz = sinc(0.5 * kz * a);
        return sx * sx * sy * sy * sz * sz;
    }
    default: return NAN;
    }
}

/* Compensated running sum (Neumaier's variant of Kahan summation). */
typedef struct { double s, c; } csum;
static void csum_add(csum *a, double x)
{
    const double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double csum_get(const csum *a) { return a->s + a->c; }

/* Phase k_n . x_j for mode (nx, ny, nz). */
static double phase(double L, int nx, int ny, int nz, double x, double y, double z)
{
    return (TWO_PI / L) * ((double)nx * x + (double)ny * y + (double)nz * z);
}

/* Deposit: rho_n = S(k_n) sum_j q_j exp(-i k_n . x_j) for each listed mode.
 * rho is interleaved (re, im) per mode. */
void sce_oracle_deposit(int64_t N, const double *x, const double *y, const double *z,
                        const double *q, double L, int64_t n_modes, const int32_t *modes,
                        int32_t kind, double a, double *rho)
{
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_modes; ++i) {
        const int nx = modes[3 * i], ny = modes[3 * i + 1], nz = modes[3 * i + 2];
        csum re = {0.0, 0.0}, im = {0.0, 0.0};
        for (int64_t j = 0; j < N; ++j) {
            const double th = phase(L, nx, ny, nz, x[j], y[j], z[j]);
            csum_add(&re, q[j] * cos(th));
            csum_add(&im, -q[j] * sin(th));
        }
        const double f = TWO_PI / L;
        const double s = sce_oracle_shape(kind, a, f * nx, f * ny, f * nz);
        rho[2 * i] = s * csum_get(&re);
        rho[2 * i + 1] = s * csum_get(&im);
    }
}

/* Field solve: psi_n = S(k_n) rho_n / (eps0 |k_n|^2 V). */
void sce_oracle_psi(int64_t n_modes, const int32_t *modes, const double *rho, double L,
                    double eps0, int32_t kind, double a, double *psi)
{
    const double f = TWO_PI / L, V = L * L * L;
    for (int64_t i = 0; i < n_modes; ++i) {
        const double kx = f * modes[3 * i], ky = f * modes[3 * i + 1], kz = f * modes[3 * i + 2];
        const double k2 = kx * kx + ky * ky + kz * kz;
        const double w = sce_oracle_shape(kind, a, kx, ky, kz) / (eps0 * k2 * V);
        psi[2 * i] = w * rho[2 * i];
        psi[2 * i + 1] = w * rho[2 * i + 1];
    }
}

/* Force: F_j = 2 q_j sum_{n in H} k_n Im(psi_n exp(i k_n . x_j)).
 * Output F is [3][N] (structure of arrays). */
void sce_oracle_force(int64_t N, const double *x, const double *y, const double *z,
                      const double *q, double L, int64_t n_modes, const int32_t *modes,
                      const double *psi, double *F)
{
    const double f = TWO_PI / L;
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        csum fx = {0.0, 0.0}, fy = {0.0, 0.0}, fz = {0.0, 0.0};
        for (int64_t i = 0; i < n_modes; ++i) {
            const int nx = modes[3 * i], ny = modes[3 * i + 1], nz = modes[3 * i + 2];
            const double th = phase(L, nx, ny, nz, x[j], y[j], z[j]);
            /* Im((pr + i pi)(cos + i sin)) = pr sin + pi cos */
            const double im = psi[2 * i] * sin(th) + psi[2 * i + 1] * cos(th);
            csum_add(&fx, f * nx * im);
            csum_add(&fy, f * ny * im);
            csum_add(&fz, f * nz * im);
        }
        F[j] = 2.0 * q[j] * csum_get(&fx);
        F[N + j] = 2.0 * q[j] * csum_get(&fy);
        F[2 * N + j] = 2.0 * q[j] * csum_get(&fz);
    }
}

/* Potential at each particle: Phi_j = 2 sum_{n in H} Re(psi_n exp(i k_n . x_j)). */
void sce_oracle_potential(int64_t N, const double *x, const double *y, const double *z,
                          double L, int64_t n_modes, const int32_t *modes, const double *psi,
                          double *Phi)
{
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        csum s = {0.0, 0.0};
        for (int64_t i = 0; i < n_modes; ++i) {
            const double th = phase(L, modes[3 * i], modes[3 * i + 1], modes[3 * i + 2],
                                    x[j], y[j], z[j]);
            csum_add(&s, psi[2 * i] * cos(th) - psi[2 * i + 1] * sin(th));
        }
        Phi[j] = 2.0 * csum_get(&s);
    }
}

/* Field energy W = (1 / (eps0 V)) sum_{n in H} |rho_n|^2 / |k_n|^2. */
double sce_oracle_field_energy(int64_t n_modes, const int32_t *modes, const double *rho,
                               double L, double eps0)
{
    const double f = TWO_PI / L, V = L * L * L;
    csum s = {0.0, 0.0};
    for (int64_t i = 0; i < n_modes; ++i) {
        const double kx = f * modes[3 * i], ky = f * modes[3 * i + 1], kz = f * modes[3 * i + 2];
        const double k2 = kx * kx + ky * ky + kz * kz;
        csum_add(&s, (rho[2 * i] * rho[2 * i] + rho[2 * i + 1] * rho[2 * i + 1]) / k2);
    }
    return csum_get(&s) / (eps0 * V);
}

/* ---------------------------------------------------------------- two dimensions
 * The paper's own test problems are two-dimensional (Section 6, the two-body
 * problem; Section 7, the thermal plasma): particles are line charges in the
 * periodic square [0, L)^2 of area A = L^2.  Same definitions with two
 * components:
 *   modes      n in Z^2, max_i |n_i| <= n_max, n != 0, k_n = 2 pi n / L.
 *   half plane H2 = { n_x > 0 } u { n_x = 0, n_y > 0 }; canonical order
 *              n_x = 0..n_max, then n_y = -n_max..n_max, keeping those in H2.
 *   shape      S(k) of the two-component wave vector (Gaussian exp(-|k|^2 a^2/2),
 *              point 1, tent sinc^2(k_x a/2) sinc^2(k_y a/2)).
 *   deposit    rho_n = S(k_n) sum_j q_j exp(-i k_n . x_j)
 *   solve      psi_n = S(k_n) rho_n / (eps0 |k_n|^2 A)
 *   force      F_j = 2 q_j sum_{n in H2} k_n Im(psi_n exp(i k_n . x_j))   ([2][N])
 *   energy     W = (1 / (eps0 A)) sum_{n in H2} |rho_n|^2 / |k_n|^2.
 * Mode arrays hold 2 ints per mode. */
static int in_half_plane(int nx, int ny) { return nx > 0 || (nx == 0 && ny > 0); }

int64_t sce_oracle_half_modes_2d(int32_t n_max, int32_t *out)
{
    int64_t c = 0;
    for (int nx = 0; nx <= n_max; ++nx)
        for (int ny = -n_max; ny <= n_max; ++ny) {
            if (!in_half_plane(nx, ny)) continue;
            if (out) { out[2 * c] = nx; out[2 * c + 1] = ny; }
            ++c;
        }
    return c;
}

/* All modes of the square except n = 0, lexicographic from (-n_max, -n_max). */
int64_t sce_oracle_square_modes(int32_t n_max, int32_t *out)
{
    int64_t c = 0;
    for (int nx = -n_max; nx <= n_max; ++nx)
        for (int ny = -n_max; ny <= n_max; ++ny) {
            if (nx == 0 && ny == 0) continue;
            if (out) { out[2 * c] = nx; out[2 * c + 1] = ny; }
            ++c;
        }
    return c;
}

/* S(k) of a two-component wave vector: the particle-shape transforms above
 * with no third component (the tent's third factor sinc^2(0) = 1). */
double sce_oracle_shape_2d(int32_t kind, double a, double kx, double ky)
{
    return sce_oracle_shape(kind, a, kx, ky, 0.0);
}

void sce_oracle_deposit_2d(int64_t N, const double *x, const double *y, const double *q, double L,
                           int64_t n_modes, const int32_t *modes, int32_t kind, double a,
                           double *rho)
{
    const double f = TWO_PI / L;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_modes; ++i) {
        const int nx = modes[2 * i], ny = modes[2 * i + 1];
        csum re = {0.0, 0.0}, im = {0.0, 0.0};
        for (int64_t j = 0; j < N; ++j) {
            const double th = f * ((double)nx * x[j] + (double)ny * y[j]);
            csum_add(&re, q[j] * cos(th));
            csum_add(&im, -q[j] * sin(th));
        }
        const double s = sce_oracle_shape_2d(kind, a, f * nx, f * ny);
        rho[2 * i] = s * csum_get(&re);
        rho[2 * i + 1] = s * csum_get(&im);
    }
}

void sce_oracle_psi_2d(int64_t n_modes, const int32_t *modes, const double *rho, double L,
                       double eps0, int32_t kind, double a, double *psi)
{
    const double f = TWO_PI / L, A = L * L;
    for (int64_t i = 0; i < n_modes; ++i) {
        const double kx = f * modes[2 * i], ky = f * modes[2 * i + 1];
        const double k2 = kx * kx + ky * ky;
        const double w = sce_oracle_shape_2d(kind, a, kx, ky) / (eps0 * k2 * A);
        psi[2 * i] = w * rho[2 * i];
        psi[2 * i + 1] = w * rho[2 * i + 1];
    }
}

void sce_oracle_force_2d(int64_t N, const double *x, const double *y, const double *q, double L,
                         int64_t n_modes, const int32_t *modes, const double *psi, double *F)
{
    const double f = TWO_PI / L;
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        csum fx = {0.0, 0.0}, fy = {0.0, 0.0};
        for (int64_t i = 0; i < n_modes; ++i) {
            const int nx = modes[2 * i], ny = modes[2 * i + 1];
            const double th = f * ((double)nx * x[j] + (double)ny * y[j]);
            const double im = psi[2 * i] * sin(th) + psi[2 * i + 1] * cos(th);
            csum_add(&fx, f * nx * im);
            csum_add(&fy, f * ny * im);
        }
        F[j] = 2.0 * q[j] * csum_get(&fx);
        F[N + j] = 2.0 * q[j] * csum_get(&fy);
    }
}

void sce_oracle_potential_2d(int64_t N, const double *x, const double *y, double L, int64_t n_modes,
                             const int32_t *modes, const double *psi, double *Phi)
{
    const double f = TWO_PI / L;
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < N; ++j) {
        csum s = {0.0, 0.0};
        for (int64_t i = 0; i < n_modes; ++i) {
            const double th = f * ((double)modes[2 * i] * x[j] + (double)modes[2 * i + 1] * y[j]);
            csum_add(&s, psi[2 * i] * cos(th) - psi[2 * i + 1] * sin(th));
        }
        Phi[j] = 2.0 * csum_get(&s);
    }
}

double sce_oracle_field_energy_2d(int64_t n_modes, const int32_t *modes, const double *rho,
                                  double L, double eps0)
{
    const double f = TWO_PI / L, A = L * L;
    csum s = {0.0, 0.0};
    for (int64_t i = 0; i < n_modes; ++i) {
        const double kx = f * modes[2 * i], ky = f * modes[2 * i + 1];
        const double k2 = kx * kx + ky * ky;
        csum_add(&s, (rho[2 * i] * rho[2 * i] + rho[2 * i + 1] * rho[2 * i + 1]) / k2);
    }
    return csum_get(&s) / (eps0 * A);
}

/* Number of threads OpenMP will use (reported with the CPU baseline). */
int32_t sce_oracle_threads(void)
{
    int n = 1;
    #pragma omp parallel
    {
        #pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}

/* Set the number of threads of the parallel loops above (the CPU baseline's
 * one-core and all-core runs); n < 1 is ignored.  The results do not depend on
 * it: each output's sum runs serially in index order. */
void sce_oracle_set_threads(int32_t n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
