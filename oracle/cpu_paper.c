/*
 * cpu_paper.c -- a CPU comparison baseline for the benchmark, written with the
 * optimisations the paper itself proposes for the mode sums (Section 8): only
 * the half space of modes is kept, and each particle evaluates D = 3
 * exponentials cis(2 pi x_d / L); every mode's phase is a product of integer
 * powers of those three (the modes are spaced by 2 pi / L).
 *
 * NOT A CHECKER.  The oracle (sce_oracle.c) is the definition the HIP library
 * is checked against; this file is only timed by the benchmark's CPU-baseline
 * leg, and the CPU tests pin it against the oracle.  Like the oracle it is
 * test and benchmark infrastructure: only the test suite and the benchmark
 * load it, and it shares no code with the HIP library.
 *
 * Layout: the half space H in the oracle's canonical order (n_x = 0..n
 * outermost, then n_y = -n..n, then n_z = -n..n, keeping those in H).  The
 * sums run over full rows (n_x, n_y, n_z = -n..n) of a dense
 * (n+1) x (2n+1) x (2n+1) box and are then read out in canonical order.
 *
 *   deposit  rho_n = S_n sum_j q_j conj(e_x^{n_x} e_y^{n_y} e_z^{n_z})
 *   force    F_j   = 2 q_j sum_{n in H} k_n Im(psi_n e_x^{n_x} e_y^{n_y} e_z^{n_z})
 * with e_d = cis(2 pi x_{j,d} / L) and k_n = 2 pi n / L.
 *
 * OpenMP over particles, in blocks of PB particles that share each row's
 * pass over the mode table.  The deposit keeps one box of sums per thread and
 * adds them in thread order at the end; the force writes each particle once.
 * Powers are formed by repeated complex multiplication from one sincos per
 * coordinate (about k ulps of rounding at power k).  Both sums return 0, or
 * -1 when a work buffer cannot be allocated (the output is then not written).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double TWO_PI = 6.283185307179586476925286766559;

enum { PB = 8 };  /* particles per block */

/* (cos, sin)(k theta) for k = -n..n into c[(k + n) * st], s[(k + n) * st] */
static void powers(double theta, int n, double *c, double *s, int st)
{
    const double c1 = cos(theta), s1 = sin(theta);
    double pc = 1.0, ps = 0.0;
    c[n * st] = 1.0;
    s[n * st] = 0.0;
    for (int k = 1; k <= n; ++k) {
        const double t = pc * c1 - ps * s1;
        ps = pc * s1 + ps * c1;
        pc = t;
        c[(n + k) * st] = pc;
        s[(n + k) * st] = ps;
        c[(n - k) * st] = pc;
        s[(n - k) * st] = -ps;
    }
}

static int in_half(int nx, int ny, int nz)
{
    return nx > 0 || (nx == 0 && (ny > 0 || (ny == 0 && nz > 0)));
}

int32_t sce_cpu_paper_threads(void)
{
#ifdef _OPENMP
    return (int32_t)omp_get_max_threads();
#else
    return 1;
#endif
}

void sce_cpu_paper_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* rho (2 doubles per mode of H, canonical order) = S_n sum_j q_j exp(-i k_n . x_j).
 * S: the shape factor per mode of H (canonical order).  Per thread, the sums
 * of a row (n_x, n_y) are two arrays over n_z (real and imaginary parts), and
 * the row loop runs over n_z for each particle of the block. */
int32_t sce_cpu_paper_deposit(int64_t N, const double *x, const double *y, const double *z,
                              const double *q, double L, int32_t n, const double *S, double *rho)
{
    const int M = 2 * n + 1;
    const size_t box = (size_t)(n + 1) * M * M;
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double *acc = (double *)calloc((size_t)nt * box * 2, sizeof(double));
    if (!acc) return -1;
    int failed = 0;
#pragma omp parallel num_threads(nt)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        double *are = acc + (size_t)t * box * 2, *aim = are + box;
        /* per particle of the block: x and y powers (k = -n..n), z powers */
        double *tab = (double *)malloc(sizeof(double) * M * PB * 6);
        if (!tab) {
#pragma omp atomic write
            failed = 1;
        }
        double *xc = tab, *xs = xc + M * PB, *yc = xs + M * PB, *ys = yc + M * PB;
        double *zc = ys + M * PB, *zs = zc + M * PB;
        const int64_t nblk = (N + PB - 1) / PB;
#pragma omp for schedule(static)
        for (int64_t b = 0; b < nblk; ++b) {
            if (!tab) continue;
            const int64_t j0 = b * PB;
            const int np = N - j0 < PB ? (int)(N - j0) : PB;
            double qq[PB];
            for (int p = 0; p < PB; ++p) {
                const int64_t j = j0 + (p < np ? p : 0);
                qq[p] = p < np ? q[j] : 0.0;
                /* exp(-i k x): powers of cis(-2 pi x / L) */
                powers(-TWO_PI * x[j] / L, n, xc + M * p, xs + M * p, 1);
                powers(-TWO_PI * y[j] / L, n, yc + M * p, ys + M * p, 1);
                powers(-TWO_PI * z[j] / L, n, zc + M * p, zs + M * p, 1);
            }
            for (int nx = 0; nx <= n; ++nx)
                for (int ny = -n; ny <= n; ++ny) {
                    if (nx == 0 && ny < 0) continue;
                    double *rr = are + ((size_t)nx * M + (ny + n)) * M;
                    double *ri = aim + ((size_t)nx * M + (ny + n)) * M;
                    for (int p = 0; p < PB; ++p) {
                        const double exr = xc[M * p + nx + n], exi = xs[M * p + nx + n];
                        const double eyr = yc[M * p + ny + n], eyi = ys[M * p + ny + n];
                        const double ar = qq[p] * (exr * eyr - exi * eyi);
                        const double ai = qq[p] * (exr * eyi + exi * eyr);
                        const double *cz = zc + M * p, *sz = zs + M * p;
                        for (int k = 0; k < M; ++k) {
                            rr[k] += ar * cz[k] - ai * sz[k];
                            ri[k] += ar * sz[k] + ai * cz[k];
                        }
                    }
                }
        }
        free(tab);
    }
    if (failed) {
        free(acc);
        return -1;
    }
    /* threads' sums in thread order, read out over H in canonical order */
    int64_t c = 0;
    for (int nx = 0; nx <= n; ++nx)
        for (int ny = -n; ny <= n; ++ny)
            for (int nz = -n; nz <= n; ++nz) {
                if (!in_half(nx, ny, nz)) continue;
                const size_t o = ((size_t)nx * M + (ny + n)) * M + (nz + n);
                double sr = 0.0, si = 0.0;
                for (int t = 0; t < nt; ++t) {
                    sr += acc[(size_t)t * box * 2 + o];
                    si += acc[(size_t)t * box * 2 + box + o];
                }
                rho[2 * c] = S[c] * sr;
                rho[2 * c + 1] = S[c] * si;
                ++c;
            }
    free(acc);
    return 0;
}

/* F [3][N] = 2 q_j sum_{n in H} k_n Im(psi_n exp(i k_n . x_j)); psi: 2 doubles
 * per mode of H in canonical order.  Per row (n_x, n_y), the block's
 * particles take T = sum_nz psi e_z^nz and Tz = sum_nz n_z psi e_z^nz side by
 * side (the z powers stored particle-fastest), then Im(e_x^nx e_y^ny T). */
int32_t sce_cpu_paper_force(int64_t N, const double *x, const double *y, const double *z,
                            const double *q, double L, int32_t n, const double *psi, double *F)
{
    const int M = 2 * n + 1;
    const size_t box = (size_t)(n + 1) * M * M;
    /* psi on the dense box (real parts, then imaginary parts), zero outside H */
    double *pre = (double *)calloc(box * 2, sizeof(double));
    if (!pre) return -1;
    int failed = 0;
    double *pim = pre + box;
    {
        int64_t c = 0;
        for (int nx = 0; nx <= n; ++nx)
            for (int ny = -n; ny <= n; ++ny)
                for (int nz = -n; nz <= n; ++nz) {
                    if (!in_half(nx, ny, nz)) continue;
                    const size_t o = ((size_t)nx * M + (ny + n)) * M + (nz + n);
                    pre[o] = psi[2 * c];
                    pim[o] = psi[2 * c + 1];
                    ++c;
                }
    }
#pragma omp parallel
    {
        double *tab = (double *)malloc(sizeof(double) * M * PB * 6);
        if (!tab) {
#pragma omp atomic write
            failed = 1;
        }
        double *xc = tab, *xs = xc + M * PB, *yc = xs + M * PB, *ys = yc + M * PB;
        double *zc = ys + M * PB, *zs = zc + M * PB;
        const int64_t nblk = (N + PB - 1) / PB;
#pragma omp for schedule(static)
        for (int64_t b = 0; b < nblk; ++b) {
            if (!tab) continue;
            const int64_t j0 = b * PB;
            const int np = N - j0 < PB ? (int)(N - j0) : PB;
            for (int p = 0; p < PB; ++p) {
                const int64_t j = j0 + (p < np ? p : 0);
                powers(TWO_PI * x[j] / L, n, xc + M * p, xs + M * p, 1);
                powers(TWO_PI * y[j] / L, n, yc + M * p, ys + M * p, 1);
                powers(TWO_PI * z[j] / L, n, zc + p, zs + p, PB);
            }
            double fx[PB] = {0}, fy[PB] = {0}, fz[PB] = {0};
            for (int nx = 0; nx <= n; ++nx)
                for (int ny = -n; ny <= n; ++ny) {
                    if (nx == 0 && ny < 0) continue;
                    const double *rr = pre + ((size_t)nx * M + (ny + n)) * M;
                    const double *ri = pim + ((size_t)nx * M + (ny + n)) * M;
                    double tr[PB] = {0}, ti[PB] = {0}, zr[PB] = {0}, zi[PB] = {0};
                    for (int k = 0; k < M; ++k) {
                        const double pr = rr[k], pi = ri[k], w = (double)(k - n);
                        const double *cz = zc + PB * k, *sz = zs + PB * k;
                        for (int p = 0; p < PB; ++p) {
                            const double ur = pr * cz[p] - pi * sz[p];
                            const double ui = pr * sz[p] + pi * cz[p];
                            tr[p] += ur;
                            ti[p] += ui;
                            zr[p] += w * ur;
                            zi[p] += w * ui;
                        }
                    }
                    for (int p = 0; p < PB; ++p) {
                        const double exr = xc[M * p + nx + n], exi = xs[M * p + nx + n];
                        const double eyr = yc[M * p + ny + n], eyi = ys[M * p + ny + n];
                        const double ar = exr * eyr - exi * eyi;
                        const double ai = exr * eyi + exi * eyr;
                        const double im0 = ar * ti[p] + ai * tr[p];  /* Im(a T) */
                        const double im1 = ar * zi[p] + ai * zr[p];  /* Im(a Tz) */
                        fx[p] += nx * im0;
                        fy[p] += ny * im0;
                        fz[p] += im1;
                    }
                }
            const double f = 2.0 * TWO_PI / L;
            for (int p = 0; p < np; ++p) {
                const int64_t j = j0 + p;
                F[j] = f * q[j] * fx[p];
                F[N + j] = f * q[j] * fy[p];
                F[2 * N + j] = f * q[j] * fz[p];
            }
        }
        free(tab);
    }
    free(pre);
    return failed ? -1 : 0;
}
