// Internal declarations shared by the HIP kernels and the host runtime of the
// spectral canonical electrostatic library (gfx950).
//
// Mode layout in HBM ("row layout").  The stored half space H is covered by
// rows r = (n_x, n_y) and a full n_z line per row:
//   rows 0..n        : n_x = 0, n_y = r            (n_y < 0 at n_x = 0 lies in -H)
//   rows n+1..R-1    : n_x = 1 + (r-n-1) / M, n_y = (r-n-1) % M - n
//   R = (n+1) + n M, M = 2n+1; padded mode p = r M + (n_z + n), P = R M.
// A two-dimensional context (line charges, modes (m_x, m_y)) keeps only rows
// 0..n: its half plane {m_x > 0} u {m_x = 0, m_y > 0} is the n_x = 0 slice of
// H with (n_y, n_z) = (m_x, m_y), so its particles are stored with x = 0 and
// (y, z) = their (x, y), and R = n + 1.
// Row 0 holds n_z = -n..0, which are not in H (0 and the negatives of row 0's
// positive half); everything else is in H, so the canonical mode index is
// simply p - (n+1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sce {

struct Geom {
    int n;       // n_max
    int M;       // 2n+1
    int n1;      // n+1
    int R;       // rows
    int Rpad;    // rows rounded up to 64
    int64_t P;   // padded modes R*M
    int64_t H;   // |H| = P - (n+1)
    int lines;   // n_x lines of the row layout: n + 1 in 3-D, 1 in 2-D (rows 0..n only)
    int nzp;     // n_z slots of the force table (n rounded up to the force chunk)
    int zslots;  // n_z slots (0..zslots-1) of the per-particle phase table, >= n+1
};

__host__ __device__ inline void row_nxny(int r, int n, int &nx, int &ny)
{
    if (r <= n) { nx = 0; ny = r; return; }
    const int rr = r - (n + 1), M = 2 * n + 1;
    nx = 1 + rr / M;
    ny = rr % M - n;
}

// n_z values per register chunk of the force kernel: 8, 16 or 32; FP64 caps
// at 16 (cos/sin of 16 n_z in 64 VGPRs keeps three waves per SIMD).
inline int force_chunk(int n, int elem_bytes)
{
    const int c = n <= 8 ? 8 : (n <= 16 ? 16 : 32);
    return elem_bytes == 8 && c > 16 ? 16 : c;
}

__host__ __device__ inline bool in_half(int nx, int ny, int nz)
{
    return nx > 0 || (nx == 0 && (ny > 0 || (ny == 0 && nz > 0)));
}

// Kernel launchers (kernels.hip).  All return hipError_t of the launch.
// Precision-templated launchers take T = float or double.

// Per-particle phase tables, theta_d = 2 pi x_d / L:
//   exy[j][d][k] = (cos, sin)(k theta_d), d = x, y, k = 0..n, FP64;
//   tz[j][k]     = (cos, sin)(k theta_z), k = 0..n, zeros up to zslots, type T.
template <typename T>
hipError_t launch_phase_table(hipStream_t s, const double *pos, int64_t N, const Geom &g,
                              double L, double2 *exy, T *tz);

// Deposit partial sums for one particle split per blockIdx.z.  part layout
// [split][n_z in 0..n][4][Rpad] doubles: (P_re, P_im, Q_re, Q_im) with
// P = sum q e^{-i(nx tx + ny ty)} cos(nz tz), Q = same with sin.
struct DepositPlan {
    int zb;             // n_z per wave group
    int groups;         // ceil(n / zb)
    int waves_per_rs;   // waves sharing one 64-row set
    int rows_per_wg;    // 64 * row sets
    int grid_y;         // ceil(groups / waves_per_rs)
    int row_blocks;     // ceil(R / rows_per_wg)
    int kc;             // particles per LDS chunk
    int splits;
    int64_t per_split;
};
DepositPlan plan_deposit(const Geom &g, int64_t N, int elem_bytes);
template <typename T>
hipError_t launch_deposit(hipStream_t s, const double2 *exy, const T *tz, const double *q, int64_t N,
                          const Geom &g, const DepositPlan &pl, double *part);

// Sum the partials over splits in fixed order, form rho and psi on the padded
// layout, the force table and the per-block (W, max|rho|) partials (one block
// per 64 cells (row, n_z); wpart holds 2 doubles per block).
// ftab layout [R][nzp][8] of T: (sig_re, sig_im, del_re, del_im, nz del_re,
// nz del_im, nz sig_re, nz sig_im) for n_z = 1..nzp with sig = psi(+nz) + psi(-nz),
// del = psi(+nz) - psi(-nz); psi0 [R][2]: psi at n_z = 0.  Partials P: FP64
// from the direct deposits, FP32 from the matrix-core one (summed in FP64).
template <typename T, typename P>
hipError_t launch_reduce_solve(hipStream_t s, const P *part, int splits, const Geom &g,
                               const double *Stab, const double *Gtab, const double *Ktab,
                               double2 *rho, double2 *psi, T *ftab, T *psi0, double *wpart,
                               int *wblocks);

// Force (and potential) at the current positions; optional kick v += kick F/m.
// Between the small-count kernel and kForceLineBlocks blocks of 256 particles
// the rows are split evenly over force_line_groups(...) groups of blocks, whose
// FP64 partial sums go to part ([groups][4][N] doubles, caller-owned) and are
// then added in a fixed order.
constexpr int kForceLineBlocks = 1024;
int force_line_groups(const Geom &g, int64_t N, int elem_bytes);
template <typename T>
hipError_t launch_force(hipStream_t s, const double *pos, const double *q, const double *m,
                        double *vel, const T *ftab, const T *psi0, const Geom &g, double L,
                        int64_t N, double kick, double *F, double *phi, double *part);

// ---- split-precision matrix-core path (kernels_mfma.hip)
struct MfmaDepositPlan {
    int row_blocks;     // blocks of 12 matrix-core waves over the groups of 16 (k_x, k_y) pairs
    int splits;
    int64_t per_split;
    int64_t perm;       // half width h of the Feistel visiting order (2^(2h) >= N)
};
MfmaDepositPlan plan_deposit_mfma(const Geom &g, int64_t N);
// Deposit partial sums (layout of launch_deposit, in FP32).  rec: scratch of
// deposit_mfma_rec_bytes(N) for the chunk images in visiting order; charges
// enter scaled by 1/qscale and the partials leave scaled back.
size_t deposit_mfma_rec_bytes(int64_t N, int n);
hipError_t launch_deposit_mfma(hipStream_t s, const double *pos, const double *q, int64_t N,
                               const Geom &g, double L, const MfmaDepositPlan &pl, double qscale,
                               float *rec, float *part);
// Pack the FP32 force table into FP16 hi/lo matrix-core fragments in quads of
// rows (line 0, then one column of n_x = 1..n per n_y, each padded to whole
// quads), each row scaled by its power-of-two scale s; rinfo
// (force_rowinfo_bytes) receives per padded row (psi(r,0) / s, 0, 0) and
// (n_x s, n_y s, s, 0).
size_t force_pack_bytes(const Geom &g);
size_t force_rowinfo_bytes(const Geom &g);
hipError_t launch_force_pack(hipStream_t s, const float *ftab, const float *psi0, const Geom &g,
                             float4 *rinfo, _Float16 *wf);
// After the force and its kick, optionally the next leapfrog step's first
// half kick v += kick F / m and drift x += drift v (wrapped into [0, L) when
// wrap), with the operations of launch_kick_drift: a KDK step's closing half
// kick, the next step's opening half kick and its drift in one pass (F
// required, phi not: the potential's variant does not take them).
struct Drift {
    double kick = 0.0;
    double drift = 0.0;
    int wrap = 0;
};
hipError_t launch_force_mfma(hipStream_t s, double *pos, const double *q, const double *m,
                             double *vel, const _Float16 *wf, const float4 *rinfo, const Geom &g,
                             double L, int64_t N, double kick, const Drift &nd, double *F,
                             double *phi);

// v += a F/m (if a != 0); x = x + b v (if b != 0), wrapped into [0, L) when wrap.
hipError_t launch_kick_drift(hipStream_t s, double *pos, double *vel, const double *F,
                             const double *m, int64_t N, double L, double a, double b, bool wrap);

// Flag bad particle input (kernels.hip k_check_particles): *flag |= 1 for a
// non-finite x, v or q, |= 2 for a mass that is not finite and > 0.  The
// caller zeroes *flag first.
hipError_t launch_check_particles(hipStream_t s, const double *pos, const double *vel,
                                  const double *q, const double *m, int64_t N, unsigned *flag);

// Wrap positions into [0, L).
hipError_t launch_wrap(hipStream_t s, double *pos, int64_t N, double L);

// Diagnostics: per-block partial sums then a single-block fixed-order finish.
// out[0] = K, out[1..3] = P, out[4] = sum m|v|, out[5] = sum q phi,
// out[6] = W, out[7] = max|rho|.
hipError_t launch_diag(hipStream_t s, const double *vel, const double *q, const double *m,
                       const double *phi, int64_t N, const double *wpart, int wblocks,
                       double eps0V, double *scratch, double *out);

// ---- small systems: many steps in one single-workgroup launch (kernels_small.hip)
constexpr int kSmallThreads = 1024;
constexpr int kSmallMaxN = 256;     // particles
constexpr int kSmallMaxH = 3072;    // stored modes
constexpr int kSmallMaxTab = 3072;  // phase-table entries N * 3 * (n + 1)
// steps KDK (kdk) or DKD steps of size dt; modes: the stored half space as
// (n_x, n_y, n_z, 0) in canonical order, wmode = S^2 / (eps0 |k|^2 V) per mode;
// F must hold the force at the current positions for KDK and holds the force
// of the last evaluation afterwards.
hipError_t launch_step_small(hipStream_t s, double *pos, double *vel, double *F, const double *q,
                             const double *m, int64_t N, const short4 *modes, const double *wmode,
                             const Geom &g, double L, double dt, int steps, bool kdk);

// ---- finite-width tent field shapes, point particles (kernels_tent.hip)
// Envelope E(x), its gradient (env [4][N]: E, dE/dx, dE/dy, dE/dz) and the
// weighted charges qw = q E; dim 2 spans only the stored y and z.
hipError_t launch_tent_prep(hipStream_t s, const double *pos, const double *q, int64_t N, int dim,
                            double L, double *qw, double *env);
// From the stored rows of rho (deposited with charges qw, S = 1, the origin
// included): expand to the full cube (X), solve M phi = rho / eps0 by the
// separable eigenbases (Vf[j M + i] = V[j][i], Vb[j M + i] = V[i][j], lam), and
// write psi, the force table, psi0 and the (W, max|rho|) block partials.
template <typename T>
hipError_t launch_tent_solve(hipStream_t s, const double2 *rho, const Geom &g, int dim,
                             const double *Vf, const double *Vb, const double *lam, double eps0,
                             double2 *X, double2 *Y, double2 *psi, T *ftab, T *psi0,
                             double *wpart, int *wblocks);
// F = E F' - q grad(E) P, phi = E P from the force kernels' F' and P; v += kick F / m.
hipError_t launch_tent_combine(hipStream_t s, const double *env, const double *q, const double *m,
                               const double *Fk, const double *Pk, int64_t N, double kick,
                               double *vel, double *F, double *phi);

}  // namespace sce
