// Direct (VALU) kernels of the spectral canonical electrostatic hot path on
// gfx950: per-particle phase tables, the deposit (type-1 nonuniform DFT), the
// cross-tile reduction with the field solve, the force (type-2 nonuniform
// DFT) with a fused kick, drift/kick, and FP64 diagnostics.
//
// Both particle x mode sums use the paper's separable phases (Section 8: with
// modes spaced 2 pi / L, each per-mode exponential is an integer power of one
// exponential per axis), plus the fact that the particle weights are real, so
// that the +n_z and -n_z modes of a row share cos(n_z theta_z) and
// sin(n_z theta_z):
//   deposit  P(r, nz) = sum_j h_j(r) cos(nz tz_j),  Q(r, nz) = sum_j h_j(r) sin(nz tz_j),
//            h_j(r) = q_j exp(-i (nx tx_j + ny ty_j)),  rho(r, +-nz) = S (P -+ i Q)
//            -> 2 real FMA per particle x mode.
//   force    U0(r) = psi(r,0) + sum_{nz>0} (sig cos + i del sin),
//            U1(r) = sum_{nz>0} nz (del cos + i sig sin),  sig/del = psi(+nz) +- psi(-nz)
//            F += (nx Im(g U0), ny Im(g U0), Im(g U1)), g = exp(i (nx tx + ny ty))
//            -> 4 real FMA per particle x mode.
// Angles are t = x / L in turns; every anchor exp(2 pi i k t) is taken with
// sincospi on an exactly reduced k t, and runs of at most 8 powers in between
// use FP64 complex multiplication.

#include "sce_internal.h"
#include "sce_device.h"

namespace sce {

template <typename T> struct C2;
template <> struct C2<float> { typedef float2 t; };
template <> struct C2<double> { typedef double2 t; };

// ------------------------------------------------------------------ phase table
// exy[j][d][k] = cis(2 pi k t_d) for d = x, y and k = 0..n in FP64 (anchors of
// the deposit's row recurrences); tz[j][k] = (cos, sin)(2 pi k t_z) in the
// working precision for k = 0..n, zeros up to zslots.
template <typename T>
__global__ void __launch_bounds__(256)
k_phase_table(const double *__restrict__ pos, int64_t N, int n, int zslots, double invL,
              double2 *__restrict__ exy, T *__restrict__ tz)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int n1 = n + 1;
    for (int d = 0; d < 3; ++d) {
        const double t = frac(pos[d * N + j] * invL);
        double c1, s1;
        cis_turns(t, c1, s1);
        double c = 1.0, s = 0.0;
        const int kend = d < 2 ? n1 : zslots;
        for (int k = 0; k < kend; ++k) {
            if (k > n) {
                c = 0.0;
                s = 0.0;
            } else if (k > 0 && (k & 7) == 0) {
                cis_turns(frac_mul(k, t), c, s);
            }
            if (d < 2) {
                exy[(j * 2 + d) * n1 + k] = make_double2(c, s);
            } else {
                tz[(j * zslots + k) * 2] = (T)c;
                tz[(j * zslots + k) * 2 + 1] = (T)s;
            }
            const double cn = c * c1 - s * s1;
            s = s * c1 + c * s1;
            c = cn;
        }
    }
}

template <typename T>
hipError_t launch_phase_table(hipStream_t s, const double *pos, int64_t N, const Geom &g,
                              double L, double2 *exy, T *tz)
{
    const int64_t blocks = (N + 255) / 256;
    hipLaunchKernelGGL(k_phase_table<T>, dim3((unsigned)blocks), dim3(256), 0, s, pos, N, g.n,
                       g.zslots, 1.0 / L, exy, tz);
    return hipGetLastError();
}

// ------------------------------------------------------------------ deposit
// Block = 4 waves.  A wave owns 64 rows (one per lane) and one group of ZB
// n_z values; waves of a block share their rows' h values, generated per chunk
// of kc particles into LDS.  The per-particle cos/sin of the wave's n_z group
// are wave-uniform: scalar loads, double-buffered so that the next particle's
// values arrive while the current particle's FMAs issue.  blockIdx.z selects
// the particle split whose partial sums the block writes.

template <typename T, int ZB>
__device__ __forceinline__ void load_cs(T (&c)[2 * ZB], const T *__restrict__ p)
{
#pragma unroll
    for (int k = 0; k < 2 * ZB; ++k) c[k] = p[k];
}

template <typename T, int ZB, typename CT>
__device__ __forceinline__ void fma_cs(const T (&c)[2 * ZB], CT h, T (&aP)[ZB][2], T (&aQ)[ZB][2])
{
#pragma unroll
    for (int k = 0; k < ZB; ++k) {
        aP[k][0] = fma(h.x, c[2 * k], aP[k][0]);
        aP[k][1] = fma(h.y, c[2 * k], aP[k][1]);
        aQ[k][0] = fma(h.x, c[2 * k + 1], aQ[k][0]);
        aQ[k][1] = fma(h.y, c[2 * k + 1], aQ[k][1]);
    }
}

// One LDS chunk for one lane: cnt particles, h from LDS (stride rows), the
// z-table rows from zt (stride zs2).  G0: this wave also sums n_z = 0.
// Software-pipelined: the loads of particle j+1 (LDS h and the scalar z row)
// are issued before the FMAs of particle j, which use registers only; past
// the end of the chunk h is zero (and the z row a valid duplicate), so the
// extra step adds nothing.
template <typename T, int ZB, bool G0, typename CT>
__device__ __forceinline__ void dep_chunk(const CT *__restrict__ hrow, int rows, const T *__restrict__ zt,
                                          int zs2, int cnt, T (&aP)[ZB][2], T (&aQ)[ZB][2],
                                          T &a0r, T &a0i)
{
    if constexpr (sizeof(T) * ZB <= 32) {
        T cA[2 * ZB], cB[2 * ZB];
        CT hA, hB;
        load_cs<T, ZB>(cA, zt);
        hA = hrow[0];
        for (int jj = 0; jj < cnt; jj += 2) {
            const int j1 = jj + 1 < cnt ? jj + 1 : cnt - 1;
            load_cs<T, ZB>(cB, zt + (int64_t)j1 * zs2);
            hB = hrow[j1 * rows];
            if (jj + 1 >= cnt) {
                hB.x = (T)0;
                hB.y = (T)0;
            }
            fma_cs<T, ZB>(cA, hA, aP, aQ);
            if (G0) {
                a0r += hA.x;
                a0i += hA.y;
            }
            const int j2 = jj + 2 < cnt ? jj + 2 : cnt - 1;
            load_cs<T, ZB>(cA, zt + (int64_t)j2 * zs2);
            hA = hrow[j2 * rows];
            fma_cs<T, ZB>(cB, hB, aP, aQ);
            if (G0) {
                a0r += hB.x;
                a0i += hB.y;
            }
        }
    } else {
        // wide rows (FP64 x 8): one z row in scalar registers at a time
        CT hA = hrow[0];
        for (int jj = 0; jj < cnt; ++jj) {
            T c[2 * ZB];
            load_cs<T, ZB>(c, zt + (int64_t)jj * zs2);
            const int j1 = jj + 1 < cnt ? jj + 1 : jj;
            const CT hB = hrow[j1 * rows];
            fma_cs<T, ZB>(c, hA, aP, aQ);
            if (G0) {
                a0r += hA.x;
                a0i += hA.y;
            }
            hA = hB;
        }
    }
}

template <typename T, int ZB>
__global__ void __launch_bounds__(256)
k_deposit(const double2 *__restrict__ exy, const T *__restrict__ tz, const double *__restrict__ q,
          int64_t N, int n, int R, int Rpad, int zslots, int groups, int waves_per_rs,
          int rows_per_wg, int kc, int64_t per_split, double *__restrict__ part)
{
    typedef typename C2<T>::t CT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    CT *hs = reinterpret_cast<CT *>(smem_raw);

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int rs = wave / waves_per_rs;
    const int group = blockIdx.y * waves_per_rs + (wave - rs * waves_per_rs);
    const bool active = (rs * 64 < rows_per_wg) && (group < groups);
    const int row_local = rs * 64 + lane;
    const int row = blockIdx.x * rows_per_wg + row_local;
    const int64_t j0 = (int64_t)blockIdx.z * per_split;
    const int64_t j1 = j0 + per_split < N ? j0 + per_split : N;
    const int z0 = 1 + group * ZB;
    const int n1 = n + 1;
    const int zs2 = 2 * zslots;
    // h generation: each thread fills seg consecutive rows of one particle
    const int seg = kc * rows_per_wg / 256;
    const int segs_per_particle = rows_per_wg / seg;
    const int g_jj = tid / segs_per_particle;
    const int g_rl0 = (tid - g_jj * segs_per_particle) * seg;

    T aP[ZB][2], aQ[ZB][2];
#pragma unroll
    for (int k = 0; k < ZB; ++k) aP[k][0] = aP[k][1] = aQ[k][0] = aQ[k][1] = (T)0;
    T a0r = 0, a0i = 0;
    // FP32 sums run over one LDS chunk (<= kc particles) and are then added
    // into FP64 totals; a long FP32 running sum over coherent (lattice-like)
    // terms would lose digits to its own growth.
    constexpr bool kFlush = sizeof(T) < sizeof(double);
    double dP[kFlush ? ZB : 1][2], dQ[kFlush ? ZB : 1][2], d0r = 0.0, d0i = 0.0;
    if (kFlush) {
#pragma unroll
        for (int k = 0; k < (kFlush ? ZB : 1); ++k) dP[k][0] = dP[k][1] = dQ[k][0] = dQ[k][1] = 0.0;
    }

    for (int64_t base = j0; base < j1; base += kc) {
        const int cnt = (int)((j1 - base) < kc ? (j1 - base) : kc);
        {
            // h(r) = q exp(-i(nx tx + ny ty)) for seg rows: anchor from the FP64
            // axis tables, then steps of exp(-i ty) along n_y (FP64).
            int r = blockIdx.x * rows_per_wg + g_rl0;
            CT *dst = hs + g_jj * rows_per_wg + g_rl0;
            if (g_jj < cnt) {
                const int64_t j = base + g_jj;
                const double2 *ex = exy + j * 2 * n1;
                const double2 *ey = ex + n1;
                const double qq = q[j];
                const double2 e1 = ey[1];
                int nx, ny;
                row_nxny(r < R ? r : R - 1, n, nx, ny);
                double hc = 0.0, hs_ = 0.0;
                bool fresh = true;
                for (int s = 0; s < seg; ++s, ++r) {
                    if (r >= R) {
                        dst[s].x = (T)0;
                        dst[s].y = (T)0;
                        continue;
                    }
                    if (fresh) {
                        // exp(-i nx tx) * exp(-i ny ty)
                        const double2 a = ex[nx];
                        const int ay = ny < 0 ? -ny : ny;
                        const double2 b = ey[ay];
                        const double bs = ny < 0 ? b.y : -b.y;
                        const double as = -a.y;
                        hc = qq * (a.x * b.x - as * bs);
                        hs_ = qq * (a.x * bs + as * b.x);
                        fresh = false;
                    }
                    dst[s].x = (T)hc;
                    dst[s].y = (T)hs_;
                    if (ny < n) {
                        ++ny;
                        const double t = hc * e1.x + hs_ * e1.y;
                        hs_ = hs_ * e1.x - hc * e1.y;
                        hc = t;
                    } else {
                        ++nx;
                        ny = -n;
                        fresh = true;
                    }
                }
            } else {
                for (int s = 0; s < seg; ++s) {
                    dst[s].x = (T)0;
                    dst[s].y = (T)0;
                }
            }
        }
        __syncthreads();
        if (active) {
            const CT *hrow = hs + row_local;
            const T *zt = tz + base * zs2 + 2 * z0;
            if (group == 0)
                dep_chunk<T, ZB, true>(hrow, rows_per_wg, zt, zs2, cnt, aP, aQ, a0r, a0i);
            else
                dep_chunk<T, ZB, false>(hrow, rows_per_wg, zt, zs2, cnt, aP, aQ, a0r, a0i);
            if (kFlush) {
#pragma unroll
                for (int k = 0; k < (kFlush ? ZB : 1); ++k) {
                    dP[k][0] += (double)aP[k][0];
                    dP[k][1] += (double)aP[k][1];
                    dQ[k][0] += (double)aQ[k][0];
                    dQ[k][1] += (double)aQ[k][1];
                    aP[k][0] = aP[k][1] = aQ[k][0] = aQ[k][1] = (T)0;
                }
                d0r += (double)a0r;
                d0i += (double)a0i;
                a0r = a0i = (T)0;
            }
        }
        __syncthreads();
    }

    if (active && row < R) {
        double *pb = part + (int64_t)blockIdx.z * (int64_t)n1 * 4 * Rpad + row;
#pragma unroll
        for (int k = 0; k < ZB; ++k) {
            const int nz = z0 + k;
            if (nz <= n) {
                const int kk = kFlush ? k : 0;
                pb[(int64_t)(nz * 4 + 0) * Rpad] = kFlush ? dP[kk][0] : (double)aP[k][0];
                pb[(int64_t)(nz * 4 + 1) * Rpad] = kFlush ? dP[kk][1] : (double)aP[k][1];
                pb[(int64_t)(nz * 4 + 2) * Rpad] = kFlush ? dQ[kk][0] : (double)aQ[k][0];
                pb[(int64_t)(nz * 4 + 3) * Rpad] = kFlush ? dQ[kk][1] : (double)aQ[k][1];
            }
        }
        if (group == 0) {
            pb[0] = kFlush ? d0r : (double)a0r;
            pb[(int64_t)Rpad] = kFlush ? d0i : (double)a0i;
            pb[(int64_t)2 * Rpad] = 0.0;
            pb[(int64_t)3 * Rpad] = 0.0;
        }
    }
}

DepositPlan plan_deposit(const Geom &g, int64_t N, int elem_bytes)
{
    DepositPlan p;
    p.zb = g.n <= 4 ? 4 : 8;
    p.groups = (g.n + p.zb - 1) / p.zb;
    p.waves_per_rs = p.groups < 4 ? p.groups : 4;
    const int rowsets = 4 / p.waves_per_rs;
    p.rows_per_wg = 64 * rowsets;
    p.grid_y = (p.groups + p.waves_per_rs - 1) / p.waves_per_rs;
    p.row_blocks = (g.R + p.rows_per_wg - 1) / p.rows_per_wg;
    // LDS chunk: keep the h tile at 32 KiB
    p.kc = (32768 / elem_bytes / 2) / p.rows_per_wg;
    if (p.kc < 4) p.kc = 4;
    // Splits: enough blocks to fill the CUs several times over, at least 256
    // particles per split, and a block count that fills whole rounds of
    // resident blocks (a nearly empty last round costs a full round).
    const int64_t blocks_per_split = (int64_t)p.row_blocks * p.grid_y;
    int64_t max_splits = N / 256 > 1 ? N / 256 : 1;
    if (max_splits > 1024) max_splits = 1024;
    int dev = 0, cus = 256, per_cu = 0;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const size_t shmem = (size_t)p.kc * p.rows_per_wg * 2 * elem_bytes;
    const void *kf = elem_bytes == 8
                         ? (p.zb == 4 ? (const void *)k_deposit<double, 4> : (const void *)k_deposit<double, 8>)
                         : (p.zb == 4 ? (const void *)k_deposit<float, 4> : (const void *)k_deposit<float, 8>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kf, 256, shmem) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (cus < 1) cus = 256;
    const int64_t slots = (int64_t)cus * per_cu;
    int64_t splits = 1;
    double best = 1e300;
    for (int64_t sp = 1; sp <= max_splits; ++sp) {
        const int64_t blocks = blocks_per_split * sp;
        if (blocks < 2 * slots && sp < max_splits) continue;  // at least two rounds when possible
        const double cost = (double)((blocks + slots - 1) / slots) / (double)sp;
        if (cost < best * (1.0 - 1e-9)) {
            best = cost;
            splits = sp;
        }
    }
    int64_t per = (N + splits - 1) / splits;
    per = (per + p.kc - 1) / p.kc * p.kc;
    p.per_split = per;
    p.splits = (int)((N + per - 1) / per);
    return p;
}

template <typename T>
hipError_t launch_deposit(hipStream_t s, const double2 *exy, const T *tz, const double *q, int64_t N,
                          const Geom &g, const DepositPlan &pl, double *part)
{
    typedef typename C2<T>::t CT;
    const size_t shmem = (size_t)pl.kc * pl.rows_per_wg * sizeof(CT);
    dim3 grid((unsigned)pl.row_blocks, (unsigned)pl.grid_y, (unsigned)pl.splits);
    if (pl.zb == 4)
        hipLaunchKernelGGL((k_deposit<T, 4>), grid, dim3(256), shmem, s, exy, tz, q, N, g.n, g.R,
                           g.Rpad, g.zslots, pl.groups, pl.waves_per_rs, pl.rows_per_wg, pl.kc,
                           pl.per_split, part);
    else
        hipLaunchKernelGGL((k_deposit<T, 8>), grid, dim3(256), shmem, s, exy, tz, q, N, g.n, g.R,
                           g.Rpad, g.zslots, pl.groups, pl.waves_per_rs, pl.rows_per_wg, pl.kc,
                           pl.per_split, part);
    return hipGetLastError();
}

// ------------------------------------------------------------------ reduce + solve
__device__ inline double block_sum(double v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    __syncthreads();
    return t;
}

__device__ inline double block_max(double v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t = fmax(t, sh[i]);
    __syncthreads();
    return t;
}

// A block covers 64 cells (row, n_z) with kReduceWays waves: wave p sums the
// splits p, p + kReduceWays, ... of each of its lane's cell (the reads of a
// wave are 64 consecutive rows), and the ways are then added in a fixed order
// through LDS, so the result does not depend on scheduling.  One thread per
// cell and all splits in one loop left most compute units idle at n_max = 16
// (37 blocks) while the loop streamed the partials.
constexpr int kReduceWays = 8;
constexpr int kReduceUnroll = 4;

template <typename T, typename P>
__global__ void __launch_bounds__(64 * kReduceWays)
k_reduce_solve(const P *__restrict__ part, int splits, int n, int R, int Rpad, int nzp,
               const double *__restrict__ Stab, const double *__restrict__ Gtab,
               const double *__restrict__ Ktab, double2 *__restrict__ rho,
               double2 *__restrict__ psi, T *__restrict__ ftab, T *__restrict__ psi0,
               double *__restrict__ wpart)
{
    __shared__ double4 ways[kReduceWays][64];
    const int n1 = n + 1, M = 2 * n + 1;
    const int lane = threadIdx.x & 63, way = threadIdx.x >> 6;
    const int64_t cell = (int64_t)blockIdx.x * 64 + lane;
    const bool valid = cell < (int64_t)n1 * R;
    {
        double Pr = 0.0, Pi = 0.0, Qr = 0.0, Qi = 0.0;
        if (valid) {
            const int nz = (int)(cell / R);
            const int row = (int)(cell - (int64_t)nz * R);
            const int64_t sstride = (int64_t)n1 * 4 * Rpad;
            const P *pp = part + (int64_t)way * sstride + (int64_t)nz * 4 * Rpad + row;
            // kReduceUnroll splits' values are loaded before any is added, so
            // their loads are in flight together; the additions keep the
            // split order
            int sp = way;
            for (; sp + (kReduceUnroll - 1) * kReduceWays < splits;
                 sp += kReduceUnroll * kReduceWays, pp += kReduceUnroll * kReduceWays * sstride) {
                P v[kReduceUnroll][4];
#pragma unroll
                for (int u = 0; u < kReduceUnroll; ++u) {
                    const P *qq = pp + (int64_t)u * kReduceWays * sstride;
                    v[u][0] = qq[0];
                    v[u][1] = qq[Rpad];
                    v[u][2] = qq[2 * (int64_t)Rpad];
                    v[u][3] = qq[3 * (int64_t)Rpad];
                }
#pragma unroll
                for (int u = 0; u < kReduceUnroll; ++u) {
                    Pr += (double)v[u][0];
                    Pi += (double)v[u][1];
                    Qr += (double)v[u][2];
                    Qi += (double)v[u][3];
                }
            }
            for (; sp < splits; sp += kReduceWays, pp += kReduceWays * sstride) {
                Pr += (double)pp[0];
                Pi += (double)pp[Rpad];
                Qr += (double)pp[2 * (int64_t)Rpad];
                Qi += (double)pp[3 * (int64_t)Rpad];
            }
        }
        ways[way][lane] = make_double4(Pr, Pi, Qr, Qi);
    }
    __syncthreads();
    if (way != 0) return;
    double w = 0.0, amax = 0.0;
    if (valid) {
        const int nz = (int)(cell / R);
        const int row = (int)(cell - (int64_t)nz * R);
        double Pr = 0.0, Pi = 0.0, Qr = 0.0, Qi = 0.0;
        for (int p = 0; p < kReduceWays; ++p) {
            const double4 v = ways[p][lane];
            Pr += v.x;
            Pi += v.y;
            Qr += v.z;
            Qi += v.w;
        }
        int nx, ny;
        row_nxny(row, n, nx, ny);
        const int64_t ti = (int64_t)nz * R + row;  // tables are [n_z][row]: consecutive lanes, consecutive rows
        const double S = Stab[ti], G = Gtab[ti], K = Ktab[ti];
        const double2 rp = make_double2(S * (Pr + Qi), S * (Pi - Qr));
        const double2 rm = make_double2(S * (Pr - Qi), S * (Pi + Qr));
        const bool hp = in_half(nx, ny, nz);
        const bool hm = nz > 0 && in_half(nx, ny, -nz);
        const double2 pp_ = hp ? make_double2(G * rp.x, G * rp.y) : make_double2(0.0, 0.0);
        const double2 pm_ = hm ? make_double2(G * rm.x, G * rm.y) : make_double2(0.0, 0.0);
        const int64_t rb = (int64_t)row * M + n;
        rho[rb + nz] = rp;
        psi[rb + nz] = pp_;
        if (nz > 0) {
            rho[rb - nz] = rm;
            psi[rb - nz] = pm_;
        }
        if (hp) {
            w += K * (rp.x * rp.x + rp.y * rp.y);
            amax = fmax(amax, sqrt(rp.x * rp.x + rp.y * rp.y));
        }
        if (hm) {
            w += K * (rm.x * rm.x + rm.y * rm.y);
            amax = fmax(amax, sqrt(rm.x * rm.x + rm.y * rm.y));
        }
        if (nz == 0) {
            psi0[2 * row] = (T)pp_.x;
            psi0[2 * row + 1] = (T)pp_.y;
        } else {
            T *f = ftab + ((int64_t)row * nzp + (nz - 1)) * 8;
            const double sr = pp_.x + pm_.x, si = pp_.y + pm_.y;
            const double dr = pp_.x - pm_.x, di = pp_.y - pm_.y;
            f[0] = (T)sr;
            f[1] = (T)si;
            f[2] = (T)dr;
            f[3] = (T)di;
            f[4] = (T)(nz * dr);
            f[5] = (T)(nz * di);
            f[6] = (T)(nz * sr);
            f[7] = (T)(nz * si);
        }
    }
    // the block's W and max|rho| over its 64 cells (one wave, fixed order)
    for (int o = 32; o > 0; o >>= 1) {
        w += __shfl_xor(w, o, 64);
        amax = fmax(amax, __shfl_xor(amax, o, 64));
    }
    if (lane == 0) {
        wpart[2 * blockIdx.x] = w;
        wpart[2 * blockIdx.x + 1] = amax;
    }
}

template <typename T, typename P>
hipError_t launch_reduce_solve(hipStream_t s, const P *part, int splits, const Geom &g,
                               const double *Stab, const double *Gtab, const double *Ktab,
                               double2 *rho, double2 *psi, T *ftab, T *psi0, double *wpart,
                               int *wblocks)
{
    const int64_t cells = (int64_t)(g.n + 1) * g.R;
    const int blocks = (int)((cells + 63) / 64);
    *wblocks = blocks;
    hipLaunchKernelGGL((k_reduce_solve<T, P>), dim3(blocks), dim3(64 * kReduceWays), 0, s, part, splits, g.n, g.R,
                       g.Rpad, g.nzp, Stab, Gtab, Ktab, rho, psi, ftab, psi0, wpart);
    return hipGetLastError();
}

// ------------------------------------------------------------------ force
// The sums of one lane's particle over the rows of the n_x lines [l0, l1)
// (r0: the row index of line l0's first row): fx, fy, fz, ph before the
// factor 2 q (2 pi / L).
template <typename T, int NZC>
__device__ __forceinline__ void force_line_sums(const T *__restrict__ ftab, const T *__restrict__ psi0,
                                                int n, int nzp, int l0, int l1, int r0, double tx,
                                                double ty, double tz, double &fx, double &fy,
                                                double &fz, double &ph)
{
    double eyc, eys;
    cis_turns(ty, eyc, eys);
    double ezc, ezs;
    cis_turns(tz, ezc, ezs);
    for (int c0 = 0; c0 < nzp; c0 += NZC) {
        T cz[NZC], sz[NZC];
        {
            double c, s;
#pragma unroll
            for (int k = 0; k < NZC; ++k) {
                if ((k & 7) == 0) {
                    cis_turns(frac_mul(c0 + 1 + k, tz), c, s);
                } else {
                    const double cn = c * ezc - s * ezs;
                    s = s * ezc + c * ezs;
                    c = cn;
                }
                cz[k] = (T)c;
                sz[k] = (T)s;
            }
        }
        int r = r0;
        for (int nx = l0; nx < l1; ++nx) {
            const int ny0 = nx == 0 ? 0 : -n;
            double hc, hs;
            cis_turns(frac_lin(nx, tx, ny0, ty), hc, hs);
            for (int ny = ny0; ny <= n; ++ny, ++r) {
                const T *ft = ftab + ((int64_t)r * nzp + c0) * 8;
                T u0r = (T)0, u0i = (T)0, u1r = (T)0, u1i = (T)0;
                if (c0 == 0) {
                    u0r = psi0[2 * r];
                    u0i = psi0[2 * r + 1];
                }
#pragma unroll
                for (int k = 0; k < NZC; ++k) {
                    const T c = cz[k], s = sz[k];
                    u0r = fma(ft[8 * k + 0], c, u0r);
                    u0i = fma(ft[8 * k + 1], c, u0i);
                    u0r = fma(-ft[8 * k + 3], s, u0r);
                    u0i = fma(ft[8 * k + 2], s, u0i);
                    u1r = fma(ft[8 * k + 4], c, u1r);
                    u1i = fma(ft[8 * k + 5], c, u1i);
                    u1r = fma(-ft[8 * k + 7], s, u1r);
                    u1i = fma(ft[8 * k + 6], s, u1i);
                }
                const double im0 = hc * (double)u0i + hs * (double)u0r;
                const double re0 = hc * (double)u0r - hs * (double)u0i;
                const double im1 = hc * (double)u1i + hs * (double)u1r;
                fx = fma((double)nx, im0, fx);
                fy = fma((double)ny, im0, fy);
                fz += im1;
                ph += re0;
                const double t = hc * eyc - hs * eys;
                hs = hs * eyc + hc * eys;
                hc = t;
            }
        }
    }
}

// One particle per lane.  Rows are visited in the same order by every lane,
// so the force table entries of a row are wave-uniform (scalar loads); the
// lane's cos/sin(n_z tz) for a chunk of NZC values stay in registers.  PLANE:
// a two-dimensional context (rows of n_x = 0 only).  The number of n_x lines
// is a compile-time choice on purpose: the row loop is bound by the latency
// of the table's scalar loads, which the compiler hides by double-buffering
// them in SGPRs, and one more live scalar (a runtime line count) leaves no
// room for the second buffer (measured: FP64 force 37 -> 55 ms at 2^20
// particles, n_max = 32).
template <typename T, int NZC, bool PLANE>
__global__ void __launch_bounds__(256)
k_force(const double *__restrict__ pos, const double *__restrict__ q,
        const double *__restrict__ m, double *__restrict__ vel, const T *__restrict__ ftab,
        const T *__restrict__ psi0, int n, int nzp, double invL, int64_t N,
        double kick, double *__restrict__ F, double *__restrict__ phi)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t jc = j < N ? j : N - 1;
    const double tx = frac(pos[jc] * invL);
    const double ty = frac(pos[N + jc] * invL);
    const double tz = frac(pos[2 * N + jc] * invL);
    double fx = 0.0, fy = 0.0, fz = 0.0, ph = 0.0;
    force_line_sums<T, NZC>(ftab, psi0, n, nzp, 0, PLANE ? 1 : n + 1, 0, tx, ty, tz, fx, fy, fz, ph);
    if (j < N) {
        const double f = 2.0 * q[j] * (6.283185307179586476925286766559 * invL);
        fx *= f;
        fy *= f;
        fz *= f;
        if (F) {
            F[j] = fx;
            F[N + j] = fy;
            F[2 * N + j] = fz;
        }
        if (phi) phi[j] = 2.0 * ph;
        if (kick != 0.0) {
            const double a = kick / m[j];
            vel[j] += a * fx;
            vel[N + j] += a * fy;
            vel[2 * N + j] += a * fz;
        }
    }
}

// Medium particle counts (too few blocks of 256 particles to fill the compute
// units): blockIdx.y takes the rows [y R / S, (y + 1) R / S), S = gridDim.y,
// and writes its raw sums to part[y][4][N] (fx, fy, fz, ph); k_force_combine
// adds the S row groups in order, scales and kicks.  A group's rows are whole
// n_x lines except possibly its first and last (clipped in n_y); the row phase
// is anchored with its own FP64 exponential at the start of each line and
// follows the recurrence along n_y, as in the one-particle-per-lane kernel.
// FP64: four waves per SIMD, since the grid is sized for one round of four
// blocks per compute unit and at 129 registers the kernel would need two.
template <typename T, int NZC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 4 : 1)))
k_force_lines(const double *__restrict__ pos, const T *__restrict__ ftab,
              const T *__restrict__ psi0, int n, int R, int nzp, double invL, int64_t N,
              double *__restrict__ part)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t jc = j < N ? j : N - 1;
    const int S = gridDim.y, y = blockIdx.y;
    const int r0 = (int)((int64_t)y * R / S), r1 = (int)((int64_t)(y + 1) * R / S);
    const double tx = frac(pos[jc] * invL);
    const double ty = frac(pos[N + jc] * invL);
    const double tz = frac(pos[2 * N + jc] * invL);
    double eyc, eys;
    cis_turns(ty, eyc, eys);
    double ezc, ezs;
    cis_turns(tz, ezc, ezs);
    double fx = 0.0, fy = 0.0, fz = 0.0, ph = 0.0;
    for (int c0 = 0; c0 < nzp; c0 += NZC) {
        T cz[NZC], sz[NZC];
        {
            double c, s;
#pragma unroll
            for (int k = 0; k < NZC; ++k) {
                if ((k & 7) == 0) {
                    cis_turns(frac_mul(c0 + 1 + k, tz), c, s);
                } else {
                    const double cn = c * ezc - s * ezs;
                    s = s * ezc + c * ezs;
                    c = cn;
                }
                cz[k] = (T)c;
                sz[k] = (T)s;
            }
        }
        // rows r0 .. r1-1: lines l0 .. l1, the first from n_y = ys, the last to n_y = ye
        int l0, ys, l1, ye;
        row_nxny(r0, n, l0, ys);
        row_nxny(r1 - 1, n, l1, ye);
        int r = r0;
        for (int nx = l0; nx <= l1; ++nx) {
            const int ny0 = nx == l0 ? ys : (nx == 0 ? 0 : -n);
            const int ny1 = nx == l1 ? ye : n;
            double hc, hs;
            cis_turns(frac_lin(nx, tx, ny0, ty), hc, hs);
            for (int ny = ny0; ny <= ny1; ++ny, ++r) {
                const T *ft = ftab + ((int64_t)r * nzp + c0) * 8;
                T u0r = (T)0, u0i = (T)0, u1r = (T)0, u1i = (T)0;
                if (c0 == 0) {
                    u0r = psi0[2 * r];
                    u0i = psi0[2 * r + 1];
                }
#pragma unroll
                for (int k = 0; k < NZC; ++k) {
                    const T c = cz[k], s = sz[k];
                    u0r = fma(ft[8 * k + 0], c, u0r);
                    u0i = fma(ft[8 * k + 1], c, u0i);
                    u0r = fma(-ft[8 * k + 3], s, u0r);
                    u0i = fma(ft[8 * k + 2], s, u0i);
                    u1r = fma(ft[8 * k + 4], c, u1r);
                    u1i = fma(ft[8 * k + 5], c, u1i);
                    u1r = fma(-ft[8 * k + 7], s, u1r);
                    u1i = fma(ft[8 * k + 6], s, u1i);
                }
                const double im0 = hc * (double)u0i + hs * (double)u0r;
                const double re0 = hc * (double)u0r - hs * (double)u0i;
                const double im1 = hc * (double)u1i + hs * (double)u1r;
                fx = fma((double)nx, im0, fx);
                fy = fma((double)ny, im0, fy);
                fz += im1;
                ph += re0;
                const double t = hc * eyc - hs * eys;
                hs = hs * eyc + hc * eys;
                hc = t;
            }
        }
    }
    if (j < N) {
        double *o = part + (int64_t)y * 4 * N + j;
        o[0] = fx;
        o[N] = fy;
        o[2 * N] = fz;
        o[3 * N] = ph;
    }
}

__global__ void __launch_bounds__(256)
k_force_combine(const double *__restrict__ part, int S, const double *__restrict__ q,
                const double *__restrict__ m, double *__restrict__ vel, int64_t N, double invL,
                double kick, double *__restrict__ F, double *__restrict__ phi)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    double fx = 0.0, fy = 0.0, fz = 0.0, ph = 0.0;
    for (int y = 0; y < S; ++y) {
        const double *o = part + (int64_t)y * 4 * N + j;
        fx += o[0];
        fy += o[N];
        fz += o[2 * N];
        ph += o[3 * N];
    }
    const double f = 2.0 * q[j] * (6.283185307179586476925286766559 * invL);
    fx *= f;
    fy *= f;
    fz *= f;
    if (F) {
        F[j] = fx;
        F[N + j] = fy;
        F[2 * N + j] = fz;
    }
    if (phi) phi[j] = 2.0 * ph;
    if (kick != 0.0) {
        const double a = kick / m[j];
        vel[j] += a * fx;
        vel[N + j] += a * fy;
        vel[2 * N + j] += a * fz;
    }
}

// Small particle counts: one block of 256 threads per particle, the rows split
// across the threads (thread t takes rows t, t + 256, ...), so that a step of a
// handful of particles is not one serial mode sum per particle.  The
// particle's cos/sin(n_z tz), n_z = 1..n, are formed once per block in LDS,
// each from its own FP64 anchor; each row's phase exp(2 pi i (n_x tx + n_y ty))
// is an FP64 anchor too.  The threads' FP64 sums are combined in a fixed
// order, so the result does not depend on scheduling.  Up to these counts it
// is faster than one particle per lane, which leaves most compute units idle
// below a few hundred blocks (measured crossover between 8K and 16K particles
// in FP32, above 16K in FP64, for n_max 8 to 32).
template <typename T> constexpr int64_t force_small_max() { return sizeof(T) == 8 ? 16384 : 8192; }

template <typename T>
__global__ void __launch_bounds__(256)
k_force_small(const double *__restrict__ pos, const double *__restrict__ q,
              const double *__restrict__ m, double *__restrict__ vel, const T *__restrict__ ftab,
              const T *__restrict__ psi0, int n, int R, int nzp, double invL, int64_t N,
              double kick, double *__restrict__ F, double *__restrict__ phi)
{
    __shared__ T csz[2][64];  // cos, sin(n_z tz) for n_z = 1..n (n <= 64)
    __shared__ double red[4][256];
    const int64_t j = blockIdx.x;
    const int t = threadIdx.x;
    const double tx = frac(pos[j] * invL);
    const double ty = frac(pos[N + j] * invL);
    const double tz = frac(pos[2 * N + j] * invL);
    if (t < n) {
        double c, sn;
        cis_turns(frac_mul(t + 1, tz), c, sn);
        csz[0][t] = (T)c;
        csz[1][t] = (T)sn;
    }
    __syncthreads();
    double fx = 0.0, fy = 0.0, fz = 0.0, ph = 0.0;
    for (int r = t; r < R; r += 256) {
        int nx, ny;
        row_nxny(r, n, nx, ny);
        double hc, hs;
        cis_turns(frac_lin(nx, tx, ny, ty), hc, hs);
        const T *ft = ftab + (int64_t)r * nzp * 8;
        double U0r = (double)psi0[2 * r], U0i = (double)psi0[2 * r + 1], U1r = 0.0, U1i = 0.0;
        // Sums over n_z in chunks of 16 in T, each chunk added in FP64.
        for (int k0 = 0; k0 < n; k0 += 16) {
            const int k1 = k0 + 16 < n ? k0 + 16 : n;
            T u0r = (T)0, u0i = (T)0, u1r = (T)0, u1i = (T)0;
            for (int k = k0; k < k1; ++k) {
                const T c = csz[0][k], sn = csz[1][k];
                u0r = fma(ft[8 * k + 0], c, u0r);
                u0i = fma(ft[8 * k + 1], c, u0i);
                u0r = fma(-ft[8 * k + 3], sn, u0r);
                u0i = fma(ft[8 * k + 2], sn, u0i);
                u1r = fma(ft[8 * k + 4], c, u1r);
                u1i = fma(ft[8 * k + 5], c, u1i);
                u1r = fma(-ft[8 * k + 7], sn, u1r);
                u1i = fma(ft[8 * k + 6], sn, u1i);
            }
            U0r += (double)u0r;
            U0i += (double)u0i;
            U1r += (double)u1r;
            U1i += (double)u1i;
        }
        const double im0 = hc * U0i + hs * U0r;
        const double re0 = hc * U0r - hs * U0i;
        const double im1 = hc * U1i + hs * U1r;
        fx = fma((double)nx, im0, fx);
        fy = fma((double)ny, im0, fy);
        fz += im1;
        ph += re0;
    }
    red[0][t] = fx;
    red[1][t] = fy;
    red[2][t] = fz;
    red[3][t] = ph;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int e = 0; e < 4; ++e) red[e][t] += red[e][t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        const double f = 2.0 * q[j] * (6.283185307179586476925286766559 * invL);
        const double Fx = f * red[0][0], Fy = f * red[1][0], Fz = f * red[2][0];
        if (F) {
            F[j] = Fx;
            F[N + j] = Fy;
            F[2 * N + j] = Fz;
        }
        if (phi) phi[j] = 2.0 * red[3][0];
        if (kick != 0.0) {
            const double a = kick / m[j];
            vel[j] += a * Fx;
            vel[N + j] += a * Fy;
            vel[2 * N + j] += a * Fz;
        }
    }
}

template <typename T, int NZC, bool PLANE>
hipError_t launch_force_chunk(hipStream_t s, const double *pos, const double *q, const double *m,
                              double *vel, const T *ftab, const T *psi0, const Geom &g, double L,
                              int64_t N, double kick, double *F, double *phi)
{
    const int64_t blocks = (N + 255) / 256;
    hipLaunchKernelGGL((k_force<T, NZC, PLANE>), dim3((unsigned)blocks), dim3(256), 0, s, pos, q, m,
                       vel, ftab, psi0, g.n, g.nzp, 1.0 / L, N, kick, F, phi);
    return hipGetLastError();
}

int force_line_groups(const Geom &g, int64_t N, int elem_bytes)
{
    if (N <= (elem_bytes == 8 ? force_small_max<double>() : force_small_max<float>())) return 1;
    const int64_t blocks = (N + 255) / 256;
    if (blocks >= kForceLineBlocks) return 1;
    const int64_t want = (kForceLineBlocks + blocks - 1) / blocks;
    return (int)(want < g.R / 8 ? want : g.R / 8);  // at least 8 rows per group
}

template <typename T, int NZC>
hipError_t launch_force_lines(hipStream_t s, const double *pos, const double *q, const double *m,
                              double *vel, const T *ftab, const T *psi0, const Geom &g, double L,
                              int64_t N, double kick, double *F, double *phi, int S, double *part)
{
    const int64_t blocks = (N + 255) / 256;
    hipLaunchKernelGGL((k_force_lines<T, NZC>), dim3((unsigned)blocks, (unsigned)S), dim3(256), 0, s, pos,
                       ftab, psi0, g.n, g.R, g.nzp, 1.0 / L, N, part);
    hipLaunchKernelGGL(k_force_combine, dim3((unsigned)blocks), dim3(256), 0, s, part, S, q, m, vel, N,
                       1.0 / L, kick, F, phi);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_force(hipStream_t s, const double *pos, const double *q, const double *m,
                        double *vel, const T *ftab, const T *psi0, const Geom &g, double L,
                        int64_t N, double kick, double *F, double *phi, double *part)
{
    if (N <= force_small_max<T>()) {
        hipLaunchKernelGGL(k_force_small<T>, dim3((unsigned)N), dim3(256), 0, s, pos, q, m, vel, ftab,
                           psi0, g.n, g.R, g.nzp, 1.0 / L, N, kick, F, phi);
        return hipGetLastError();
    }
    const int nzc = force_chunk(g.n, (int)sizeof(T));
    const int S = force_line_groups(g, N, (int)sizeof(T));
    if (S > 1) {
        if (!part) return hipErrorInvalidValue;
        if (nzc == 8) return launch_force_lines<T, 8>(s, pos, q, m, vel, ftab, psi0, g, L, N, kick, F, phi, S, part);
        if (nzc == 16 || sizeof(T) == 8) return launch_force_lines<T, 16>(s, pos, q, m, vel, ftab, psi0, g, L, N, kick, F, phi, S, part);
        if constexpr (sizeof(T) == 4) return launch_force_lines<T, 32>(s, pos, q, m, vel, ftab, psi0, g, L, N, kick, F, phi, S, part);
    }
    if (g.lines == 1) {
        if (nzc == 8) return launch_force_chunk<T, 8, true>(s, pos, q, m, vel, ftab, psi0, g, L, N, kick, F, phi);
        if (nzc == 16 || sizeof(T) == 8) return launch_force_chunk<T, 16, true>(s, pos, q, m, vel, ftab, psi0, g, L, N, kick, F, phi);
        if constexpr (sizeof(T) == 4) return launch_force_chunk<T, 32, true>(s, pos, q, m, vel, ftab, psi0, g, L, N, kick, F, phi);
    } else {
        if (nzc == 8) return launch_force_chunk<T, 8, false>(s, pos, q, m, vel, ftab, psi0, g, L, N, kick, F, phi);
        if (nzc == 16 || sizeof(T) == 8) return launch_force_chunk<T, 16, false>(s, pos, q, m, vel, ftab, psi0, g, L, N, kick, F, phi);
        if constexpr (sizeof(T) == 4) return launch_force_chunk<T, 32, false>(s, pos, q, m, vel, ftab, psi0, g, L, N, kick, F, phi);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ drift / kick
__global__ void __launch_bounds__(256)
k_kick_drift(double *__restrict__ pos, double *__restrict__ vel, const double *__restrict__ F,
             const double *__restrict__ m, int64_t N, double L, double invL, double a, double b,
             int wrap)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    const double am = a != 0.0 ? a / m[j] : 0.0;
    for (int d = 0; d < 3; ++d) {
        double v = vel[d * N + j];
        if (a != 0.0) {
            v += am * F[d * N + j];
            vel[d * N + j] = v;
        }
        if (b != 0.0) {
            const double x = pos[d * N + j] + b * v;
            pos[d * N + j] = wrap ? wrap_box(x, L, invL) : x;
        }
    }
}

hipError_t launch_kick_drift(hipStream_t s, double *pos, double *vel, const double *F,
                             const double *m, int64_t N, double L, double a, double b, bool wrap)
{
    const int64_t blocks = (N + 255) / 256;
    hipLaunchKernelGGL(k_kick_drift, dim3((unsigned)blocks), dim3(256), 0, s, pos, vel, F, m, N,
                       L, 1.0 / L, a, b, wrap ? 1 : 0);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256)
k_wrap(double *__restrict__ pos, int64_t n3, double L, double invL)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n3) pos[i] = wrap_box(pos[i], L, invL);
}

hipError_t launch_wrap(hipStream_t s, double *pos, int64_t N, double L)
{
    const int64_t blocks = (3 * N + 255) / 256;
    hipLaunchKernelGGL(k_wrap, dim3((unsigned)blocks), dim3(256), 0, s, pos, 3 * N, L, 1.0 / L);
    return hipGetLastError();
}

// Input check of a particle set: bit 0 of *flag for a non-finite position,
// velocity or charge, bit 1 for a mass that is not finite and > 0.  *flag
// must be zero before the launch.
__global__ void __launch_bounds__(256)
k_check_particles(const double *__restrict__ pos, const double *__restrict__ vel,
                  const double *__restrict__ q, const double *__restrict__ m, int64_t N,
                  unsigned *__restrict__ flag)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    unsigned bad = 0;
    if (j < N) {
        for (int d = 0; d < 3; ++d)
            bad |= (isfinite(pos[d * N + j]) && isfinite(vel[d * N + j])) ? 0u : 1u;
        bad |= isfinite(q[j]) ? 0u : 1u;
        bad |= (isfinite(m[j]) && m[j] > 0.0) ? 0u : 2u;
    }
    if (bad) atomicOr(flag, bad);
}

hipError_t launch_check_particles(hipStream_t s, const double *pos, const double *vel,
                                  const double *q, const double *m, int64_t N, unsigned *flag)
{
    const int64_t blocks = (N + 255) / 256;
    hipLaunchKernelGGL(k_check_particles, dim3((unsigned)blocks), dim3(256), 0, s, pos, vel, q, m,
                       N, flag);
    return hipGetLastError();
}

// ------------------------------------------------------------------ diagnostics
// scratch: [blocks][6] partial sums, written in block order.
__global__ void __launch_bounds__(256)
k_diag_partial(const double *__restrict__ vel, const double *__restrict__ q,
               const double *__restrict__ m, const double *__restrict__ phi, int64_t N,
               double *__restrict__ scratch)
{
    __shared__ double sh[8];
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (j < N) {
        const double vx = vel[j], vy = vel[N + j], vz = vel[2 * N + j], mm = m[j];
        const double v2 = vx * vx + vy * vy + vz * vz;
        v[0] = 0.5 * mm * v2;
        v[1] = mm * vx;
        v[2] = mm * vy;
        v[3] = mm * vz;
        v[4] = mm * sqrt(v2);
        v[5] = phi ? q[j] * phi[j] : 0.0;
    }
    for (int i = 0; i < 6; ++i) {
        const double t = block_sum(v[i], sh);
        if (threadIdx.x == 0) scratch[6 * blockIdx.x + i] = t;
    }
}

__global__ void __launch_bounds__(256)
k_diag_finish(const double *__restrict__ scratch, int nb, const double *__restrict__ wpart,
              int wb, double *__restrict__ out)
{
    __shared__ double sh[8];
    for (int i = 0; i < 6; ++i) {
        double t = 0.0;
        for (int b = threadIdx.x; b < nb; b += 256) t += scratch[6 * b + i];
        t = block_sum(t, sh);
        if (threadIdx.x == 0) out[i] = t;
    }
    double w = 0.0, mx = 0.0;
    for (int b = threadIdx.x; b < wb; b += 256) {
        w += wpart[2 * b];
        mx = fmax(mx, wpart[2 * b + 1]);
    }
    w = block_sum(w, sh);
    mx = block_max(mx, sh);
    if (threadIdx.x == 0) {
        out[6] = w;
        out[7] = mx;
    }
}

hipError_t launch_diag(hipStream_t s, const double *vel, const double *q, const double *m,
                       const double *phi, int64_t N, const double *wpart, int wblocks,
                       double eps0V, double *scratch, double *out)
{
    (void)eps0V;
    const int nb = (int)((N + 255) / 256);
    hipLaunchKernelGGL(k_diag_partial, dim3(nb), dim3(256), 0, s, vel, q, m, phi, N, scratch);
    hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(256), 0, s, scratch, nb, wpart, wblocks, out);
    return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_phase_table<float>(hipStream_t, const double *, int64_t, const Geom &, double, double2 *, float *);
template hipError_t launch_phase_table<double>(hipStream_t, const double *, int64_t, const Geom &, double, double2 *, double *);
template hipError_t launch_deposit<float>(hipStream_t, const double2 *, const float *, const double *, int64_t, const Geom &, const DepositPlan &, double *);
template hipError_t launch_deposit<double>(hipStream_t, const double2 *, const double *, const double *, int64_t, const Geom &, const DepositPlan &, double *);
template hipError_t launch_reduce_solve<float, double>(hipStream_t, const double *, int, const Geom &, const double *, const double *, const double *, double2 *, double2 *, float *, float *, double *, int *);
template hipError_t launch_reduce_solve<double, double>(hipStream_t, const double *, int, const Geom &, const double *, const double *, const double *, double2 *, double2 *, double *, double *, double *, int *);
template hipError_t launch_reduce_solve<float, float>(hipStream_t, const float *, int, const Geom &, const double *, const double *, const double *, double2 *, double2 *, float *, float *, double *, int *);
template hipError_t launch_force<float>(hipStream_t, const double *, const double *, const double *, double *, const float *, const float *, const Geom &, double, int64_t, double, double *, double *, double *);
template hipError_t launch_force<double>(hipStream_t, const double *, const double *, const double *, double *, const double *, const double *, const Geom &, double, int64_t, double, double *, double *, double *);

}  // namespace sce
