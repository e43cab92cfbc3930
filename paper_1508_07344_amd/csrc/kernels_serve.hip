// Batched kernels of the serving path (gfx950): one launch per phase advances
// every resident request by one pass (see sce_serve.h for the pass schedule).
//
// The sums are the same separable ones as the single-simulation direct path
// (Section 8: one exponential per axis, integer powers by multiplication, and
// the +n_z / -n_z modes of a row sharing cos and sin of n_z theta_z because
// the particle weights are real):
//   deposit  P(r, nz) = sum_j h_j(r) cos(nz tz_j),  Q(r, nz) = sum_j h_j(r) sin(nz tz_j),
//            h_j(r) = q_j exp(-i (nx tx_j + ny ty_j)),  rho(r, +-nz) = S (P -+ i Q)
//   force    F_j = 2 q_j (2 pi / L) (sum nx Im(g U0), sum ny Im(g U0), sum Im(g U1))
//            U0 = psi(r,0) + sum (sig cos + i del sin), U1 = sum nz (del cos + i sig sin)
// Every block serves one work item of one request; blocks of requests of
// different size run side by side in the same launch.  Kernels are templated
// on the working precision T (float: FP32 phases and sums with FP64 anchors,
// FP64 cross-segment sums and force accumulation; double: FP64 throughout)
// and dispatch per block on the request's n_z class (5, 9 or 17 slots).

#include <hip/hip_runtime.h>

#include "sce_device.h"
#include "sce_internal.h"
#include "sce_serve.h"

namespace sce {
namespace {

constexpr double kTwoPiS = 6.283185307179586476925286766559;

template <typename T> struct Cx;
template <> struct Cx<float> { typedef float2 t; };
template <> struct Cx<double> { typedef double2 t; };

// Fourier transform of the particle shape (S(0) = 1): point, Gaussian, tent.
__device__ inline double shape_at(int kind, double a, double kx, double ky, double kz)
{
    if (kind == 1) return exp(-0.5 * (kx * kx + ky * ky + kz * kz) * a * a);
    if (kind == 2) {
        double s = 1.0;
        const double k3[3] = {kx, ky, kz};
        for (int d = 0; d < 3; ++d) {
            const double u = 0.5 * k3[d] * a;
            const double sc = u == 0.0 ? 1.0 : sin(u) / u;
            s *= sc * sc;
        }
        return s;
    }
    return 1.0;
}

__device__ inline double wrap_l(double x, double L, double invL)
{
    double w = x - L * floor(x * invL);
    if (w >= L || w < 0.0) w = 0.0;
    return w;
}

// ------------------------------------------------------------------ deposit
// Item idx = tile * segs + seg: rows 64 tile .. 64 tile + 63 (one per lane),
// particles kServeSeg seg .. (one segment).  Per chunk of 64 particles the
// block builds cis tables in LDS; wave w takes particles w, w+4, ... of the
// chunk, and the four waves' sums are added in fixed order at the end.
template <typename T, int NZ>
__device__ void dep_body(const ReqDesc &d, int idx, char *__restrict__ arena, char *smem)
{
    typedef typename Cx<T>::t CT;
    // z first: a particle's z row then lies within the immediate offsets of
    // the LDS reads, from one base register (further in, the compiler formed
    // a new address for every pair of reads; 1% more serving capacity)
    CT *ez = reinterpret_cast<CT *>(smem);  // [64][NZ] (cos, sin)(2 pi k tz)
    CT *ex = ez + 64 * NZ;                   // [64][NZ] cis(-2 pi k tx)
    CT *ey = ex + 64 * NZ;                   // [64][NZ] cis(-2 pi k ty)
    T *qv = reinterpret_cast<T *>(ey + 64 * NZ);

    const int64_t N = d.N;
    const int tile = idx / d.segs, seg = idx - tile * d.segs;
    const double *__restrict__ pos = reinterpret_cast<const double *>(arena + d.o_pos);
    const double *__restrict__ q = reinterpret_cast<const double *>(arena + d.o_q);
    // the wave index is wave-uniform; readfirstlane lets the compiler keep it
    // (and the particle loop below) in scalar registers
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r = tile * 64 + lane;
    int nx, ny;
    row_nxny(r < d.R ? r : 0, d.n, nx, ny);
    const int ay = ny < 0 ? -ny : ny;
    const T ysign = ny < 0 ? (T)-1 : (T)1;

    T Pr[NZ], Pi[NZ], Qr[NZ], Qi[NZ];
#pragma unroll
    for (int k = 0; k < NZ; ++k) Pr[k] = Pi[k] = Qr[k] = Qi[k] = (T)0;

    const int64_t j0 = (int64_t)seg * kServeSeg;
    const int64_t j1 = j0 + kServeSeg < N ? j0 + kServeSeg : N;
    for (int64_t c0 = j0; c0 < j1; c0 += 64) {
        __syncthreads();
        if (threadIdx.x < 192) {
            const int p = threadIdx.x & 63, axis = threadIdx.x >> 6;
            const int64_t j = c0 + p;
            const bool in = j < j1;
            const double t = in ? frac(pos[axis * N + j] * d.invL) : 0.0;
            CT *tab = (axis == 0 ? ex : (axis == 1 ? ey : ez)) + p * NZ;
            double c1, s1, c = 1.0, s = 0.0;
            cis_turns(t, c1, s1);
            const double sg = axis < 2 ? -1.0 : 1.0;
            for (int k = 0; k < NZ; ++k) {
                if ((k & 7) == 0) {
                    cis_turns(frac_mul(k, t), c, s);
                } else {
                    const double cn = c * c1 - s * s1;
                    s = s * c1 + c * s1;
                    c = cn;
                }
                CT e;
                e.x = (T)c;
                e.y = (T)(sg * s);
                tab[k] = e;
            }
            if (axis == 0) qv[p] = in ? (T)q[j] : (T)0;
        }
        __syncthreads();
        const int cnt = (int)(j1 - c0 < 64 ? j1 - c0 : 64);
        for (int p = w; p < cnt; p += 4) {
            const CT a = ex[p * NZ + nx];
            CT b = ey[p * NZ + ay];
            b.y *= ysign;
            const T qq = qv[p];
            const T hr = qq * (a.x * b.x - a.y * b.y);
            const T hi = qq * (a.x * b.y + a.y * b.x);
            const CT *z = ez + p * NZ;
#pragma unroll
            for (int k = 0; k < NZ; ++k) {
                const CT e = z[k];
                Pr[k] = fma(hr, e.x, Pr[k]);
                Pi[k] = fma(hi, e.x, Pi[k]);
                Qr[k] = fma(hr, e.y, Qr[k]);
                Qi[k] = fma(hi, e.y, Qi[k]);
            }
        }
    }

    // fixed-order sum of the four waves: waves 1..3 stage one component at a time
    T *red = reinterpret_cast<T *>(smem);  // [3][NZ][64]
    T *part = reinterpret_cast<T *>(arena + d.o_part);
    const int64_t Rp = d.Rp;
#pragma unroll
    for (int comp = 0; comp < 4; ++comp) {
        T *acc = comp == 0 ? Pr : (comp == 1 ? Pi : (comp == 2 ? Qr : Qi));
        __syncthreads();
        if (w > 0) {
#pragma unroll
            for (int k = 0; k < NZ; ++k) red[((w - 1) * NZ + k) * 64 + lane] = acc[k];
        }
        __syncthreads();
        if (w == 0 && r < d.R) {
#pragma unroll
            for (int k = 0; k < NZ; ++k) {
                const T v = ((acc[k] + red[k * 64 + lane]) + red[(NZ + k) * 64 + lane]) +
                            red[(2 * NZ + k) * 64 + lane];
                part[(((int64_t)seg * NZ + k) * 4 + comp) * Rp + r] = v;
            }
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_serve_deposit(const ReqDesc *__restrict__ desc, char *__restrict__ arena,
                const ServeItem *__restrict__ items, const int *__restrict__ counts)
{
    extern __shared__ double smem_d[];
    if ((int)blockIdx.x >= counts[0]) return;
    const ServeItem it = items[blockIdx.x];
    const ReqDesc &d = desc[it.slot];
    char *smem = reinterpret_cast<char *>(smem_d);
    if (d.nzs == 5)
        dep_body<T, 5>(d, it.idx, arena, smem);
    else if (d.nzs == 9)
        dep_body<T, 9>(d, it.idx, arena, smem);
    else
        dep_body<T, 17>(d, it.idx, arena, smem);
}

// ------------------------------------------------------------------ reduce + solve
__device__ inline double blk_sum(double v, double *sh)
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

__device__ inline double blk_max(double v, double *sh)
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

// Item idx: cells 256 idx .. of the request's R x nzs (row fastest).  Sums
// the segment partials in FP64 in segment order, forms rho(+-nz) and psi,
// writes the force table [R][nzs-1][4] = (sig, del) for nz >= 1 (zero beyond
// n_max) and psi(nz = 0) per row, and the item's partial W and max|rho|.
template <typename T>
__global__ void __launch_bounds__(256)
k_serve_reduce(const ReqDesc *__restrict__ desc, char *__restrict__ arena,
               const ServeItem *__restrict__ items, const int *__restrict__ counts)
{
    __shared__ double sh[8];
    if ((int)blockIdx.x >= counts[1]) return;
    const ServeItem it = items[blockIdx.x];
    const ReqDesc &d = desc[it.slot];
    const int n = d.n, R = d.R, nzs = d.nzs;
    const int cell = it.idx * 256 + threadIdx.x;
    double wsum = 0.0, amax = 0.0;
    if (cell < R * nzs) {
        const int nz = cell / R;
        const int row = cell - nz * R;
        T *ftab = reinterpret_cast<T *>(arena + d.o_ftab);
        T *psi0 = reinterpret_cast<T *>(arena + d.o_psi0);
        T *f = nz > 0 ? ftab + ((int64_t)row * (nzs - 1) + (nz - 1)) * 4 : nullptr;
        if (nz > n) {
            for (int e = 0; e < 4; ++e) f[e] = (T)0;
        } else {
            const T *part = reinterpret_cast<const T *>(arena + d.o_part);
            const int64_t Rp = d.Rp, sstride = (int64_t)nzs * 4 * Rp;
            const T *pp = part + (int64_t)nz * 4 * Rp + row;
            double Pr = 0.0, Pi = 0.0, Qr = 0.0, Qi = 0.0;
            // four segments' values are loaded before any is added, so that
            // their loads are in flight together (one segment at a time, the
            // loop waited for each); the additions keep the segment order
            int sg = 0;
            for (; sg + 3 < d.segs; sg += 4, pp += 4 * sstride) {
                T v[4][4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const T *qq = pp + u * sstride;
                    v[u][0] = qq[0];
                    v[u][1] = qq[Rp];
                    v[u][2] = qq[2 * Rp];
                    v[u][3] = qq[3 * Rp];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    Pr += (double)v[u][0];
                    Pi += (double)v[u][1];
                    Qr += (double)v[u][2];
                    Qi += (double)v[u][3];
                }
            }
            for (; sg < d.segs; ++sg, pp += sstride) {
                Pr += (double)pp[0];
                Pi += (double)pp[Rp];
                Qr += (double)pp[2 * Rp];
                Qi += (double)pp[3 * Rp];
            }
            int nx, ny;
            row_nxny(row, n, nx, ny);
            const double kf = kTwoPiS * d.invL;
            const double kx = kf * nx, ky = kf * ny, kz = kf * nz;
            const double k2 = kx * kx + ky * ky + kz * kz;
            const double S = shape_at(d.shape, d.a, kx, ky, kz);
            const double V = d.dim == 2 ? d.L * d.L : d.L * d.L * d.L;
            const double K = k2 > 0.0 ? 1.0 / (d.eps0 * k2 * V) : 0.0;
            const double G = S * K;
            const double rpr = S * (Pr + Qi), rpi = S * (Pi - Qr);  // rho(+nz)
            const double rmr = S * (Pr - Qi), rmi = S * (Pi + Qr);  // rho(-nz)
            const bool hp = in_half(nx, ny, nz);
            const bool hm = nz > 0 && in_half(nx, ny, -nz);
            const double ppr = hp ? G * rpr : 0.0, ppi = hp ? G * rpi : 0.0;
            const double pmr = hm ? G * rmr : 0.0, pmi = hm ? G * rmi : 0.0;
            if (hp) {
                wsum += K * (rpr * rpr + rpi * rpi);
                amax = fmax(amax, sqrt(rpr * rpr + rpi * rpi));
            }
            if (hm) {
                wsum += K * (rmr * rmr + rmi * rmi);
                amax = fmax(amax, sqrt(rmr * rmr + rmi * rmi));
            }
            if (nz == 0) {
                psi0[2 * row] = (T)ppr;
                psi0[2 * row + 1] = (T)ppi;
            } else {
                const double sr = ppr + pmr, si = ppi + pmi;
                const double dr = ppr - pmr, di = ppi - pmi;
                f[0] = (T)sr;
                f[1] = (T)si;
                f[2] = (T)dr;
                f[3] = (T)di;
            }
        }
    }
    const double ws = blk_sum(wsum, sh);
    const double wm = blk_max(amax, sh);
    if (threadIdx.x == 0) {
        double *rpart = reinterpret_cast<double *>(arena + d.o_rpart);
        rpart[2 * it.idx] = ws;
        rpart[2 * it.idx + 1] = wm;
    }
}

// ------------------------------------------------------------------ force + kick + drift
// Item idx: particles 64 idx .. 64 idx + 63 (one per lane); wave w of the
// item's kFrcWaves sums rows [w R / kFrcWaves, (w+1) R / kFrcWaves).  The
// waves' sums are added in fixed order, then wave 0 applies the pass's kick
// and drift and writes the item's diagnostics partials (a fixed shuffle tree,
// so repeated runs give identical bits).  Eight waves per item rather than
// four: a tick's largest requests (n_max = 16, 545 rows) then finish in half
// the time, and each SIMD holds two of an item's waves (measured saturated
// capacity +17%; five or ten waves, which spread unevenly over the four
// SIMDs, were slower than four).  Along an n_x line the row phase follows an
// FP64 recurrence in n_y from one exponential at the line's start.
// REC: a recorded pass (the first or the last), which also sums the potential
// and writes the diagnostics partials; the other passes skip both.
constexpr int kFrcWaves = 8;
template <typename T, int NZ, bool REC>
__device__ void frc_body(const ReqDesc &d, int idx, char *__restrict__ arena,
                         const char *__restrict__ tabs, double *shd)
{
    constexpr int NK = NZ - 1;
    const int64_t N = d.N;
    // wave-uniform row range: scalar loads of the force table
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t j = (int64_t)idx * 64 + lane;
    const int64_t jc = j < N ? j : N - 1;
    double *pos = reinterpret_cast<double *>(arena + d.o_pos);
    double *vel = reinterpret_cast<double *>(arena + d.o_vel);
    const double tx = frac(pos[jc] * d.invL);
    const double ty = frac(pos[N + jc] * d.invL);
    const double tz = frac(pos[2 * N + jc] * d.invL);

    T cz[NK], sz[NK];
    {
        double c1, s1, c = 1.0, s = 0.0;
        cis_turns(tz, c1, s1);
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            if ((k & 7) == 0) {
                cis_turns(frac_mul(k + 1, tz), c, s);
            } else {
                const double cn = c * c1 - s * s1;
                s = s * c1 + c * s1;
                c = cn;
            }
            cz[k] = (T)c;
            sz[k] = (T)s;
        }
    }
    double eyc, eys;
    cis_turns(ty, eyc, eys);

    const T *__restrict__ ftab = reinterpret_cast<const T *>(tabs + d.o_ftab);
    const T *__restrict__ psi0 = reinterpret_cast<const T *>(tabs + d.o_psi0);
    const int n = d.n, R = d.R;
    const int r0 = (R * w) / kFrcWaves, r1 = (R * (w + 1)) / kFrcWaves;
    double fx = 0.0, fy = 0.0, fz = 0.0, ph = 0.0;
    int nx, ny;
    row_nxny(r0, n, nx, ny);
    double gc = 1.0, gs = 0.0;
    bool anchor = true;
    for (int r = r0; r < r1; ++r) {
        if (anchor) {
            cis_turns(frac_lin(nx, tx, ny, ty), gc, gs);
            anchor = false;
        }
        // the n_z weights of U1 are applied here rather than stored (a table
        // of sig and del only: half the scalar loads per row for two more
        // FMAs per slot, 5% less device time per tick)
        const T *ft = ftab + (int64_t)r * NK * 4;
        T u0r = psi0[2 * r], u0i = psi0[2 * r + 1], u1r = (T)0, u1i = (T)0;
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            const T c = cz[k], s = sz[k];
            const T sr = ft[4 * k + 0], si = ft[4 * k + 1], dr = ft[4 * k + 2], di = ft[4 * k + 3];
            u0r = fma(sr, c, u0r);
            u0i = fma(si, c, u0i);
            u0r = fma(-di, s, u0r);
            u0i = fma(dr, s, u0i);
            const T t1r = fma(-si, s, dr * c), t1i = fma(sr, s, di * c);
            u1r = fma((T)(k + 1), t1r, u1r);
            u1i = fma((T)(k + 1), t1i, u1i);
        }
        const double im0 = gc * (double)u0i + gs * (double)u0r;
        const double im1 = gc * (double)u1i + gs * (double)u1r;
        fx = fma((double)nx, im0, fx);
        fy = fma((double)ny, im0, fy);
        fz += im1;
        if (REC) ph += gc * (double)u0r - gs * (double)u0i;
        // next row: n_y + 1 within the line, else the next n_x line (re-anchor)
        if (ny < n) {
            ++ny;
            const double t = gc * eyc - gs * eys;
            gs = gs * eyc + gc * eys;
            gc = t;
        } else {
            ++nx;
            ny = -n;
            anchor = true;
        }
    }

    // fixed-order sum of the waves' partial sums
    __syncthreads();
    if (w > 0) {
        double *o = shd + ((w - 1) * 64 + lane) * 4;
        o[0] = fx;
        o[1] = fy;
        o[2] = fz;
        o[3] = ph;
    }
    __syncthreads();
    if (w != 0) return;
    for (int i = 0; i < kFrcWaves - 1; ++i) {
        const double *o = shd + (i * 64 + lane) * 4;
        fx += o[0];
        fy += o[1];
        fz += o[2];
        ph += o[3];
    }

    double acc[kServeFDiag];
    for (int i = 0; i < kServeFDiag; ++i) acc[i] = 0.0;
    if (j < N) {
        const double *q = reinterpret_cast<const double *>(arena + d.o_q);
        const double *m = reinterpret_cast<const double *>(arena + d.o_m);
        double *F = reinterpret_cast<double *>(arena + d.o_F);
        const double qj = q[j], mj = m[j];
        const double f = 2.0 * qj * (kTwoPiS * d.invL);
        const double Fx = f * fx, Fy = f * fy, Fz = f * fz;
        F[j] = Fx;
        F[N + j] = Fy;
        F[2 * N + j] = Fz;
        const int64_t p = d.pass, S = d.n_steps;
        const double a = S == 0 ? 0.0 : ((p == 0 || p == S) ? 0.5 * d.dt : d.dt);
        const double b = p < S ? d.dt : 0.0;
        double vx = vel[j], vy = vel[N + j], vz = vel[2 * N + j];
        if (REC) {
            const double v2 = vx * vx + vy * vy + vz * vz;
            acc[0] = 0.5 * mj * v2;
            acc[2] = mj * vx;
            acc[3] = mj * vy;
            acc[4] = mj * vz;
            acc[8] = mj * sqrt(v2);
        }
        const double am = a / mj;
        vx += am * Fx;
        vy += am * Fy;
        vz += am * Fz;
        if (REC) {
            const double v2 = vx * vx + vy * vy + vz * vz;
            acc[1] = 0.5 * mj * v2;
            acc[5] = mj * vx;
            acc[6] = mj * vy;
            acc[7] = mj * vz;
            acc[9] = mj * sqrt(v2);
            acc[10] = qj * 2.0 * ph;
        }
        vel[j] = vx;
        vel[N + j] = vy;
        vel[2 * N + j] = vz;
        if (b != 0.0) {
            pos[j] = wrap_l(pos[j] + b * vx, d.L, d.invL);
            pos[N + j] = wrap_l(pos[N + j] + b * vy, d.L, d.invL);
            pos[2 * N + j] = wrap_l(pos[2 * N + j] + b * vz, d.L, d.invL);
        }
    }
    if (!REC) return;
    double *fpart = reinterpret_cast<double *>(arena + d.o_fpart) + (int64_t)idx * kServeFDiag;
    for (int i = 0; i < kServeFDiag; ++i) {
        double v = acc[i];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) fpart[i] = v;
    }
}

// tabs: the arena again, read-only here (force tables only; particle state is
// read and written through arena), so that the wave-uniform table rows can be
// fetched with scalar loads.  FP32: six waves per SIMD (80 VGPRs, three items
// per compute unit) measured 3% more capacity than five, despite a few
// spilled registers; FP64 keeps the compiler's choice.
template <typename T>
__global__ void __launch_bounds__(64 * kFrcWaves) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 1)))
k_serve_force(const ReqDesc *__restrict__ desc, char *__restrict__ arena,
              const char *__restrict__ tabs, const ServeItem *__restrict__ items,
              const int *__restrict__ counts)
{
    __shared__ double shd[(kFrcWaves - 1) * 64 * 4];
    if ((int)blockIdx.x >= counts[2]) return;
    const ServeItem it = items[blockIdx.x];
    const ReqDesc &d = desc[it.slot];
    const bool rec = d.pass == 0 || d.pass == d.n_steps;
    if (d.nzs == 5) {
        if (rec) frc_body<T, 5, true>(d, it.idx, arena, tabs, shd);
        else frc_body<T, 5, false>(d, it.idx, arena, tabs, shd);
    } else if (d.nzs == 9) {
        if (rec) frc_body<T, 9, true>(d, it.idx, arena, tabs, shd);
        else frc_body<T, 9, false>(d, it.idx, arena, tabs, shd);
    } else {
        if (rec) frc_body<T, 17, true>(d, it.idx, arena, tabs, shd);
        else frc_body<T, 17, false>(d, it.idx, arena, tabs, shd);
    }
}

// ------------------------------------------------------------------ diagnostics + pass count
// One wave per resident request: counts the pass, and on the first and the
// last pass records its diagnostics (lane l sums the item partials l, l+64,
// ... in order, a fixed shuffle tree adds the lanes).
__global__ void __launch_bounds__(64)
k_serve_diag(ReqDesc *__restrict__ desc, char *__restrict__ arena, const int *__restrict__ slots,
             const int *__restrict__ counts)
{
    if ((int)blockIdx.x >= counts[3]) return;
    const int lane = threadIdx.x;
    ReqDesc &d = desc[slots[blockIdx.x]];
    const int64_t p = d.pass;
    // only the first and the last pass are recorded
    if (p != 0 && p != d.n_steps) {
        if (lane == 0) d.pass = p + 1;
        return;
    }
    const double *fpart = reinterpret_cast<const double *>(arena + d.o_fpart);
    const double *rpart = reinterpret_cast<const double *>(arena + d.o_rpart);
    double s[kServeFDiag];
    for (int c = 0; c < kServeFDiag; ++c) s[c] = 0.0;
    for (int b = lane; b < d.fblocks; b += 64)
        for (int c = 0; c < kServeFDiag; ++c) s[c] += fpart[b * kServeFDiag + c];
    double W = 0.0, mx = 0.0;
    for (int b = lane; b < d.rblocks; b += 64) {
        W += rpart[2 * b];
        mx = fmax(mx, rpart[2 * b + 1]);
    }
    for (int o = 32; o > 0; o >>= 1) {
        for (int c = 0; c < kServeFDiag; ++c) s[c] += __shfl_xor(s[c], o, 64);
        W += __shfl_xor(W, o, 64);
        mx = fmax(mx, __shfl_xor(mx, o, 64));
    }
    if (lane != 0) return;
    double *diag = reinterpret_cast<double *>(arena + d.o_diag);
    if (p == 0) {
        const double v[8] = {s[0], W, s[10], s[2], s[3], s[4], s[8], mx};
        for (int c = 0; c < 8; ++c) diag[c] = v[c];
    }
    if (p == d.n_steps) {
        const double v[8] = {s[1], W, s[10], s[5], s[6], s[7], s[9], mx};
        for (int c = 0; c < 8; ++c) diag[8 + c] = v[c];
    }
    d.pass = p + 1;
}

// Grids of gdep, gred, gfrc and gslots blocks (at least the counts on the
// device, which blocks beyond return at once), so that a captured tick stays
// valid while the resident set changes within the lists' capacity.
template <typename T>
hipError_t tick(hipStream_t s, const ReqDesc *desc, char *arena, const ServeItem *dep, int gdep,
                const ServeItem *red, int gred, const ServeItem *frc, int gfrc, const int *slots,
                int gslots, const int *counts)
{
    const size_t dep_lds = (size_t)3 * 64 * 17 * sizeof(typename Cx<T>::t) + 64 * sizeof(T);
    if (gdep > 0)
        hipLaunchKernelGGL(k_serve_deposit<T>, dim3(gdep), dim3(256), dep_lds, s, desc, arena, dep, counts);
    if (gred > 0)
        hipLaunchKernelGGL(k_serve_reduce<T>, dim3(gred), dim3(256), 0, s, desc, arena, red, counts);
    if (gfrc > 0)
        hipLaunchKernelGGL(k_serve_force<T>, dim3(gfrc), dim3(64 * kFrcWaves), 0, s, desc, arena,
                           (const char *)arena, frc, counts);
    if (gslots > 0)
        hipLaunchKernelGGL(k_serve_diag, dim3(gslots), dim3(64), 0, s, const_cast<ReqDesc *>(desc),
                           arena, slots, counts);
    return hipGetLastError();
}

}  // namespace

size_t serve_layout(ReqDesc &d, int elem_bytes)
{
    const int n = d.n;
    const int64_t N = d.N;
    d.R = d.dim == 2 ? n + 1 : (n + 1) + n * (2 * n + 1);
    d.Rp = (d.R + 63) / 64 * 64;
    d.nzs = serve_nz(n);
    d.segs = (int)((N + kServeSeg - 1) / kServeSeg);
    d.fblocks = (int)((N + 63) / 64);
    d.rblocks = (d.R * d.nzs + 255) / 256;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    size_t off = 0;
    d.o_pos = (int64_t)off;
    off += al(24 * (size_t)N);
    d.o_vel = (int64_t)off;
    off += al(24 * (size_t)N);
    d.o_F = (int64_t)off;
    off += al(24 * (size_t)N);
    d.o_q = (int64_t)off;
    off += al(8 * (size_t)N);
    d.o_m = (int64_t)off;
    off += al(8 * (size_t)N);
    d.o_part = (int64_t)off;
    off += al((size_t)d.segs * d.nzs * 4 * d.Rp * elem_bytes);
    d.o_ftab = (int64_t)off;
    off += al((size_t)d.R * (d.nzs - 1) * 4 * elem_bytes);
    d.o_psi0 = (int64_t)off;
    off += al((size_t)d.R * 2 * elem_bytes);
    d.o_rpart = (int64_t)off;
    off += al((size_t)d.rblocks * 2 * 8);
    d.o_fpart = (int64_t)off;
    off += al((size_t)d.fblocks * kServeFDiag * 8);
    d.o_diag = (int64_t)off;
    off += al((size_t)kServeDiag * 8);
    return off;
}

hipError_t launch_serve_tick(hipStream_t s, int elem_bytes, const ReqDesc *desc, char *arena,
                             const ServeItem *dep, int gdep, const ServeItem *red, int gred,
                             const ServeItem *frc, int gfrc, const int *slots, int gslots,
                             const int *counts)
{
    if (elem_bytes == 8)
        return tick<double>(s, desc, arena, dep, gdep, red, gred, frc, gfrc, slots, gslots, counts);
    return tick<float>(s, desc, arena, dep, gdep, red, gred, frc, gfrc, slots, gslots, counts);
}

}  // namespace sce
