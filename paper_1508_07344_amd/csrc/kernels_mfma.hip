// Split-precision matrix-core kernels (gfx950, v_mfma_f32_16x16x32_f16) for
// the two particle x mode sums.
//
// With separable phases (modes spaced 2 pi / L, Section 8) both sums are dense
// contractions:
//   deposit  C[c, r] = sum_j CS[c, j] H[j, r]         (K = particles)
//            CS[c, j] = cos(c tz_j) for c = 0..n, sin((c-n) tz_j) for c = n+1..2n
//            H[j, r]  = q_j exp(-i (nx tx_j + ny ty_j))   (real and imaginary parts
//                       as two GEMMs), so C gives P (cos rows) and Q (sin rows).
//   force    U[(r, e), j] = sum_k W[(r, e), k] CS'[k, j]   (K = cos and sin of n_z = 1..)
//            e = (Re U0, Im U0, Re U1, Im U1) of the row's n_z sums, then
//            F_j += (nx Im(g U0), ny Im(g U0), Im(g U1)), g = exp(i (nx tx + ny ty)).
// Every FP32 operand x is carried as two FP16 values hi = fp16(x),
// lo = fp16(x - hi); a product uses hi*hi + hi*lo + lo*hi (the lo*lo term,
// ~2^-22 relative, is dropped), accumulated in FP32 by the matrix core.
// Operands are scaled to magnitude <= 1 first (charges by 1/max|q|, each
// force-table row by a power of two) so FP16's range is never exceeded.
//
// Fragment layout of v_mfma_f32_16x16x32_f16 (lane l, element i):
//   A[m][k]: m = l % 16, k = 8 (l / 16) + i     (8 halves)
//   B[k][n]: k = 8 (l / 16) + i, n = l % 16     (8 halves)
//   D[m][n]: m = 4 (l / 16) + i, n = l % 16     (4 floats)

#include "sce_internal.h"
#include "sce_device.h"

namespace sce {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline void split_f16(float x, _Float16 &hi, _Float16 &lo)
{
    hi = (_Float16)x;
    lo = (_Float16)(x - (float)hi);
}

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef float float2_t __attribute__((ext_vector_type(2)));

// lo parts of two values whose hi parts (round to nearest) are packed in hi:
// lo = fp16(x - hi), the difference formed exactly inside the mixed-precision
// FMA and rounded once, as fp16(x - (float)hi) is (that difference is exact in
// FP32).  Two instructions instead of two conversions back, two subtractions
// and a packing conversion.
__device__ inline half2_t split_lo2(float2_t x, half2_t hi)
{
    half2_t lo;
    asm("v_fma_mixlo_f16 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]\n\t"
        "v_fma_mixhi_f16 %0, -%1, 1.0, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
        : "=&v"(lo)
        : "v"(hi), "v"(x[0]), "v"(x[1]));
    return lo;
}

__device__ inline f32x4 mfma16(half8 a, half8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// acc += (ah + al)(bh + bl) without the al*bl term
__device__ inline f32x4 mfma_split(half8 ah, half8 al, half8 bh, half8 bl, f32x4 acc)
{
    acc = mfma16(al, bh, acc);
    acc = mfma16(ah, bl, acc);
    return mfma16(ah, bh, acc);
}

// The deposit visits the particles of a split in a pseudo-random order, so
// that each split is an unstructured sample of the particles: its FP32 sums
// then grow like random walks for every mode, whatever the input order (an
// affine order i*A mod N is a rank-1 lattice and stays coherent for some wave
// vectors).  The order is a bijection of [0, N): a 4-round Feistel network on
// 2h bits (2^(2h) >= N), each round (L, R) -> (R, L ^ f_r(R)), with cycle
// walking back into [0, N).  Particle j's record goes to slot feistel_inv(j).

// ------------------------------------------------------------------ deposit
// Particles are taken in chunks of 32 (the K depth of one matrix instruction).
constexpr int kDepChunk = 32;
// Both deposit operands are multiplied by 7/8 before the split (and the
// result by 64/49 in FP64).  Unscaled, cos(n_z theta) and h crowd just below
// 1.0 for particles near the origin, where round-to-nearest FP16 gives hi = 1
// and a negative lo in both operands: the dropped lo*lo term then has a
// consistent sign and acts like a spurious charge at the origin.  At 7/8 no
// operand sits at an FP16 exponent boundary and the lo parts are unbiased.
constexpr float kDepOpScale = 0.875f;
// The matrix core rounds its FP32 accumulation per group of products and, when
// the running sum is much larger than each increment, slightly toward -inf.
// Over thousands of chunks that directional bias is identical in every
// accumulator and would act like a spurious charge at the origin.  The running
// sum therefore changes sign every 2^kDepFlipLog chunks (accumulator and CS
// operand negated together), so the bias alternates direction and cancels.

// Per-particle record in visiting order, FP32, for nb = ceil((n+1)/8) blocks
// of 8 powers per axis: [d][blk] = cis(2 pi 8 blk t_d) (anchors, formed in
// FP64), then [d] = cis(2 pi t_d) (steps), then the scaled charge
// (q / max|q|) * 7/8; padded to a multiple of 4 floats.
__host__ __device__ inline int dep_rec_floats(int n)
{
    const int nb = (n + 1 + 7) / 8;
    return (3 * (nb + 1) * 2 + 1 + 3) / 4 * 4;
}

// Inverse of the visiting-order map: its rounds undone in reverse order,
// walking back into [0, N) the way the forward map walks out of it.
__device__ inline uint32_t feistel_inv(uint32_t j, uint32_t N, int h)
{
    const uint32_t mask = h >= 16 ? 0xFFFFu : ((1u << h) - 1u);
    uint32_t y = j;
    do {
        uint32_t L = y >> h, R = y & mask;
#pragma unroll
        for (int r = 3; r >= 0; --r) {
            uint32_t f = L * 0x9E3779B1u + 0x7F4A7C15u * (uint32_t)(r + 1);
            f ^= f >> 15;
            f *= 0x85EBCA6Bu;
            f ^= f >> 13;
            const uint32_t pl = (R ^ f) & mask;
            R = L;
            L = pl;
        }
        y = (L << h) | R;
    } while (y >= N);
    return y;
}

// Thread j takes particle j (coalesced reads) and writes its record at its
// place in the visiting order, feistel_inv(j), as 16-byte stores; NB anchor
// blocks per axis, so the record sits in registers with static indices.
template <int NB>
__global__ void __launch_bounds__(256)
k_deposit_prep(const double *__restrict__ pos, const double *__restrict__ q, int64_t N,
               double invL, int h, double qfac, float *__restrict__ rec)
{
    constexpr int RF = (3 * (NB + 1) * 2 + 1 + 3) / 4 * 4;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    const int64_t i = feistel_inv((uint32_t)j, (uint32_t)N, h);
    float r[RF];
#pragma unroll
    for (int e = 0; e < RF; ++e) r[e] = 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double t = frac(pos[d * N + j] * invL);
#pragma unroll
        for (int blk = 0; blk < NB; ++blk) {
            double c, sn;
            cis_turns(frac_mul(8 * blk, t), c, sn);
            r[2 * (d * NB + blk)] = (float)c;
            r[2 * (d * NB + blk) + 1] = (float)sn;
        }
        double c, sn;
        cis_turns(t, c, sn);
        r[2 * (3 * NB + d)] = (float)c;
        r[2 * (3 * NB + d) + 1] = (float)sn;
    }
    r[6 * (NB + 1)] = (float)(q[j] * qfac);
    float4 *o = reinterpret_cast<float4 *>(rec + i * RF);
#pragma unroll
    for (int e = 0; e < RF / 4; ++e) o[e] = make_float4(r[4 * e], r[4 * e + 1], r[4 * e + 2], r[4 * e + 3]);
}

// LDS table layouts of the deposit.  Row strides are those of the largest
// n_max of the tile class (8 MT), fixed at compile time, so that the
// matrix-core waves address the 8 particles of their lane group with the
// read instruction's immediate offset.  Row of particle p in the a table
// (8 MT + 1 entries, k = 0..n used): groups of 8 particles separated by 4
// float2, so the four lane groups (particles 8g..8g+7) start in different
// banks.  b table (16 MT + 1 entries, k = -n..n used around column n): the
// group padding of 8 float2 makes the groups' rows start 128 bytes apart
// modulo the 256-byte bank cycle, so that lane groups 0/1 and 2/3, which read
// 16 consecutive entries each in the same pass, use disjoint banks.  The CS
// operand is stored in the matrix core's fragment order (cs_idx), so that a
// lane's 16-byte fragment read is at 16 lane + const: 16-byte LDS reads run at
// full rate only when the lanes' addresses are consecutive.  A table entry read as a volatile LDS double, which the compiler keeps as a
// read of its own.
typedef const volatile double __attribute__((address_space(3))) lds_f2;
__device__ inline float2 lds_read(lds_f2 *p)
{
    const double d = *p;
    return __builtin_bit_cast(float2, d);
}

template <int MT>
struct DepTab {
    static constexpr int wa = 8 * MT + 1;
    static constexpr int wb = 16 * MT + 1;
    static constexpr int pada = 4;
    static constexpr int padb = 8;  // wb = 1 mod 4
};
__device__ inline int tab_row(int p, int w, int pad) { return p * w + (p >> 3) * pad; }
// CS element (row, particle p of the chunk) in fragment order: tile mt =
// row / 16 holds 64 lanes x 8 halves, lane = row % 16 + 16 (p / 8), half p % 8.
__device__ inline int cs_idx(int row, int p)
{
    return (row >> 4) * 512 + (p >> 3) * 128 + (row & 15) * 8 + (p & 7);
}

// Running sums change sign every 2^kDepFlipLog chunks.
constexpr int kDepFlipLog = 3;
// FP32 sums of the n_z = 0 row are added into FP64 every 2^kDepDcLog chunks.
constexpr int kDepDcLog = 4;

// CS rows of the matrix-core operand: cos(n_z theta) for n_z = 1..n (rows
// 0..n-1), sin(n_z theta) for n_z = 1..n (rows n..2n-1), zero padding to 16s.
// The n_z = 0 row (all ones) is summed on the VALU instead.
__host__ __device__ inline int mfma_cs_tiles(int n) { return (2 * n + 15) / 16; }

template <int MT>
__host__ __device__ constexpr size_t dep_buf_bytes()
{
    using T = DepTab<MT>;
    return (size_t)MT * 16 * kDepChunk * 2 * sizeof(_Float16) +
           (size_t)(kDepChunk * T::wa + 4 * T::pada + kDepChunk * T::wb + 4 * T::padb) * sizeof(float2);
}

// Block = kDepCompW matrix-core waves + kDepBuildW table-builder waves for
// one (row block, particle split) pair; the split's particles are visited in
// the pseudo-random order of the particle records, and the block's rows are
// 16 NTW rows per matrix-core wave.
// Per chunk of 32 particles the builder waves write the LDS tables of the
// next chunk from the records: a = q cis(-k tx) for k = 0..n, b = cis(-k ty)
// for k = -n..n (FP32), and the CS operand as FP16 hi/lo, while the
// matrix-core waves multiply the current chunk out of the other buffer; one
// barrier per chunk.  Each matrix-core lane forms its own H = a b fragment (8
// particles x 1 row), splits it into hi/lo and adds its n_z = 0 contribution
// on the VALU.
constexpr int kDepCompW = 12;
constexpr int kDepBuildW = 4;
constexpr int kDepThreads = 64 * (kDepCompW + kDepBuildW);

__host__ __device__ inline int dep_ntw(int MT) { return MT <= 4 ? 2 : 1; }
__host__ __device__ inline int dep_rows_per_block(int MT) { return 16 * dep_ntw(MT) * kDepCompW; }

// XCD-aware block order: consecutive blocks go to different XCDs (each with
// its own L2), so the grid is numbered such that the row blocks of one
// particle split are dispatched to the same XCD one after another and their
// reads of the split's particle records hit that XCD's L2.  Linear block L
// runs on XCD L % 8; its position t = L / 8 in that XCD's sequence selects
// row block t % row_blocks of split (t / row_blocks) * 8 + L % 8.
constexpr int kXcds = 8;

template <int MT>
__global__ void __launch_bounds__(kDepThreads)
k_deposit_mfma(const float *__restrict__ rec, int64_t N, int n, int R, int Rpad,
               int64_t per_split, int row_blocks, int splits, double unscale_mf, double unscale_dc,
               float *__restrict__ part)
{
    const int blk_l = blockIdx.x;
    const int blk_t = blk_l / kXcds;
    const int rblk = blk_t % row_blocks;
    const int split = (blk_t / row_blocks) * kXcds + blk_l % kXcds;
    if (split >= splits) return;
    constexpr int NTW = MT <= 4 ? 2 : 1;
    extern __shared__ __align__(16) unsigned char smem[];
    const int n1 = n + 1;
    constexpr int CSR = MT * 16;
    constexpr size_t bufb = dep_buf_bytes<MT>();
    using T = DepTab<MT>;
    auto cs_hi = [&](int b) { return reinterpret_cast<_Float16 *>(smem + b * bufb); };
    auto cs_lo = [&](int b) { return reinterpret_cast<_Float16 *>(smem + b * bufb) + CSR * kDepChunk; };
    auto tab_a = [&](int b) {
        return reinterpret_cast<float2 *>(smem + b * bufb + (size_t)CSR * kDepChunk * 2 * sizeof(_Float16));
    };
    auto tab_b = [&](int b) { return tab_a(b) + kDepChunk * T::wa + 4 * T::pada; };

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t j0 = (int64_t)split * per_split;
    const int64_t j1 = j0 + per_split < N ? j0 + per_split : N;
    const int64_t nchunks = (j1 - j0 + kDepChunk - 1) / kDepChunk;
    const int nb = (n1 + 7) / 8;

    for (int idx = tid; idx < (CSR - 2 * n) * kDepChunk; idx += kDepThreads)
        for (int b = 0; b < 2; ++b) {
            const int e = cs_idx(2 * n + idx / kDepChunk, idx % kDepChunk);
            cs_hi(b)[e] = (_Float16)0.0f;
            cs_lo(b)[e] = (_Float16)0.0f;
        }

    if (wave >= kDepCompW) {
        // ---------------- table builders
        // raised issue priority: the next chunk's tables are the critical path,
        // the matrix-core waves fill the remaining issue slots
        __builtin_amdgcn_s_setprio(2);
        // tasks (axis d, block of 8 powers blk, particle p), particle fastest.
        // A wave takes 64 tasks at a time, a pair of blocks of one axis (the
        // block count is padded to even per axis), so its two half-waves never
        // take different branches: wave slot ws = 4 sl + (builder wave) is
        // axis ws / npair, block pair ws % npair.  The record fields of the
        // next chunk's tasks are loaded one chunk ahead.
        constexpr int kDepSlots = 6;  // enough for n_max <= 64
        const int bw = wave - kDepCompW;
        const int npair = (nb + 1) / 2;
        const int rf = dep_rec_floats(n);
        float rc[kDepSlots], rs[kDepSlots], sc[kDepSlots], ss[kDepSlots], rq[kDepSlots];
        auto task_of = [&](int sl, int &d, int &blk, int &p) {
            const int ws = sl * kDepBuildW + bw;
            d = ws / npair;
            blk = 2 * (ws - d * npair) + (lane >> 5);
            p = lane & (kDepChunk - 1);
            return d < 3 && blk < nb;
        };
        auto load_chunk = [&](int64_t c) {
#pragma unroll
            for (int sl = 0; sl < kDepSlots; ++sl) {
                int d, blk, p;
                const bool ok = task_of(sl, d, blk, p);
                const int64_t j = j0 + c * kDepChunk + p;
                rc[sl] = 1.f;
                rs[sl] = 0.f;
                sc[sl] = 1.f;
                ss[sl] = 0.f;
                rq[sl] = 0.f;
                if (ok && c < nchunks && j < j1) {
                    const float *r0 = rec + j * rf;
                    rc[sl] = r0[2 * (d * nb + blk)];
                    rs[sl] = r0[2 * (d * nb + blk) + 1];
                    sc[sl] = r0[2 * (3 * nb + d)];
                    ss[sl] = r0[2 * (3 * nb + d) + 1];
                    rq[sl] = r0[6 * (nb + 1)];
                }
            }
        };
        // Powers by complex multiplication from the block's anchor; the anchor
        // carries the factor each table needs (q and the conjugation for a, the
        // running-sum sign and the 7/8 operand scale for CS), so the recurrence
        // propagates it at no cost.
        auto build_chunk = [&](int64_t c) {
            const int b = (int)(c & 1);
            const float csg = ((c >> kDepFlipLog) & 1) ? -kDepOpScale : kDepOpScale;
#pragma unroll
            for (int sl = 0; sl < kDepSlots; ++sl) {
                int d, blk, p;
                if (!task_of(sl, d, blk, p)) continue;
                const float c1 = sc[sl], s1 = ss[sl];
                const int k0 = 8 * blk;
                const int kend = n1 - k0 < 8 ? n1 - k0 : 8;
                if (d == 0) {
                    // u_k = q cis(-k tx): anchor q conj(cis), step conj(cis(tx))
                    float uc = rq[sl] * rc[sl], us = -rq[sl] * rs[sl];
                    float2 *dst = tab_a(b) + tab_row(p, T::wa, T::pada) + k0;
                    for (int kk = 0; kk < kend; ++kk) {
                        dst[kk] = make_float2(uc, us);
                        const float t = uc * c1 + us * s1;
                        us = us * c1 - uc * s1;
                        uc = t;
                    }
                } else if (d == 1) {
                    float fc = rc[sl], fs = rs[sl];
                    float2 *dst = tab_b(b) + tab_row(p, T::wb, T::padb) + n;
                    for (int kk = 0; kk < kend; ++kk) {
                        const int k = k0 + kk;
                        dst[k] = make_float2(fc, -fs);
                        dst[-k] = make_float2(fc, fs);
                        const float t = fc * c1 - fs * s1;
                        fs = fc * s1 + fs * c1;
                        fc = t;
                    }
                } else {
                    float2_t v;
                    v[0] = csg * rc[sl];
                    v[1] = csg * rs[sl];
                    _Float16 *hi = cs_hi(b), *lo = cs_lo(b);
                    for (int kk = 0; kk < kend; ++kk) {
                        const int k = k0 + kk;
                        if (k > 0) {
                            // (cos, sin) split two at a time
                            const half2_t h = __builtin_convertvector(v, half2_t);
                            const half2_t l = split_lo2(v, h);
                            hi[cs_idx(k - 1, p)] = h[0];
                            lo[cs_idx(k - 1, p)] = l[0];
                            hi[cs_idx(n + k - 1, p)] = h[1];
                            lo[cs_idx(n + k - 1, p)] = l[1];
                        }
                        const float t = v[0] * c1 - v[1] * s1;
                        v[1] = v[0] * s1 + v[1] * c1;
                        v[0] = t;
                    }
                }
            }
        };
        load_chunk(0);
        build_chunk(0);
        load_chunk(1);
        __syncthreads();
        for (int64_t c = 0; c < nchunks; ++c) {
            if (c + 1 < nchunks) {
                build_chunk(c + 1);
                load_chunk(c + 2);
            }
            __syncthreads();
        }
        return;
    }

    // ---------------- matrix-core waves
    const int g = lane >> 4;   // lane group: particles 8g..8g+7 of a chunk
    const int ln = lane & 15;  // row within an N tile
    const int row0 = rblk * dep_rows_per_block(MT) + wave * 16 * NTW;
    int rnx[NTW], rnyo[NTW];
    bool rok[NTW];
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt) {
        const int r = row0 + nt * 16 + ln;
        rok[nt] = r < R;
        int ny;
        row_nxny(r < R ? r : R - 1, n, rnx[nt], ny);
        rnyo[nt] = ny + n;  // column of k = ny in the b table
    }

    f32x4 acc[MT][NTW][2];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) acc[mt][nt][0] = acc[mt][nt][1] = f32x4{0.f, 0.f, 0.f, 0.f};
    // FP32 sums of the n_z = 0 row, added into this lane's FP64 slots in LDS
    // (after the two table buffers) every 2^kDepDcLog chunks
    float dc[NTW][2];
    double *dcd = reinterpret_cast<double *>(smem + 2 * bufb) + (wave * NTW * 2) * 64 + lane;
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt) {
        dc[nt][0] = dc[nt][1] = 0.f;
        dcd[(2 * nt) * 64] = 0.0;
        dcd[(2 * nt + 1) * 64] = 0.0;
    }

    // lane bases of the a and b rows of particle 8 g of a chunk, column of the lane's row
    int abase[NTW], bbase[NTW];
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt) {
        abase[nt] = tab_row(8 * g, T::wa, T::pada) + rnx[nt];
        bbase[nt] = tab_row(8 * g, T::wb, T::padb) + rnyo[nt];
    }

    __syncthreads();  // chunk 0's tables
    if (row0 >= R) {
        // every row of this wave lies past the last row (the last row block of a
        // grid whose rows do not fill it): only the block's barriers remain
        for (int64_t c = 0; c < nchunks; ++c) __syncthreads();
        return;
    }
    // groups of 2^kDepFlipLog chunks; the running sums change sign between groups
    for (int64_t c0 = 0; c0 < nchunks; c0 += (1 << kDepFlipLog)) {
      const int64_t ce = c0 + (1 << kDepFlipLog) < nchunks ? c0 + (1 << kDepFlipLog) : nchunks;
      for (int64_t c = c0; c < ce; ++c) {
        const int b = (int)(c & 1);
        const float2 *ta = tab_a(b), *tb = tab_b(b);
        const _Float16 *chi = cs_hi(b), *clo = cs_lo(b);
        // H fragments of every row tile first, then each CS tile read once
        // and multiplied with all of them
        half8 bre_h[NTW], bre_l[NTW], bim_h[NTW], bim_l[NTW];
#pragma unroll
        for (int nt = 0; nt < NTW; ++nt) {
            float sre = 0.f, sim = 0.f;
            // one 8-byte read per table entry: the compiler would otherwise pair
            // the reads of two particles into one two-address read, whose halves
            // fall in overlapping banks (the group padding is laid out for single
            // reads) and which runs slower
            lds_f2 *pa = (lds_f2 *)(ta + abase[nt]);
            lds_f2 *pbt = (lds_f2 *)(tb + bbase[nt]);
#pragma unroll
            for (int i = 0; i < 8; i += 2) {
                const float2 a0 = lds_read(pa + i * T::wa);
                const float2 b0 = lds_read(pbt + i * T::wb);
                const float2 a1 = lds_read(pa + (i + 1) * T::wa);
                const float2 b1 = lds_read(pbt + (i + 1) * T::wb);
                float2_t hr, hm;
                hr[0] = a0.x * b0.x - a0.y * b0.y;
                hm[0] = a0.x * b0.y + a0.y * b0.x;
                hr[1] = a1.x * b1.x - a1.y * b1.y;
                hm[1] = a1.x * b1.y + a1.y * b1.x;
                sre += hr[0] + hr[1];
                sim += hm[0] + hm[1];
                const half2_t rh = __builtin_convertvector(hr, half2_t);
                const half2_t mh = __builtin_convertvector(hm, half2_t);
                const half2_t rl = split_lo2(hr, rh);
                const half2_t ml = split_lo2(hm, mh);
                bre_h[nt][i] = rh[0];
                bre_h[nt][i + 1] = rh[1];
                bre_l[nt][i] = rl[0];
                bre_l[nt][i + 1] = rl[1];
                bim_h[nt][i] = mh[0];
                bim_h[nt][i + 1] = mh[1];
                bim_l[nt][i] = ml[0];
                bim_l[nt][i + 1] = ml[1];
            }
            dc[nt][0] += sre;
            dc[nt][1] += sim;
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const half8 ah = *reinterpret_cast<const half8 *>(&chi[(mt * 64 + lane) * 8]);
            const half8 al = *reinterpret_cast<const half8 *>(&clo[(mt * 64 + lane) * 8]);
#pragma unroll
            for (int nt = 0; nt < NTW; ++nt) {
                acc[mt][nt][0] = mfma_split(ah, al, bre_h[nt], bre_l[nt], acc[mt][nt][0]);
                acc[mt][nt][1] = mfma_split(ah, al, bim_h[nt], bim_l[nt], acc[mt][nt][1]);
            }
        }
        if ((c & ((1 << kDepDcLog) - 1)) == ((1 << kDepDcLog) - 1)) {
#pragma unroll
            for (int nt = 0; nt < NTW; ++nt) {
                dcd[(2 * nt) * 64] += (double)dc[nt][0];
                dcd[(2 * nt + 1) * 64] += (double)dc[nt][1];
                dc[nt][0] = dc[nt][1] = 0.f;
            }
        }
        __syncthreads();
      }
      if (ce < nchunks) {
#pragma unroll
          for (int mt = 0; mt < MT; ++mt)
#pragma unroll
              for (int nt = 0; nt < NTW; ++nt) {
                  acc[mt][nt][0] = -acc[mt][nt][0];
                  acc[mt][nt][1] = -acc[mt][nt][1];
              }
      }
    }

    // after chunk c the running sums carry the sign (-1)^((c >> kDepFlipLog) & 1)
    const int64_t last = nchunks - 1;
    const double fsign = last >= 0 && ((last >> kDepFlipLog) & 1) ? -1.0 : 1.0;
    const double outscale = unscale_mf * fsign;
    // FP32 partials (each already an FP32 sum; the splits are added in FP64)
    float *pb = part + (int64_t)split * (int64_t)n1 * 4 * Rpad;
#pragma unroll
    for (int nt = 0; nt < NTW; ++nt) {
        // n_z = 0: the four lane groups' sums, added in a fixed order
        double dre = dcd[(2 * nt) * 64] + (double)dc[nt][0], dim = dcd[(2 * nt + 1) * 64] + (double)dc[nt][1];
        dre += __shfl_xor(dre, 16, 64);
        dim += __shfl_xor(dim, 16, 64);
        dre += __shfl_xor(dre, 32, 64);
        dim += __shfl_xor(dim, 32, 64);
        const int r = row0 + nt * 16 + ln;
        if (!rok[nt]) continue;
        if (g == 0) {
            pb[0 * Rpad + r] = (float)(unscale_dc * dre);
            pb[1 * (int64_t)Rpad + r] = (float)(unscale_dc * dim);
            pb[2 * (int64_t)Rpad + r] = 0.f;
            pb[3 * (int64_t)Rpad + r] = 0.f;
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = mt * 16 + 4 * g + i;
                int nz, slot;
                if (m < n) {
                    nz = m + 1;
                    slot = 0;
                } else if (m < 2 * n) {
                    nz = m - n + 1;
                    slot = 2;
                } else {
                    continue;
                }
                pb[((int64_t)nz * 4 + slot) * Rpad + r] = (float)(outscale * (double)acc[mt][nt][0][i]);
                pb[((int64_t)nz * 4 + slot + 1) * Rpad + r] = (float)(outscale * (double)acc[mt][nt][1][i]);
            }
        }
    }
}

template <int MT>
static constexpr size_t deposit_mfma_lds_mt()
{
    return 2 * dep_buf_bytes<MT>() + (size_t)kDepCompW * dep_ntw(MT) * 2 * 64 * sizeof(double);
}

size_t deposit_mfma_lds(int n)
{
    switch (mfma_cs_tiles(n)) {
    case 1: return deposit_mfma_lds_mt<1>();
    case 2: return deposit_mfma_lds_mt<2>();
    case 3: return deposit_mfma_lds_mt<3>();
    case 4: return deposit_mfma_lds_mt<4>();
    case 5: return deposit_mfma_lds_mt<5>();
    case 6: return deposit_mfma_lds_mt<6>();
    case 7: return deposit_mfma_lds_mt<7>();
    default: return deposit_mfma_lds_mt<8>();
    }
}

// Particle splits: one block per (row block, split) holds a whole CU (16
// waves, 96 KB of LDS at n_max = 32), so the grid runs in rounds of one block
// per CU.  The split count is a multiple of kXcds (the XCD-aware numbering
// needs whole groups) chosen to minimise rounds per particle, i.e. to avoid a
// last round that is nearly empty; ties go to fewer splits (fewer partials).
// A split holds at most kDepMaxRun particles: its matrix-core sums run in FP32
// over the whole split, so their length is bounded whatever N is (more
// particles mean more splits and FP64 cross-split sums instead).
constexpr int64_t kDepMaxRun = 8192;
MfmaDepositPlan plan_deposit_mfma(const Geom &g, int64_t N)
{
    MfmaDepositPlan p;
    const int rpb = dep_rows_per_block(mfma_cs_tiles(g.n));
    p.row_blocks = (g.R + rpb - 1) / rpb;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus < 1) cus = 256;
    const int64_t smax = N / 512 >= kXcds ? (N / 512) / kXcds * kXcds : 0;
    int64_t splits = N / 512 > 1 ? N / 512 : 1;  // small N: fewer splits than one XCD group
    // fewest splits that keep every run within kDepMaxRun, in whole XCD groups
    const int64_t smin = ((N + kDepMaxRun - 1) / kDepMaxRun + kXcds - 1) / kXcds * kXcds;
    if (smax >= kXcds) {
        double best = 1e300;
        for (int64_t sp = smin > kXcds ? smin : kXcds; sp <= smax && sp <= (int64_t)1 << 20; sp += kXcds) {
            const int64_t blocks = (int64_t)p.row_blocks * sp;
            const double cost = (double)((blocks + cus - 1) / cus) / (double)sp;
            if (cost < best * (1.0 - 1e-9)) {
                best = cost;
                splits = sp;
            }
        }
    }
    int64_t per = (N + splits - 1) / splits;
    per = (per + kDepChunk - 1) / kDepChunk * kDepChunk;
    p.per_split = per;
    p.splits = (int)((N + per - 1) / per);
    // Feistel half width h: 2^(2h) >= N
    int h = 0;
    while (h < 16 && ((int64_t)1 << (2 * h)) < N) ++h;
    p.perm = h;
    return p;
}

template <int MT>
static void launch_dep_mt(hipStream_t s, const float *rec, int64_t N, const Geom &g,
                          const MfmaDepositPlan &pl, double unscale_mf, double unscale_dc,
                          float *part)
{
    // splits rounded up to whole groups of kXcds; blocks past the last split return
    const int groups = (pl.splits + kXcds - 1) / kXcds;
    hipLaunchKernelGGL(k_deposit_mfma<MT>, dim3(groups * kXcds * pl.row_blocks), dim3(kDepThreads),
                       deposit_mfma_lds(g.n), s, rec, N, g.n, g.R, g.Rpad, pl.per_split,
                       pl.row_blocks, pl.splits, unscale_mf, unscale_dc, part);
}

size_t deposit_mfma_rec_bytes(int64_t N, int n) { return (size_t)N * dep_rec_floats(n) * sizeof(float); }

hipError_t launch_deposit_mfma(hipStream_t s, const double *pos, const double *q, int64_t N,
                               const Geom &g, double L, const MfmaDepositPlan &pl, double qscale,
                               float *rec, float *part)
{
    const dim3 pg((unsigned)((N + 255) / 256));
    const double qf = (double)kDepOpScale / qscale;
    const int hp = (int)pl.perm;
    switch ((g.n + 1 + 7) / 8) {
    case 1: hipLaunchKernelGGL(k_deposit_prep<1>, pg, dim3(256), 0, s, pos, q, N, 1.0 / L, hp, qf, rec); break;
    case 2: hipLaunchKernelGGL(k_deposit_prep<2>, pg, dim3(256), 0, s, pos, q, N, 1.0 / L, hp, qf, rec); break;
    case 3: hipLaunchKernelGGL(k_deposit_prep<3>, pg, dim3(256), 0, s, pos, q, N, 1.0 / L, hp, qf, rec); break;
    case 4: hipLaunchKernelGGL(k_deposit_prep<4>, pg, dim3(256), 0, s, pos, q, N, 1.0 / L, hp, qf, rec); break;
    case 5: hipLaunchKernelGGL(k_deposit_prep<5>, pg, dim3(256), 0, s, pos, q, N, 1.0 / L, hp, qf, rec); break;
    case 6: hipLaunchKernelGGL(k_deposit_prep<6>, pg, dim3(256), 0, s, pos, q, N, 1.0 / L, hp, qf, rec); break;
    case 7: hipLaunchKernelGGL(k_deposit_prep<7>, pg, dim3(256), 0, s, pos, q, N, 1.0 / L, hp, qf, rec); break;
    case 8: hipLaunchKernelGGL(k_deposit_prep<8>, pg, dim3(256), 0, s, pos, q, N, 1.0 / L, hp, qf, rec); break;
    default: hipLaunchKernelGGL(k_deposit_prep<9>, pg, dim3(256), 0, s, pos, q, N, 1.0 / L, hp, qf, rec); break;
    }
    // H carries q / qscale scaled by 7/8, the CS operand another 7/8
    const double unscale_dc = qscale / (double)kDepOpScale;
    const double unscale_mf = unscale_dc / (double)kDepOpScale;
    switch (mfma_cs_tiles(g.n)) {
    case 1: launch_dep_mt<1>(s, rec, N, g, pl, unscale_mf, unscale_dc, part); break;
    case 2: launch_dep_mt<2>(s, rec, N, g, pl, unscale_mf, unscale_dc, part); break;
    case 3: launch_dep_mt<3>(s, rec, N, g, pl, unscale_mf, unscale_dc, part); break;
    case 4: launch_dep_mt<4>(s, rec, N, g, pl, unscale_mf, unscale_dc, part); break;
    case 5: launch_dep_mt<5>(s, rec, N, g, pl, unscale_mf, unscale_dc, part); break;
    case 6: launch_dep_mt<6>(s, rec, N, g, pl, unscale_mf, unscale_dc, part); break;
    case 7: launch_dep_mt<7>(s, rec, N, g, pl, unscale_mf, unscale_dc, part); break;
    default: launch_dep_mt<8>(s, rec, N, g, pl, unscale_mf, unscale_dc, part); break;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ force table pack
// The force visits rows in quads of 4 (one row per lane group), in runs that
// hold one coordinate fixed, so that a lane's row phase advances by the same
// step at every quad of a run: first line 0 (n_x = 0, n_y = 0..n, q0 quads,
// n_y of lane group i = 4 t + i), then, in a three-dimensional context, one
// column per n_y = -n..n with n_x = 1..n (qC quads each, n_x of lane group i
// = 4 t' + i + 1).  Runs are padded to whole quads (a column needs no padding
// when 4 divides n), and the row arrays further to a multiple of
// kForceQuadAlign quads (whole LDS stages of the force kernel).  Padding rows
// carry zero weights.
constexpr int kForceQuadAlign = 8;
// quads per LDS stage of the force kernel for KS K steps of 32
template <int KS>
constexpr int force_tm() { return 8; }

struct ForceQuads {
    int q0, qC, Q, Qpad;  // quads of line 0, per column, in all
};

// lines = n + 1 in three dimensions (line 0 and 2n + 1 columns), 1 in two
// (line 0 only)
__host__ __device__ inline ForceQuads force_quads(int n, int lines)
{
    ForceQuads f;
    f.q0 = (n + 1 + 3) / 4;
    f.qC = (n + 3) / 4;
    f.Q = f.q0 + (lines > 1 ? (2 * n + 1) * f.qC : 0);
    f.Qpad = (f.Q + kForceQuadAlign - 1) / kForceQuadAlign * kForceQuadAlign;
    return f;
}

// padded row pr = 4 t + i (quad t, lane group i) -> row of the row layout, or
// -1 for a padding row; (nx, ny) of the row
__host__ __device__ inline int force_row(int pr, int n, const ForceQuads &f, int &nx, int &ny)
{
    const int t = pr >> 2, i = pr & 3;
    if (t >= f.Q) return -1;
    if (t < f.q0) {
        nx = 0;
        ny = 4 * t + i;
        return ny <= n ? ny : -1;
    }
    const int c = (t - f.q0) / f.qC;
    nx = 4 * ((t - f.q0) - c * f.qC) + i + 1;
    ny = c - n;
    return nx <= n ? (n + 1) + (nx - 1) * (2 * n + 1) + c : -1;
}

// Per padded row, two records of four floats:
//   A = (Re psi(r, 0) / s, Im psi(r, 0) / s, 0, 0): the matrix core's starting
//       accumulator of (Re U0, Im U0, Re U1, Im U1) / s, so the n_z = 0 term
//       costs no vector instruction;
//   B = (n_x s, n_y s, s, 0): the weights of Im(g U0) / s in F_x and F_y, and
//       of Im(g U1) / s in F_z.
// s is the power of two at or above the row's largest |entry| (1 for an
// all-zero row), so that every entry enters FP16 with magnitude <= 1 and small
// rows keep their own relative precision; power-of-two scaling is exact.  s is
// kept within the normal FP32 range, and no smaller than 2^-60 |psi(r, 0)| so
// that psi / s stays far from overflow.  Records are stored interleaved,
// rinfo[2 pr] = A, rinfo[2 pr + 1] = B, for 4 Qpad padded rows.
__global__ void __launch_bounds__(256)
k_force_rows(const float *__restrict__ ftab, const float *__restrict__ psi0, int n, int lines,
             int nzp, float4 *__restrict__ rinfo)
{
    // one wave per padded row: the row's table entries read by the 64 lanes
    // together, their largest magnitude by a butterfly
    const ForceQuads f = force_quads(n, lines);
    const int pr = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (pr >= 4 * f.Qpad) return;
    int nx = 0, ny = 0;
    const int r = force_row(pr, n, f, nx, ny);
    if (r < 0) {
        if (lane == 0) {
            rinfo[2 * pr] = make_float4(0.f, 0.f, 0.f, 0.f);
            rinfo[2 * pr + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        return;
    }
    float m = 0.f;
    const float *fr = ftab + (int64_t)r * nzp * 8;
    for (int i = lane; i < n * 8; i += 64) m = fmaxf(m, fabsf(fr[i]));
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if (lane != 0) return;
    const float pre = psi0[2 * r], pim = psi0[2 * r + 1];
    m = fmaxf(m, ldexpf(fmaxf(fabsf(pre), fabsf(pim)), -60));
    int e = 0;
    if (m > 0.f) {
        frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
        e = e < -126 ? -126 : (e > 126 ? 126 : e);
    }
    const float s = m > 0.f ? ldexpf(1.0f, e) : 1.0f;
    const float inv = m > 0.f ? ldexpf(1.0f, -e) : 1.0f;
    rinfo[2 * pr] = make_float4(pre * inv, pim * inv, 0.f, 0.f);
    rinfo[2 * pr + 1] = make_float4((float)nx * s, (float)ny * s, s, 0.f);
}

// W fragments: wf[t][s][h][lane][8] halves, t = quad (< Qpad), s = K step, h = hi/lo.
// Lane l, element i: A row m = l % 16 -> padded row 4t + m/4, component
// e = m % 4; K index k = 32 s + 8 (l/16) + i -> cos (k < nzk) or sin of
// n_z = (k mod nzk) + 1.
__global__ void __launch_bounds__(256)
k_force_pack(const float *__restrict__ ftab, const float4 *__restrict__ rinfo, int n, int lines,
             int nzp, int nzk, int ks, _Float16 *__restrict__ wf)
{
    const ForceQuads f = force_quads(n, lines);
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t total = (int64_t)f.Qpad * ks * 64;
    if (gid >= total) return;
    const int lane = (int)(gid & 63);
    const int64_t ts = gid >> 6;
    const int s = (int)(ts % ks);
    const int t = (int)(ts / ks);
    const int mrow = lane & 15;
    const int pr = 4 * t + (mrow >> 2);
    const int e = mrow & 3;
    int nx, ny;
    const int r = force_row(pr, n, f, nx, ny);
    const float inv = r >= 0 ? 1.0f / rinfo[2 * pr + 1].z : 1.0f;
    _Float16 hi[8], lo[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = 32 * s + 8 * (lane >> 4) + i;
        const bool is_sin = k >= nzk;
        const int nz = (is_sin ? k - nzk : k) + 1;
        float v = 0.f;
        if (r >= 0 && nz <= n) {
            const float *fe = ftab + ((int64_t)r * nzp + (nz - 1)) * 8;
            // fe: sig_r sig_i del_r del_i nz*del_r nz*del_i nz*sig_r nz*sig_i
            switch (e) {
            case 0: v = is_sin ? -fe[3] : fe[0]; break;  // Re U0: sig_r cos - del_i sin
            case 1: v = is_sin ? fe[2] : fe[1]; break;   // Im U0: sig_i cos + del_r sin
            case 2: v = is_sin ? -fe[7] : fe[4]; break;  // Re U1: nz (del_r cos - sig_i sin)
            default: v = is_sin ? fe[6] : fe[5]; break;  // Im U1: nz (del_i cos + sig_r sin)
            }
        }
        split_f16(v * inv, hi[i], lo[i]);
    }
    _Float16 *o = wf + ((((int64_t)t * ks + s) * 2) * 64 + lane) * 8;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        o[i] = hi[i];
        o[64 * 8 + i] = lo[i];
    }
}

size_t force_rowinfo_bytes(const Geom &g) { return (size_t)2 * 4 * force_quads(g.n, g.lines).Qpad * sizeof(float4); }

hipError_t launch_force_pack(hipStream_t s, const float *ftab, const float *psi0, const Geom &g,
                             float4 *rinfo, _Float16 *wf)
{
    const ForceQuads f = force_quads(g.n, g.lines);
    hipLaunchKernelGGL(k_force_rows, dim3((unsigned)f.Qpad), dim3(256), 0, s, ftab, psi0, g.n,
                       g.lines, g.nzp, rinfo);
    const int nzk = (g.n + 15) / 16 * 16;
    const int ks = nzk / 16;
    const int64_t total = (int64_t)f.Qpad * ks * 64;
    hipLaunchKernelGGL(k_force_pack, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, ftab,
                       rinfo, g.n, g.lines, g.nzp, nzk, ks, wf);
    return hipGetLastError();
}

// ------------------------------------------------------------------ force
// Block = 8 waves x 32 particles (NT = 2 N tiles of 16 particles per wave).
// The W fragments and row records of kForceTM quads at a time (a stage) are
// copied into LDS for the whole block with direct global-to-LDS loads, double
// buffered in two separate LDS arrays: the next stage streams into one while
// the current one is multiplied out of the other, one barrier per stage.  The
// quads are padded to whole stages (the padding contributes zero), so every
// stage runs the same fixed loop.  (With
// the buffers as distinct objects the compiler can tell that reads of the
// current one need not wait for the copies into the other.)  Every wave keeps
// its particles' CS fragments in registers.  Lane group g = l/16 handles row
// 4t + g of each quad t, so the four groups sum disjoint rows of the same
// particles and are combined at the end.  The matrix products of quad t+1 are
// issued before the epilogue of quad t.
//
// The epilogue of a (quad, 16-particle tile) is 11 vector instructions: with
// the accumulator started at psi(r, 0) / s (record A), the matrix core returns
// (U0, U1) / s, and
//   Im(g U0) / s, Im(g U1) / s       4
//   F += (n_x s, n_y s, s) (...)     3   (record B)
//   g <- g e4                        4
// where g = exp(2 pi i (n_x t_x + n_y t_y)) is the lane's row phase in FP32
// and e4 = cis(4 theta_y) along line 0, cis(4 theta_x) along the columns (the
// lane's copy waits in LDS until line 0 ends).  Quads never cross runs, so the
// step is the same for every lane.  At each run end the FP32 sums go into
// FP64 and g restarts from the next column's phase, kept by an FP64 complex
// recurrence in t_y (exact to ~1e-15 over all columns), so FP32 phase steps
// never run longer than one run.  PHI: also sum the potential (the
// diagnostics and finite-width field shapes need it).
constexpr int kForceWaves = 8;
constexpr int kForceNT = 2;
constexpr int kForceBlockParticles = kForceWaves * kForceNT * 16;

// Copy pieces [0, npieces) of 64 half8 (1 KB) from src to LDS dst, piece p by
// wave p % kForceWaves: lane l moves the 16 bytes at src[64 p + l] to dst[64 p + l].
__device__ inline void stage_w(const half8 *__restrict__ src, half8 *dst, int npieces, int wave,
                               int lane)
{
    for (int p = wave; p < npieces; p += kForceWaves)
        __builtin_amdgcn_global_load_lds(
            (const void *)(src + 64 * p + lane),
            (__attribute__((address_space(3))) void *)(dst + 64 * p), 16, 0, 0);
}

// For KS <= 2 the launch bound asks for 4 waves per SIMD (two blocks per CU):
// without it the variant that also sums the potential takes 132 VGPRs at
// KS = 2 and runs 3 waves per SIMD; with it the compiler schedules it into 126
// without spills.  KS = 3, 4 need more than 128 VGPRs and run 2 waves per SIMD.
template <int KS, bool PHI>
__global__ void __launch_bounds__(64 * kForceWaves, KS <= 2 ? 4 : 2)
k_force_mfma(const double *__restrict__ pos, const double *__restrict__ q,
             const double *__restrict__ m, double *__restrict__ vel, const _Float16 *__restrict__ wf,
             const float4 *__restrict__ rinfo, int n, int lines, double invL, int64_t N, double kick,
             double *__restrict__ F, double *__restrict__ phi)
{
    constexpr int NT = kForceNT;
    constexpr int kForceTM = force_tm<KS>();
    constexpr int kForceRecWaves = (8 * kForceTM + 63) / 64;  // waves that load a stage's row records
    static_assert(kForceRecWaves <= kForceWaves && kForceTM % 2 == 0 && kForceQuadAlign % kForceTM == 0,
                  "stage shape");
    constexpr int PIECES = kForceTM * KS * 2;          // 1 KB W pieces per stage
    constexpr int STAGE = PIECES * 64 + 8 * kForceTM;  // half8 per stage buffer (W, records A, B)
    __shared__ half8 wbuf0[STAGE], wbuf1[STAGE];
    __shared__ float2 e4x[NT][64 * kForceWaves];  // each lane's cis(4 theta_x)

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int g = lane >> 4;
    const int ln = lane & 15;
    const int nzk = 16 * KS;
    const ForceQuads fq = force_quads(n, lines);
    const half8 *wsrc = reinterpret_cast<const half8 *>(wf);
    const half8 *isrc = reinterpret_cast<const half8 *>(rinfo);
    const int nstage = fq.Qpad / kForceTM;  // padding quads contribute zero

    auto stage = [&](int st, half8 *dst) {
        const int t0 = st * kForceTM;
        stage_w(wsrc + (int64_t)t0 * KS * 2 * 64, dst, PIECES, wave, lane);
        // the interleaved records A, B of the stage's 4 kForceTM rows, one per
        // lane (the array is padded to whole stages)
        const int rw = wave - (kForceWaves - kForceRecWaves);
        if (rw >= 0 && 64 * rw + lane < 8 * kForceTM)
            __builtin_amdgcn_global_load_lds((const void *)(isrc + 8 * t0 + 64 * rw + lane),
                                             (__attribute__((address_space(3))) void *)(dst + PIECES * 64 + 64 * rw),
                                             16, 0, 0);
    };
    // first stage in flight while the particle fragments are formed
    stage(0, wbuf0);

    half8 bh[NT][KS], bl[NT][KS];
    float gc[NT], gs[NT], e4c[NT], e4s[NT];
    double lc[NT], ls[NT], stc[NT], sts[NT];  // next column's phase; step cis(t_y)
    double fx[NT], fy[NT], fz[NT], fp[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        const int64_t j = (int64_t)blockIdx.x * kForceBlockParticles + wave * (NT * 16) + nt * 16 + ln;
        const int64_t jc = j < N ? j : N - 1;
        const double tx = frac(pos[jc] * invL);
        const double ty = frac(pos[N + jc] * invL);
        const double tz = frac(pos[2 * N + jc] * invL);
        double ezc, ezs;
        cis_turns(tz, ezc, ezs);
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            // k = 32 s + 8 g + i: cos for k < nzk, else sin; n_z consecutive in i
            const int k0 = 32 * s + 8 * g;
            const bool is_sin = k0 >= nzk;
            const int nz0 = (is_sin ? k0 - nzk : k0) + 1;
            double c, sn;
            cis_turns(frac_mul(nz0, tz), c, sn);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                _Float16 h, l;
                split_f16((float)(is_sin ? sn : c), h, l);
                bh[nt][s][i] = h;
                bl[nt][s][i] = l;
                const double t = c * ezc - sn * ezs;
                sn = sn * ezc + c * ezs;
                c = t;
            }
        }
        double a, b;
        cis_turns(frac_mul(4, ty), a, b);
        e4c[nt] = (float)a;
        e4s[nt] = (float)b;
        cis_turns(frac_mul(4, tx), a, b);
        e4x[nt][tid] = make_float2((float)a, (float)b);
        // line 0 starts at n_y = g; the first column at (n_x, n_y) = (g + 1, -n)
        cis_turns(frac_mul(g, ty), a, b);
        gc[nt] = (float)a;
        gs[nt] = (float)b;
        cis_turns(frac_lin(g + 1, tx, -n, ty), lc[nt], ls[nt]);
        cis_turns(ty, stc[nt], sts[nt]);
        fx[nt] = fy[nt] = fz[nt] = fp[nt] = 0.0;
    }
    float sx[NT], sy[NT], sz[NT], sp[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) sx[nt] = sy[nt] = sz[nt] = sp[nt] = 0.f;
    int next_run = fq.q0;  // first quad of the next run

    auto products = [&](const half8 *wl, int tt, f32x4 (&acc)[NT]) {
        half8 ah[KS], al[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            ah[s] = wl[((tt * KS + s) * 2 + 0) * 64 + lane];
            al[s] = wl[((tt * KS + s) * 2 + 1) * 64 + lane];
        }
        const float4 ci = reinterpret_cast<const float4 *>(wl + PIECES * 64)[2 * (4 * tt + g)];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            acc[nt] = f32x4{ci.x, ci.y, ci.z, ci.w};
#pragma unroll
            for (int s = 0; s < KS; ++s) acc[nt] = mfma_split(ah[s], al[s], bh[nt][s], bl[nt][s], acc[nt]);
        }
    };
    auto epilogue = [&](const half8 *wl, int tt, int t, const f32x4 (&acc)[NT]) {
        const float4 w = reinterpret_cast<const float4 *>(wl + PIECES * 64)[2 * (4 * tt + g) + 1];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const float im0 = gc[nt] * acc[nt][1] + gs[nt] * acc[nt][0];
            const float im1 = gc[nt] * acc[nt][3] + gs[nt] * acc[nt][2];
            sx[nt] = fmaf(w.x, im0, sx[nt]);
            sy[nt] = fmaf(w.y, im0, sy[nt]);
            sz[nt] = fmaf(w.z, im1, sz[nt]);
            if (PHI) sp[nt] = fmaf(w.z, gc[nt] * acc[nt][0] - gs[nt] * acc[nt][1], sp[nt]);
            const float c = gc[nt] * e4c[nt] - gs[nt] * e4s[nt];
            gs[nt] = gs[nt] * e4c[nt] + gc[nt] * e4s[nt];
            gc[nt] = c;
        }
        if (t + 1 == next_run) {
            // end of a run: FP32 sums into FP64, phase of the next column's first row
            if (t + 1 == fq.q0) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const float2 e = e4x[nt][tid];
                    e4c[nt] = e.x;
                    e4s[nt] = e.y;
                }
            }
            next_run += fq.qC;
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                fx[nt] += (double)sx[nt];
                fy[nt] += (double)sy[nt];
                fz[nt] += (double)sz[nt];
                if (PHI) fp[nt] += (double)sp[nt];
                sx[nt] = sy[nt] = sz[nt] = sp[nt] = 0.f;
                gc[nt] = (float)lc[nt];
                gs[nt] = (float)ls[nt];
                const double c = lc[nt] * stc[nt] - ls[nt] * sts[nt];
                ls[nt] = lc[nt] * sts[nt] + ls[nt] * stc[nt];
                lc[nt] = c;
            }
        }
    };
    auto run_stage = [&](int st, const half8 *wl, half8 *next) {
        const int t0 = st * kForceTM;
        if (st + 1 < nstage) stage(st + 1, next);
        // quads of the stage to multiply out: the whole stage but in the last
        // one, whose padding quads past Q (zero weights) are skipped but for
        // the one that completes a pair
        const int cnt = fq.Q - t0 >= kForceTM ? kForceTM : ((fq.Q - t0 + 1) & ~1);
        f32x4 accA[NT], accB[NT];
        products(wl, 0, accA);
#pragma unroll 1
        for (int tt = 0; tt < cnt; tt += 2) {
            products(wl, tt + 1, accB);
            epilogue(wl, tt, t0 + tt, accA);
            if (tt + 2 < cnt) products(wl, tt + 2, accA);
            epilogue(wl, tt + 1, t0 + tt + 1, accB);
        }
        // the next stage's copies have landed, and every wave is done with this one
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    };

    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int st = 0; st < nstage; st += 2) {
        run_stage(st, wbuf0, wbuf1);
        if (st + 1 < nstage) run_stage(st + 1, wbuf1, wbuf0);
    }
    // combine the four lane groups (same particles, disjoint rows)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        for (int o = 16; o <= 32; o <<= 1) {
            fx[nt] += __shfl_xor(fx[nt], o, 64);
            fy[nt] += __shfl_xor(fy[nt], o, 64);
            fz[nt] += __shfl_xor(fz[nt], o, 64);
            if (PHI) fp[nt] += __shfl_xor(fp[nt], o, 64);
        }
        const int64_t j = (int64_t)blockIdx.x * kForceBlockParticles + wave * (NT * 16) + nt * 16 + ln;
        if (g == 0 && j < N) {
            const double f = 2.0 * q[j] * (6.283185307179586476925286766559 * invL);
            const double Fx = f * fx[nt], Fy = f * fy[nt], Fz = f * fz[nt];
            if (F) {
                F[j] = Fx;
                F[N + j] = Fy;
                F[2 * N + j] = Fz;
            }
            if (PHI) phi[j] = 2.0 * fp[nt];
            if (kick != 0.0) {
                const double a = kick / m[j];
                vel[j] += a * Fx;
                vel[N + j] += a * Fy;
                vel[2 * N + j] += a * Fz;
            }
        }
    }
}

template <int KS>
static void launch_force_ks(hipStream_t s, dim3 grid, dim3 block, const double *pos, const double *q,
                            const double *m, double *vel, const _Float16 *wf, const float4 *rinfo,
                            int n, int lines, double invL, int64_t N, double kick, double *F,
                            double *phi)
{
    if (phi)
        hipLaunchKernelGGL((k_force_mfma<KS, true>), grid, block, 0, s, pos, q, m, vel, wf, rinfo, n,
                           lines, invL, N, kick, F, phi);
    else
        hipLaunchKernelGGL((k_force_mfma<KS, false>), grid, block, 0, s, pos, q, m, vel, wf, rinfo, n,
                           lines, invL, N, kick, F, phi);
}

hipError_t launch_force_mfma(hipStream_t s, const double *pos, const double *q, const double *m,
                             double *vel, const _Float16 *wf, const float4 *rinfo, const Geom &g,
                             double L, int64_t N, double kick, double *F, double *phi)
{
    const int ks = (g.n + 15) / 16;
    const int64_t blocks = (N + kForceBlockParticles - 1) / kForceBlockParticles;
    const dim3 grid((unsigned)blocks), block(64 * kForceWaves);
    switch (ks) {
    case 1: launch_force_ks<1>(s, grid, block, pos, q, m, vel, wf, rinfo, g.n, g.lines, 1.0 / L, N, kick, F, phi); break;
    case 2: launch_force_ks<2>(s, grid, block, pos, q, m, vel, wf, rinfo, g.n, g.lines, 1.0 / L, N, kick, F, phi); break;
    case 3: launch_force_ks<3>(s, grid, block, pos, q, m, vel, wf, rinfo, g.n, g.lines, 1.0 / L, N, kick, F, phi); break;
    default: launch_force_ks<4>(s, grid, block, pos, q, m, vel, wf, rinfo, g.n, g.lines, 1.0 / L, N, kick, F, phi); break;
    }
    return hipGetLastError();
}

size_t force_pack_bytes(const Geom &g)
{
    const int ks = (g.n + 15) / 16;
    return (size_t)force_quads(g.n, g.lines).Qpad * ks * 2 * 64 * 8 * sizeof(_Float16);
}

}  // namespace sce
