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

// lo parts of two values x whose hi parts (round to nearest) are packed in
// hi: lo = fp16(x - hi), x - hi being exact in FP32.
__device__ inline half2_t split_lo2(float2_t x, half2_t hi)
{
    const float2_t d = {x[0] - (float)hi[0], x[1] - (float)hi[1]};
    return __builtin_convertvector(d, half2_t);
}

__device__ inline f32x4 mfma16(half8 a, half8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// acc += (ah + al)(bh + bl) without the al*bl term.
//
// The kernels issue each accumulator's products back to back
// (a dependent chain) rather than interleaving accumulators.  The matrix
// core then runs measurably faster on this power-limited chip: a probe of
// 16 accumulators per wave reached 2.11 PFLOP/s chained against 1.82
// interleaved, and the split force at 2^20 particles took 2.54 instead of
// 2.69 ms (the deposit 1.71 instead of 1.77), bit for bit the same sums.
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
// walking back into [0, N).  Slot s of the visiting order holds particle
// feistel_fwd(s).

// ------------------------------------------------------------------ deposit
// Particles are taken in chunks of 32 (the K depth of one matrix instruction).
constexpr int kDepChunk = 32;
// Both deposit operands are multiplied by 7/8 before the split (and the
// result by 64/49 in FP64).  Unscaled, cos(n_z theta) and the x-y products
// crowd just below 1.0 for particles near the origin, where round-to-nearest
// FP16 gives hi = 1 and a negative lo in both operands: the dropped lo*lo term
// then has a consistent sign and acts like a spurious charge at the origin.
// At 7/8 no operand sits at an FP16 exponent boundary and the lo parts are
// unbiased.
constexpr float kDepOpScale = 0.875f;
// The matrix core rounds its FP32 accumulation per group of products and, when
// the running sum is much larger than each increment, slightly toward -inf.
// Over thousands of chunks that directional bias is identical in every
// accumulator and would act like a spurious charge at the origin.  The running
// sum therefore changes sign every 2^kDepFlipLog chunks (accumulator and CS
// operand negated together), so the bias alternates direction and cancels.
constexpr int kDepFlipLog = 3;
// FP32 sums of the n_z = 0 row are added into FP64 every 2^kDepDcLog chunks.
constexpr int kDepDcLog = 4;

__host__ __device__ inline uint32_t feistel_round(uint32_t x, int r)
{
    uint32_t f = x * 0x9E3779B1u + 0x7F4A7C15u * (uint32_t)(r + 1);
    f ^= f >> 15;
    f *= 0x85EBCA6Bu;
    f ^= f >> 13;
    return f;
}

// The visiting-order map: slot s -> particle, rounds applied in order and
// repeated while the result lies outside [0, N) (cycle walking).
__host__ __device__ inline uint32_t feistel_fwd(uint32_t s, uint32_t N, int h)
{
    const uint32_t mask = h >= 16 ? 0xFFFFu : ((1u << h) - 1u);
    uint32_t y = s;
    do {
        uint32_t L = y >> h, R = y & mask;
        for (int r = 0; r < 4; ++r) {
            const uint32_t nr = (L ^ feistel_round(R, r)) & mask;
            L = R;
            R = nr;
        }
        y = (L << h) | R;
    } while (y >= N);
    return y;
}

// Chunk image: the LDS tables of one chunk of 32 particles p of the visiting
// order, exactly as the matrix-core kernel reads them (it copies images into
// LDS unchanged):
//   CS hi, CS lo: the A operand, cos and sin(2 pi n_z t_z) for n_z = 1..n
//       (rows 0..n-1 and n..2n-1, zero rows up to 16 MT), times the running-sum
//       sign and 7/8, as FP16 halves in the matrix core's fragment order
//       (cs_idx), so that a lane's 16-byte fragment read sits at 16 lane +
//       const: 16-byte LDS reads run at full rate only when the lanes'
//       addresses are consecutive;
//   X[p][k] = q' (cos, sin)(2 pi k t_x), k = 0..n, q' = (7/8) q / max|q|;
//   Y[p][k] = (cos, sin)(2 pi k t_y), k = 0..n.
// X and Y rows have a compile-time stride (k = 0..8 MT, the largest n_max of
// the tile class) rounded up to 2 (mod 4) float2 entries, so the rows of
// particles p and p + 8, which lane groups 0/1 (and 2/3) read in the same pass
// of an 8-byte read, start 128 bytes apart modulo the 256-byte bank cycle.
// An image is a whole number of KB.
template <int MT>
struct DepTab {
    static constexpr int kmax = 8 * MT + 1;
    static constexpr int sxy = kmax + (6 - kmax % 4) % 4;  // = 2 (mod 4)
    static constexpr int cs_halves = MT * 16 * kDepChunk;   // one of hi, lo
    static constexpr size_t x_off = (size_t)2 * cs_halves * sizeof(_Float16);
    static constexpr size_t y_off = x_off + (size_t)kDepChunk * sxy * sizeof(float2);
    static constexpr size_t bytes = y_off + (size_t)kDepChunk * sxy * sizeof(float2);
    static_assert(bytes % 1024 == 0, "whole KB");
};
// CS element (row, particle p of the chunk) in fragment order: tile mt =
// row / 16 holds 64 lanes x 8 halves, lane = row % 16 + 16 (p / 8), half p % 8.
__host__ __device__ inline int cs_idx(int row, int p)
{
    return (row >> 4) * 512 + (p >> 3) * 128 + (row & 15) * 8 + (p & 7);
}

// CS rows of the matrix-core operand: cos(n_z theta) for n_z = 1..n (rows
// 0..n-1), sin(n_z theta) for n_z = 1..n (rows n..2n-1), zero padding to 16s.
// The n_z = 0 row (all ones) is summed on the VALU instead.
__host__ __device__ inline int mfma_cs_tiles(int n) { return (2 * n + 15) / 16; }
// CS tiles per matrix-core wave: all of them up to 4 (n_max <= 32), else the
// tiles are split over two waves that share the pairs.
__host__ __device__ constexpr int dep_mtw(int MT) { return MT <= 4 ? MT : (MT + 1) / 2; }
__host__ __device__ constexpr int dep_halves(int MT) { return MT <= 4 ? 1 : 2; }

size_t dep_image_bytes(int n)
{
    switch (mfma_cs_tiles(n)) {
    case 1: return DepTab<1>::bytes;
    case 2: return DepTab<2>::bytes;
    case 3: return DepTab<3>::bytes;
    case 4: return DepTab<4>::bytes;
    case 5: return DepTab<5>::bytes;
    case 6: return DepTab<6>::bytes;
    case 7: return DepTab<7>::bytes;
    default: return DepTab<8>::bytes;
    }
}

// One block of 4 waves per chunk image.  Tasks (axis d, block of 8 powers blk,
// particle p), particle fastest: a wave takes 64 tasks at a time, a pair of
// blocks of one axis (lanes 0-31 and 32-63), so its two half-waves never take
// different branches.  Each task takes its anchor cis(2 pi 8 blk t_d) (FP64)
// and step cis(2 pi t_d), formed once per particle and axis, and raises them
// to 8 powers by FP32 complex multiplication; the anchor carries the factor
// its table needs (q' for X, the running-sum sign and 7/8 for CS).  Slots past
// N hold q = 0.  cps: chunks per particle split (the running-sum sign counts a
// split's own chunks).
template <int MT>
__global__ void __launch_bounds__(256)
k_deposit_build(const double *__restrict__ pos, const double *__restrict__ q, int64_t N, int n,
                double invL, int h, double qfac, int64_t cps, float *__restrict__ img)
{
    using T = DepTab<MT>;
    __shared__ __align__(16) unsigned char sm[T::bytes];
    // per (axis, slot): the anchors cis(2 pi 8 b t) of the blocks of 8 powers
    // and the one-step factor cis(2 pi t)
    constexpr int NBMAX = MT + 1;
    __shared__ double2 anc[3][kDepChunk][NBMAX];
    __shared__ float2 stp[3][kDepChunk];
    __shared__ double qsl[kDepChunk];
    _Float16 *hi = reinterpret_cast<_Float16 *>(sm);
    _Float16 *lo = hi + T::cs_halves;
    float2 *tx = reinterpret_cast<float2 *>(sm + T::x_off);
    float2 *ty = reinterpret_cast<float2 *>(sm + T::y_off);
    const int64_t chunk = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n1 = n + 1, nb = (n1 + 7) / 8, npair = (nb + 1) / 2;
    for (int idx = tid; idx < (16 * MT - 2 * n) * kDepChunk; idx += 256) {
        const int e = cs_idx(2 * n + idx / kDepChunk, idx % kDepChunk);
        hi[e] = (_Float16)0.0f;
        lo[e] = (_Float16)0.0f;
    }
    const int64_t cl = chunk - (chunk / cps) * cps;
    const float csg = ((cl >> kDepFlipLog) & 1) ? -kDepOpScale : kDepOpScale;
    // One thread per (slot, axis) gathers its particle's coordinate, forms
    // e = cis(2 pi t) of its turns t = frac(x / L) (one FP64 sincos), e^8 by
    // three FP64 squarings and the anchors (e^8)^b by FP64 products, and
    // leaves them with q' in LDS for the tasks.
    if (tid < 3 * kDepChunk) {
        const int d = tid / kDepChunk, sl = tid - d * kDepChunk;
        const int64_t s = chunk * kDepChunk + sl;
        double t = 0.0, qq = 0.0;
        if (s < N) {
            const int64_t j = feistel_fwd((uint32_t)s, (uint32_t)N, h);
            t = frac(pos[d * N + j] * invL);
            if (d == 0) qq = q[j] * qfac;
        }
        double ec, es;
        cis_turns(t, ec, es);
        stp[d][sl] = make_float2((float)ec, (float)es);
        double e8c = ec, e8s = es;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const double c2 = e8c * e8c - e8s * e8s;
            e8s = 2.0 * e8c * e8s;
            e8c = c2;
        }
        double ac = 1.0, as = 0.0;
        for (int b = 0; b < nb; ++b) {
            anc[d][sl][b] = make_double2(ac, as);
            const double c2 = ac * e8c - as * e8s;
            as = ac * e8s + as * e8c;
            ac = c2;
        }
        if (d == 0) qsl[sl] = qq;
    }
    __syncthreads();
    const int p = lane & (kDepChunk - 1);
    for (int ws = wave; ws < 3 * npair; ws += 4) {
        const int d = ws / npair;
        const int blk = 2 * (ws - d * npair) + (lane >> 5);
        if (blk >= nb) continue;
        const double qq = qsl[p];
        const double2 an = anc[d][p][blk];
        const double ac = an.x, as = an.y;
        const float2 st = stp[d][p];
        const float c1 = st.x, s1 = st.y;
        const int k0 = 8 * blk;
        const int kend = n1 - k0 < 8 ? n1 - k0 : 8;
        if (d < 2) {
            // X_k = q' cis(2 pi k t_x) or Y_k = cis(2 pi k t_y)
            float uc = (float)(d == 0 ? qq * ac : ac), us = (float)(d == 0 ? qq * as : as);
            float2 *dst = (d == 0 ? tx : ty) + p * T::sxy + k0;
            for (int kk = 0; kk < kend; ++kk) {
                dst[kk] = make_float2(uc, us);
                const float tt = uc * c1 - us * s1;
                us = uc * s1 + us * c1;
                uc = tt;
            }
        } else {
            float2_t v;
            v[0] = csg * (float)ac;
            v[1] = csg * (float)as;
            for (int kk = 0; kk < kend; ++kk) {
                const int k = k0 + kk;
                if (k > 0) {
                    // (cos, sin) split two at a time
                    const half2_t hh = __builtin_convertvector(v, half2_t);
                    const half2_t ll = split_lo2(v, hh);
                    hi[cs_idx(k - 1, p)] = hh[0];
                    lo[cs_idx(k - 1, p)] = ll[0];
                    hi[cs_idx(n + k - 1, p)] = hh[1];
                    lo[cs_idx(n + k - 1, p)] = ll[1];
                }
                const float tt = v[0] * c1 - v[1] * s1;
                v[1] = v[0] * s1 + v[1] * c1;
                v[0] = tt;
            }
        }
    }
    // X and Y entries past n (up to the compile-time stride) are never read
    __syncthreads();
    const float4 *src = reinterpret_cast<const float4 *>(sm);
    float4 *dst = reinterpret_cast<float4 *>(img) + chunk * (int64_t)(T::bytes / 16);
    for (int i = tid; i < (int)(T::bytes / 16); i += 256) dst[i] = src[i];
}

// The sum is taken in real form.  With X_u, Y_v the cos (u, v = 0) and sin
// (1) tables of the x and y phases and Z_w those of z, the matrix core forms
// the eight real sums T_uvw(k_x, k_y, n_z) = sum_j X_u(k_x) Y_v(k_y) Z_w(n_z)
// over the block's particles for k_x, k_y = 0..n; every complex sum of the
// half space follows by signs, since exp(-i a) = cos a - i sin a:
//   P(k_x, +k_y, n_z) = T_ccc - T_ssc - i (T_scc + T_csc)
//   P(k_x, -k_y, n_z) = T_ccc + T_ssc + i (T_csc - T_scc)
// (P: w = c; Q, the sin(n_z) sums: w = s), which is the layout the
// reduction reads.  The B operand of a (k_x, k_y) pair is then one product
// per particle, X_u Y_v, formed and split into FP16 hi/lo by two
// mixed-precision FMAs on the exact FP32 product.
//
// Block = kDepWaves matrix-core waves for one (row block, particle split)
// pair; each wave owns 16 (k_x, k_y) pairs (one per lane of a 16-lane group)
// and their four B tiles uv = cc, cs, sc, ss, and lane group g takes particles
// 8g..8g+7 of a chunk.  The chunk images of the split stream into a ring of
// LDS buffers (three where they fit, else two) with direct global-to-LDS
// copies, the later chunks' in flight while the current one is multiplied
// out; one barrier per chunk.  The n_z = 0 sums (Z = 1) are accumulated on the
// VALU with one FMA per product.
constexpr int kDepWaves = 12;
constexpr int kDepThreads = 64 * kDepWaves;

// XCD-aware block order: consecutive blocks go to different XCDs (each with
// its own L2), so the grid is numbered such that the row blocks of one
// particle split are dispatched to the same XCD one after another and their
// reads of the split's chunk images hit that XCD's L2.  Linear block L runs on
// XCD L % 8; its position t = L / 8 in that XCD's sequence selects row block
// t % row_blocks of split (t / row_blocks) * 8 + L % 8.
constexpr int kXcds = 8;

// A table entry read as a volatile LDS double, which the compiler keeps as a
// read of its own.
typedef const volatile double __attribute__((address_space(3))) lds_f2;
__device__ inline float2 lds_read(lds_f2 *p)
{
    const double d = *p;
    return __builtin_bit_cast(float2, d);
}

template <bool B>
struct BoolC {
    static constexpr bool value = B;
};

template <int MT>
__global__ void __launch_bounds__(kDepThreads)
k_deposit_mfma(const float *__restrict__ img, int64_t N, int n, int lines, int Rpad,
               int64_t per_split, int row_blocks, int splits, double unscale_mf, double unscale_dc,
               float *__restrict__ part)
{
    using T = DepTab<MT>;
    const int blk_l = blockIdx.x;
    const int blk_t = blk_l / kXcds;
    const int rblk = blk_t % row_blocks;
    const int split = (blk_t / row_blocks) * kXcds + blk_l % kXcds;
    if (split >= splits) return;
    constexpr int MTW = dep_mtw(MT);
    constexpr int NH = dep_halves(MT);
    constexpr int SXY = T::sxy;
    constexpr int PIECES = (int)(T::bytes / 1024);
    // image buffers as separate static arrays: the copies into one never make
    // the reads of the others wait.  Three where they fit in LDS beside the
    // FP64 n_z = 0 sums (n_max <= 56), else two.
    constexpr size_t kDcBytes = (size_t)kDepWaves * 4 * 64 * sizeof(double);
    constexpr int NBUF = 3 * T::bytes + kDcBytes <= 160 * 1024 ? 3 : 2;
    __shared__ half8 buf0[T::bytes / 16], buf1[T::bytes / 16], buf2[NBUF == 3 ? T::bytes / 16 : 1];
    __shared__ double dcs[kDepWaves * 4 * 64];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t j0 = (int64_t)split * per_split;
    const int64_t j1 = j0 + per_split < N ? j0 + per_split : N;
    const int64_t nchunks = (j1 - j0 + kDepChunk - 1) / kDepChunk;
    const half8 *src = reinterpret_cast<const half8 *>(img) + (j0 / kDepChunk) * (int64_t)(T::bytes / 16);
    auto stage = [&](int64_t c, half8 *dst) {
        const half8 *sc = src + c * (int64_t)(T::bytes / 16);
        for (int pc = wave; pc < PIECES; pc += kDepWaves)
            __builtin_amdgcn_global_load_lds((const void *)(sc + 64 * pc + lane),
                                             (__attribute__((address_space(3))) void *)(dst + 64 * pc),
                                             16, 0, 0);
    };
    // images NBUF - 1 chunks ahead of the one being multiplied out
    stage(0, buf0);
    if (NBUF == 3 && nchunks > 1) stage(1, buf1);

    const int n1 = n + 1;
    const int g = lane >> 4;   // lane group: particles 8g..8g+7 of a chunk
    const int ln = lane & 15;  // pair within the wave
    const int task = rblk * kDepWaves + wave;
    const int pg = task / NH;                // group of 16 (k_x, k_y) pairs
    const int mt0 = (task - pg * NH) * MTW;  // first CS tile of this wave
    const int npairs = lines * n1;
    const int pair = pg * 16 + ln;
    const bool pok = pair < npairs;
    const int pc = pok ? pair : npairs - 1;
    const int kx = pc / n1, ky = pc - (pc / n1) * n1;
    const bool idle = pg * 16 >= npairs;  // the last row block's spare waves
    // Two of the three waves of each SIMD (waves 4..11) run a chunk behind in
    // their vector work: they multiply out chunk c with the fragments formed
    // during chunk c - 1 and then form those of chunk c + 1, so that waves in
    // both orders share each SIMD (measured within 3% of one or three late
    // waves per SIMD, and of none).
    const bool late = NBUF == 3 && (wave >> 2) != 0;

    f32x4 acc[MTW][4];
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[mt][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // FP32 sums of the n_z = 0 row (tiles uv), added into this lane's FP64
    // slots in LDS every 2^kDepDcLog chunks
    float dc[4] = {0.f, 0.f, 0.f, 0.f};
    double *dcd = dcs + (wave * 4) * 64 + lane;
#pragma unroll
    for (int t = 0; t < 4; ++t) dcd[t * 64] = 0.0;
    const int xo = (8 * g) * SXY + kx;
    const int yo = (8 * g) * SXY + ky;
    // B fragments of the four tiles (8 particles x 1 pair per lane)
    half8 bh[4], bl[4];

    auto form = [&](const half8 *buf) {
        const unsigned char *cb = reinterpret_cast<const unsigned char *>(buf);
        lds_f2 *px = (lds_f2 *)(reinterpret_cast<const float2 *>(cb + T::x_off) + xo);
        lds_f2 *py = (lds_f2 *)(reinterpret_cast<const float2 *>(cb + T::y_off) + yo);
#pragma unroll
        for (int i = 0; i < 8; i += 2) {
            const float2 x0 = lds_read(px + i * SXY);
            const float2 y0 = lds_read(py + i * SXY);
            const float2 x1 = lds_read(px + (i + 1) * SXY);
            const float2 y1 = lds_read(py + (i + 1) * SXY);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const float a0 = (t & 2) ? x0.y : x0.x, a1 = (t & 2) ? x1.y : x1.x;
                const float b0 = (t & 1) ? y0.y : y0.x, b1 = (t & 1) ? y1.y : y1.x;
                // p = fp32(a b), hi = fp16(p) and lo = fp16(a b - hi), the
                // difference formed in FP32 (exactly, up to the product's
                // own rounding); two values per packed conversion
                const float2_t pv = {a0 * b0, a1 * b1};
                const half2_t hh = __builtin_convertvector(pv, half2_t);
                const float2_t lv = {pv[0] - (float)hh[0], pv[1] - (float)hh[1]};
                const half2_t ll = __builtin_convertvector(lv, half2_t);
                bh[t][i] = hh[0];
                bh[t][i + 1] = hh[1];
                bl[t][i] = ll[0];
                bl[t][i + 1] = ll[1];
                dc[t] += pv[0];
                dc[t] += pv[1];
            }
        }
    };
    auto multiply = [&](int64_t c, const half8 *buf) {
        if (c > 0 && (c & ((1 << kDepFlipLog) - 1)) == 0) {
            // the running sums change sign every 2^kDepFlipLog chunks
#pragma unroll
            for (int mt = 0; mt < MTW; ++mt)
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[mt][t] = -acc[mt][t];
        }
        const _Float16 *chi = reinterpret_cast<const _Float16 *>(buf);
        const _Float16 *clo = chi + T::cs_halves;
#pragma unroll
        for (int mt = 0; mt < MTW; ++mt) {
            if (NH > 1 && mt0 + mt >= MT) continue;  // wave-uniform
            const half8 ah = *reinterpret_cast<const half8 *>(&chi[((mt0 + mt) * 64 + lane) * 8]);
            const half8 al = *reinterpret_cast<const half8 *>(&clo[((mt0 + mt) * 64 + lane) * 8]);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                acc[mt][t] = mfma_split(ah, al, bh[t], bl[t], acc[mt][t]);
                // each accumulator's three products back to back (see mfma_split)
                __builtin_amdgcn_sched_barrier(0);
            }
        }
        if ((c & ((1 << kDepDcLog) - 1)) == ((1 << kDepDcLog) - 1)) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                dcd[t * 64] += (double)dc[t];
                dc[t] = 0.f;
            }
        }
    };
    // The chunk loop, one copy per role so that each is register-allocated on
    // its own.  Chunk c from cur; nxt holds chunk c + 1, and chunk c + NBUF - 1
    // goes into nx2.
    auto run = [&](auto role) {
        constexpr bool LATE = decltype(role)::value;
        auto chunk = [&](int64_t c, const half8 *cur, const half8 *nxt, half8 *nx2) {
            if (c + NBUF - 1 < nchunks) stage(c + NBUF - 1, nx2);
            if (!idle) {
                if constexpr (!LATE) {
                    form(cur);
                    multiply(c, cur);
                } else {
                    // a late wave's products take issue priority over the
                    // early wave's, so that they end first and its vector
                    // work for the next chunk overlaps the early wave's
                    // products instead of trailing them
                    __builtin_amdgcn_s_setprio(2);
                    multiply(c, cur);
                    __builtin_amdgcn_s_setprio(0);
                    if (c + 1 < nchunks) form(nxt);
                }
            }
            __syncthreads();
        };
        __syncthreads();  // the first NBUF - 1 chunks
        if (LATE && !idle) form(buf0);
        if constexpr (NBUF == 3) {
            // triples of chunks, so that each iteration names its buffers statically
            for (int64_t c = 0; c < nchunks; c += 3) {
                chunk(c, buf0, buf1, buf2);
                if (c + 1 < nchunks) chunk(c + 1, buf1, buf2, buf0);
                if (c + 2 < nchunks) chunk(c + 2, buf2, buf0, buf1);
            }
        } else {
            for (int64_t c = 0; c < nchunks; c += 2) {
                chunk(c, buf0, buf1, buf1);
                if (c + 1 < nchunks) chunk(c + 1, buf1, buf0, buf0);
            }
        }
    };
    if (late)
        run(BoolC<true>{});
    else
        run(BoolC<false>{});
    if (idle) return;

    // after chunk c the running sums carry the sign (-1)^((c >> kDepFlipLog) & 1)
    const int64_t last = nchunks - 1;
    const double fsign = last >= 0 && ((last >> kDepFlipLog) & 1) ? -1.0 : 1.0;
    const double outscale = unscale_mf * fsign;
    // the pair's rows of the row layout: (k_x, +k_y), and (k_x, -k_y) when
    // both are non-zero (n_x = 0 rows with n_y < 0 lie in -H)
    const int M = 2 * n + 1;
    const int rp = kx == 0 ? ky : (n + 1) + (kx - 1) * M + (ky + n);
    const int rm = (kx > 0 && ky > 0) ? (n + 1) + (kx - 1) * M + (n - ky) : -1;
    // FP32 partials (each already an FP32 sum; the splits are added in FP64)
    float *pb = part + (int64_t)split * (int64_t)n1 * 4 * Rpad;
    // n_z = 0: the four lane groups' sums, added in a fixed order
    double d[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        d[t] = dcd[t * 64] + (double)dc[t];
        d[t] += __shfl_xor(d[t], 16, 64);
        d[t] += __shfl_xor(d[t], 32, 64);
        d[t] *= unscale_dc;
    }
    if (!pok) return;
    if (g == 0 && mt0 == 0) {
        pb[0 * (int64_t)Rpad + rp] = (float)(d[0] - d[3]);
        pb[1 * (int64_t)Rpad + rp] = (float)(-(d[2] + d[1]));
        pb[2 * (int64_t)Rpad + rp] = 0.f;
        pb[3 * (int64_t)Rpad + rp] = 0.f;
        if (rm >= 0) {
            pb[0 * (int64_t)Rpad + rm] = (float)(d[0] + d[3]);
            pb[1 * (int64_t)Rpad + rm] = (float)(d[1] - d[2]);
            pb[2 * (int64_t)Rpad + rm] = 0.f;
            pb[3 * (int64_t)Rpad + rm] = 0.f;
        }
    }
#pragma unroll
    for (int mt = 0; mt < MTW; ++mt) {
        if (NH > 1 && mt0 + mt >= MT) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = (mt0 + mt) * 16 + 4 * g + i;
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
            const double cc = outscale * (double)acc[mt][0][i], cs = outscale * (double)acc[mt][1][i];
            const double sc = outscale * (double)acc[mt][2][i], ss = outscale * (double)acc[mt][3][i];
            float *o = pb + ((int64_t)nz * 4 + slot) * Rpad;
            o[rp] = (float)(cc - ss);
            o[Rpad + rp] = (float)(-(sc + cs));
            if (rm >= 0) {
                o[rm] = (float)(cc + ss);
                o[Rpad + rm] = (float)(cs - sc);
            }
        }
    }
}

// Particle splits: one block per (row block, split) holds a whole CU, so the
// grid runs in rounds of one block per CU.  The split count is a multiple of
// kXcds (the XCD-aware numbering needs whole groups) chosen to minimise rounds
// per particle, i.e. to avoid a last round that is nearly empty; ties go to
// fewer splits (fewer partials).  A split holds at most kDepMaxRun particles:
// its matrix-core sums run in FP32 over the whole split, so their length is
// bounded whatever N is (more particles mean more splits and FP64 cross-split
// sums instead).
constexpr int64_t kDepMaxRun = 8192;
MfmaDepositPlan plan_deposit_mfma(const Geom &g, int64_t N)
{
    MfmaDepositPlan p;
    // matrix-core wave tasks: groups of 16 (k_x, k_y) pairs, k_x on the
    // context's n_x lines, times the CS halves
    const int MT = mfma_cs_tiles(g.n);
    const int tasks = (g.lines * g.n1 + 15) / 16 * dep_halves(MT);
    p.row_blocks = (tasks + kDepWaves - 1) / kDepWaves;
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
static void launch_dep_mt(hipStream_t s, const double *pos, const double *q, int64_t N, const Geom &g,
                          double L, const MfmaDepositPlan &pl, double qfac, double unscale_mf,
                          double unscale_dc, float *img, float *part)
{
    const int64_t chunks = (N + kDepChunk - 1) / kDepChunk;
    hipLaunchKernelGGL(k_deposit_build<MT>, dim3((unsigned)chunks), dim3(256), 0, s, pos, q, N, g.n,
                       1.0 / L, (int)pl.perm, qfac, pl.per_split / kDepChunk, img);
    // splits rounded up to whole groups of kXcds; blocks past the last split return
    const int groups = (pl.splits + kXcds - 1) / kXcds;
    hipLaunchKernelGGL(k_deposit_mfma<MT>, dim3(groups * kXcds * pl.row_blocks), dim3(kDepThreads), 0, s,
                       img, N, g.n, g.lines, g.Rpad, pl.per_split, pl.row_blocks, pl.splits, unscale_mf,
                       unscale_dc, part);
}

size_t deposit_mfma_rec_bytes(int64_t N, int n)
{
    return (size_t)((N + kDepChunk - 1) / kDepChunk) * dep_image_bytes(n);
}

hipError_t launch_deposit_mfma(hipStream_t s, const double *pos, const double *q, int64_t N,
                               const Geom &g, double L, const MfmaDepositPlan &pl, double qscale,
                               float *rec, float *part)
{
    const double qf = (double)kDepOpScale / qscale;
    // X carries q / qscale scaled by 7/8, the CS operand another 7/8
    const double unscale_dc = qscale / (double)kDepOpScale;
    const double unscale_mf = unscale_dc / (double)kDepOpScale;
    switch (mfma_cs_tiles(g.n)) {
    case 1: launch_dep_mt<1>(s, pos, q, N, g, L, pl, qf, unscale_mf, unscale_dc, rec, part); break;
    case 2: launch_dep_mt<2>(s, pos, q, N, g, L, pl, qf, unscale_mf, unscale_dc, rec, part); break;
    case 3: launch_dep_mt<3>(s, pos, q, N, g, L, pl, qf, unscale_mf, unscale_dc, rec, part); break;
    case 4: launch_dep_mt<4>(s, pos, q, N, g, L, pl, qf, unscale_mf, unscale_dc, rec, part); break;
    case 5: launch_dep_mt<5>(s, pos, q, N, g, L, pl, qf, unscale_mf, unscale_dc, rec, part); break;
    case 6: launch_dep_mt<6>(s, pos, q, N, g, L, pl, qf, unscale_mf, unscale_dc, rec, part); break;
    case 7: launch_dep_mt<7>(s, pos, q, N, g, L, pl, qf, unscale_mf, unscale_dc, rec, part); break;
    default: launch_dep_mt<8>(s, pos, q, N, g, L, pl, qf, unscale_mf, unscale_dc, rec, part); break;
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
//
// W fragments: wf[t][s][h][lane][8] halves, t = quad (< Qpad), s = K step, h = hi/lo.
// Lane l, element i: A row m = l % 16 -> padded row 4t + m/4, component
// e = m % 4; K index k = 32 s + 8 (l/16) + i -> cos (k < nzk) or sin of
// n_z = (k mod nzk) + 1.
// One wave per (quad, K step): the 16 lanes of each of the quad's four rows
// (m / 4 fixed) first find the row's scale together, reading the whole row
// (all K steps), then each lane packs its 8 entries; the K step 0 wave writes
// the row records.  The kernel is small and bound by load latency, so every
// load a lane makes is issued before the first wait: its 8 entries, psi(r, 0)
// and (for n_max <= 16) its whole share of the row, from addresses clamped
// into the row, with the values past the row's n_max entries dropped.
__global__ void __launch_bounds__(256)
k_force_pack(const float *__restrict__ ftab, const float *__restrict__ psi0, int n, int lines,
             int nzp, int nzk, int ks, float4 *__restrict__ rinfo, _Float16 *__restrict__ wf)
{
    const ForceQuads f = force_quads(n, lines);
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t total = (int64_t)f.Qpad * ks * 64;
    if (gid >= total) return;  // whole waves: total is a multiple of 64
    const int lane = (int)(gid & 63);
    const int64_t ts = gid >> 6;
    const int s = (int)(ts % ks);
    const int t = (int)(ts / ks);
    const int mrow = lane & 15;
    const int pr = 4 * t + (mrow >> 2);
    const int e = mrow & 3;
    int nx = 0, ny = 0;
    const int r = force_row(pr, n, f, nx, ny);
    const bool ok = r >= 0;
    const float *fr = ftab + (int64_t)(ok ? r : 0) * nzp * 8;
    // entry of the force table packed by component e: cos terms sig_r, sig_i,
    // nz del_r, nz del_i (0, 1, 4, 5), sin terms -del_i, del_r, -nz sig_i,
    // nz sig_r (3, 2, 7, 6)
    //   Re U0 = sig_r cos - del_i sin        Im U0 = sig_i cos + del_r sin
    //   Re U1 = nz (del_r cos - sig_i sin)   Im U1 = nz (del_i cos + sig_r sin)
    const int cbase = 4 * (e >> 1);
    float v[8];
    bool use[8], neg[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int k = 32 * s + 8 * (lane >> 4) + i;
        const bool is_sin = k >= nzk;
        const int nz = (is_sin ? k - nzk : k) + 1;
        use[i] = ok && nz <= n;
        neg[i] = is_sin && !(e & 1);
        const int comp = cbase + (is_sin ? 3 - (e & 1) : (e & 1));
        v[i] = fr[(use[i] ? nz - 1 : 0) * 8 + comp];
    }
    const float2 p0 = reinterpret_cast<const float2 *>(psi0)[ok ? r : 0];
    // the row's largest |entry|: lane (e, lane group g) reads entries e + 4 g + 16 j
    float mx = 0.f;
    const int i0 = e + 4 * (lane >> 4);
    for (int j0 = 0; j0 < 8 * n; j0 += 16 * 8) {
        float a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + j0 + 16 * u;
            const bool in = i < 8 * n;
            a[u] = fr[in ? i : 0];
            if (!in) a[u] = 0.f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) mx = fmaxf(mx, fabsf(a[u]));
    }
    if (!ok) mx = 0.f;
    for (int o = 1; o <= 32; o <<= 1)
        if (o != 4 && o != 8) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    float inv = 1.0f;
    if (ok) {
        mx = fmaxf(mx, ldexpf(fmaxf(fabsf(p0.x), fabsf(p0.y)), -60));
        int ex = 0;
        if (mx > 0.f) {
            frexpf(mx, &ex);  // mx = f 2^ex, f in [0.5, 1)
            ex = ex < -126 ? -126 : (ex > 126 ? 126 : ex);
        }
        const float sc = mx > 0.f ? ldexpf(1.0f, ex) : 1.0f;
        inv = mx > 0.f ? ldexpf(1.0f, -ex) : 1.0f;
        if (s == 0 && e == 0 && lane < 16) {
            rinfo[2 * pr] = make_float4(p0.x * inv, p0.y * inv, 0.f, 0.f);
            rinfo[2 * pr + 1] = make_float4((float)nx * sc, (float)ny * sc, sc, 0.f);
        }
    } else if (s == 0 && e == 0 && lane < 16) {
        rinfo[2 * pr] = make_float4(0.f, 0.f, 0.f, 0.f);
        rinfo[2 * pr + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    _Float16 hi[8], lo[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float x = use[i] ? (neg[i] ? -v[i] : v[i]) : 0.f;
        split_f16(x * inv, hi[i], lo[i]);
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
    const int nzk = (g.n + 15) / 16 * 16;
    const int ks = nzk / 16;
    const int64_t total = (int64_t)f.Qpad * ks * 64;
    hipLaunchKernelGGL(k_force_pack, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, ftab,
                       psi0, g.n, g.lines, g.nzp, nzk, ks, rinfo, wf);
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
// step is the same for every lane.  At each run end g restarts from the
// next column's phase, kept by an FP64 complex recurrence in t_y (exact to
// ~1e-15 over all columns), so FP32 phase steps never run longer than one
// run; at every fourth run end (and after the last) the FP32 sums go into
// FP64, so an FP32 sum spans at most 4 runs (32 quads at n_max = 32).
// Adding them at every run end cost 1.2% more time at 2^20 particles, with
// no gain in accuracy.  PHI: also sum the potential (the
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
k_force_mfma(double *__restrict__ pos, const double *__restrict__ q,
             const double *__restrict__ m, double *__restrict__ vel, const _Float16 *__restrict__ wf,
             const float4 *__restrict__ rinfo, int n, int lines, double L, double invL, int64_t N,
             double kick, Drift nd, double *__restrict__ F, double *__restrict__ phi)
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
    int runs = 0;          // runs finished

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
            // one tile's products back to back (see mfma_split); with a single
            // K step the chain is short, and interleaving the tiles hides its
            // latency better.  Not in the variant with the potential, which
            // then needs more than 128 VGPRs.
            if constexpr (KS > 1 && !PHI) __builtin_amdgcn_sched_barrier(0);
        }
    };
    // KS = 1: the W fragments and record A of a quad, read from LDS one quad
    // before its products are issued, so that the read's latency hides behind
    // an epilogue (12 more VGPRs, still four waves per SIMD: 2.5% less force
    // time at n_max = 16; at KS = 2 the extra registers cost a wave per SIMD)
    struct WFrag {
        half8 ah, al;
        float4 ci;
    };
    auto load_w = [&](const half8 *wl, int tt) {
        WFrag f;
        f.ah = wl[(tt * 2 + 0) * 64 + lane];
        f.al = wl[(tt * 2 + 1) * 64 + lane];
        f.ci = reinterpret_cast<const float4 *>(wl + PIECES * 64)[2 * (4 * tt + g)];
        return f;
    };
    auto products_w = [&](const WFrag &f, f32x4 (&acc)[NT]) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            acc[nt] = f32x4{f.ci.x, f.ci.y, f.ci.z, f.ci.w};
            acc[nt] = mfma_split(f.ah, f.al, bh[nt][0], bl[nt][0], acc[nt]);
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
            if ((++runs & 3) == 1) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    fx[nt] += (double)sx[nt];
                    fy[nt] += (double)sy[nt];
                    fz[nt] += (double)sz[nt];
                    if (PHI) fp[nt] += (double)sp[nt];
                    sx[nt] = sy[nt] = sz[nt] = sp[nt] = 0.f;
                }
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
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
        if constexpr (KS == 1 && !PHI) {
            // cnt is even: quads tt + 2 and tt + 3 exist together
            WFrag wa = load_w(wl, 0), wb = load_w(wl, 1);
            products_w(wa, accA);
#pragma unroll 1
            for (int tt = 0; tt < cnt; tt += 2) {
                products_w(wb, accB);
                const bool more = tt + 2 < cnt;
                if (more) wa = load_w(wl, tt + 2);
                epilogue(wl, tt, t0 + tt, accA);
                if (more) {
                    products_w(wa, accA);
                    wb = load_w(wl, tt + 3);
                }
                epilogue(wl, tt + 1, t0 + tt + 1, accB);
            }
        } else {
            products(wl, 0, accA);
#pragma unroll 1
            for (int tt = 0; tt < cnt; tt += 2) {
                products(wl, tt + 1, accB);
                epilogue(wl, tt, t0 + tt, accA);
                if (tt + 2 < cnt) products(wl, tt + 2, accA);
                epilogue(wl, tt + 1, t0 + tt + 1, accB);
            }
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
    // what the last runs left in FP32
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        fx[nt] += (double)sx[nt];
        fy[nt] += (double)sy[nt];
        fz[nt] += (double)sz[nt];
        if (PHI) fp[nt] += (double)sp[nt];
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
            if (!PHI && (nd.kick != 0.0 || nd.drift != 0.0)) {
                // the next step's first half kick and drift, as a separate
                // kick-drift pass would apply them (same operations in the
                // same order); this thread is the only one that reads x_j
                const double am = nd.kick != 0.0 ? nd.kick / m[j] : 0.0;
                const double Fd[3] = {Fx, Fy, Fz};
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    double v = vel[d * N + j];
                    if (nd.kick != 0.0) {
                        v += am * Fd[d];
                        vel[d * N + j] = v;
                    }
                    if (nd.drift != 0.0) {
                        const double x = pos[d * N + j] + nd.drift * v;
                        pos[d * N + j] = nd.wrap ? wrap_box(x, L, invL) : x;
                    }
                }
            }
        }
    }
}

template <int KS>
static void launch_force_ks(hipStream_t s, dim3 grid, dim3 block, double *pos, const double *q,
                            const double *m, double *vel, const _Float16 *wf, const float4 *rinfo,
                            int n, int lines, double L, int64_t N, double kick, const Drift &nd,
                            double *F, double *phi)
{
    if (phi)
        hipLaunchKernelGGL((k_force_mfma<KS, true>), grid, block, 0, s, pos, q, m, vel, wf, rinfo, n,
                           lines, L, 1.0 / L, N, kick, nd, F, phi);
    else
        hipLaunchKernelGGL((k_force_mfma<KS, false>), grid, block, 0, s, pos, q, m, vel, wf, rinfo, n,
                           lines, L, 1.0 / L, N, kick, nd, F, phi);
}

hipError_t launch_force_mfma(hipStream_t s, double *pos, const double *q, const double *m,
                             double *vel, const _Float16 *wf, const float4 *rinfo, const Geom &g,
                             double L, int64_t N, double kick, const Drift &nd, double *F,
                             double *phi)
{
    // the next step's kick and drift: with F, and not in the variant that
    // also sums the potential
    if ((nd.kick != 0.0 || nd.drift != 0.0) && (!F || phi)) return hipErrorInvalidValue;
    const int ks = (g.n + 15) / 16;
    const int64_t blocks = (N + kForceBlockParticles - 1) / kForceBlockParticles;
    const dim3 grid((unsigned)blocks), block(64 * kForceWaves);
    switch (ks) {
    case 1: launch_force_ks<1>(s, grid, block, pos, q, m, vel, wf, rinfo, g.n, g.lines, L, N, kick, nd, F, phi); break;
    case 2: launch_force_ks<2>(s, grid, block, pos, q, m, vel, wf, rinfo, g.n, g.lines, L, N, kick, nd, F, phi); break;
    case 3: launch_force_ks<3>(s, grid, block, pos, q, m, vel, wf, rinfo, g.n, g.lines, L, N, kick, nd, F, phi); break;
    default: launch_force_ks<4>(s, grid, block, pos, q, m, vel, wf, rinfo, g.n, g.lines, L, N, kick, nd, F, phi); break;
    }
    return hipGetLastError();
}

size_t force_pack_bytes(const Geom &g)
{
    const int ks = (g.n + 15) / 16;
    return (size_t)force_quads(g.n, g.lines).Qpad * ks * 2 * 64 * 8 * sizeof(_Float16);
}

}  // namespace sce
