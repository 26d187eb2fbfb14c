// Split-precision chi sum: chi = pf * X_w^T (X + iY) (real embedding of
// M^H diag(w) M, see chi.hip) computed from BF16 digit slices on MFMA with
// FP32 accumulation, recombined in FP64.
//
// Digits.  The real contraction index k' = 2t + part is cut into chunks of
// 192 (96 pairs, six MFMA k-steps).  Within a chunk every column G of X gets a power-of-two
// scale 2^eB (eB = exponent of the chunk-column max of |Re M|, |Im M|), and
// every column of X_w, for each weight vector, the scale 2^eA of the
// chunk-column max of |w_t Re M|, |w_t Im M| (both found by k_split_slice in
// its pass over M).  Each scaled value y = x 2^(8-e), |y| < 256, is written
// as four signed digits in base 512:
//     y = d1 + d2 2^-9 + d3 2^-18 + d4 2^-27 + r,  |di| <= 256,  |r| <= 2^-28,
// every digit an integer of magnitude <= 256 and so exact in BF16 (eight
// significant bits).  The unweighted side's digits do not depend on the
// frequency: k_split_slice stores them once per q (8 bytes per real value).
// The weighted side is sliced inside the GEMM from M and w, in registers,
// for each frequency, so no weighted slices are stored at all.
//
// Products (k_chi_split), grouped by weight 2^-9p, one FP32 sum per group:
//     p = 0: a1 b1                                   (exact: |sum| <= 2^16 * 192 < 2^24)
//     p = 1: a1 b2 + a2 b1                           (exact while |sum| < 2^24)
//     p = 2: a1 b3 + a2 b2 + a3 b1
//            + a1' b4 + a2' b3 + a3' b2 + a4' b1     (rounded at 2^-24 of the group)
// where ai' = ai 2^-9 (exact in BF16) folds the weight-2^-27 products into
// the third group.  Ten BF16 MFMA products per (Re, Im); at each chunk end
// the three FP32 sums are combined in FP64 with the chunk scales
// 2^(eA + eB - 16) and added to FP64 accumulators.  Terms of weight
// <= 2^-36 are dropped, and so is the remainder r.  The second group's
// partial sums pass 2^24 only if most of the chunk's 384 products reach
// 2^16 with one sign; FP32 then rounds at 2^-24 of that group, 2^-33 of the
// chunk's leading term.  Expected relative error: a few 1e-11 for positive
// weights, a few 1e-10 where the weights change sign across a resonance.
//
// The head row/column (G = 0) is recomputed in FP64 from M (k_headwing)
// because v(q+G) ~ 1/q^2 amplifies it in epsilon.
#include <algorithm>
#include <cstdlib>

#include "common.h"

namespace bgw {

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

namespace {
constexpr int SK = 192;       // real contraction rows per chunk (one set of exponents, FP32 group sums)
constexpr int SKP = SK / 2;   // pairs per chunk
constexpr int KS = 32;        // real rows per MFMA k-step (16x16x32)
constexpr int KSP = KS / 2;   // pairs per k-step
constexpr int NKS = SK / KS;  // k-steps per chunk
constexpr int NSL = 4;        // stored slices
constexpr int NGR = 3;        // FP32 product groups
constexpr int TR = 64;        // output tile rows: weighted side, sliced in registers
constexpr int TC = 128;       // output tile columns: unweighted side, digit slices through LDS
constexpr int XT = 512;       // GEMM block: 8 waves (two per SIMD), 4 x 2 over the tile
constexpr int kMinExp = -500; // chunk exponents are clamped here (values below 2^-500 count as zero)

__device__ inline double pow2(int e) { return __longlong_as_double((long long)(e + 1023) << 52); }

__device__ inline int chunk_exp(double mx) {
    int e = 0;
    if (mx > 0.0) (void)frexp(mx, &e);  // mx < 2^e
    return max(e, kMinExp);
}

__device__ inline unsigned short bf16_bits_exact(double v) {
    // v is an integer of at most 9 significant bits: exact in BF16
    const float f = (float)v;
    return (unsigned short)(__float_as_uint(f) >> 16);
}
}  // namespace

// Digit slices of the unweighted side for chunks [c0, c0 + nchunk) of one q,
// and the chunk-column exponents of the weighted side of every weight vector.
// Block = one chunk x 32 columns, 384 threads.  Thread t owns column G = 32
// blockIdx.x + (t/4) % 32 and, in each of the k-steps 2 (t/128) and
// 2 (t/128) + 1, the four pairs 4 (t%4) .. +3; with this assignment every
// 16-byte store instruction of a wave writes 1 KB of contiguous slice memory.
// S: [NSL][nchunk][NKS][gpad][KS] bf16 bits, each group of 8 values holding four
// pairs as (Re t0..t3, Im t0..t3); E: [nchunk][gpad] (2^E above the chunk-column
// max of |Re M|, |Im M|); EA: [nvec][nchunk][gpad], 2^EA above the chunk-column
// max of |w_v(t) Re M|, |w_v(t) Im M| (clamped to [-128, 127]: a value below
// 2^-128 only keeps fewer digits).  Pairs >= K are zero.
constexpr int SLICE_T = 32 * 4 * (NKS / 2);  // 384
__global__ __launch_bounds__(SLICE_T) void k_split_slice(const double2 *__restrict__ M, long long K, int ng, int gpad,
                                                         long long c0, int nchunk, unsigned short *__restrict__ S,
                                                         int *__restrict__ E, const double *__restrict__ w,
                                                         long long wstride, int nvec, signed char *__restrict__ EA) {
    constexpr int NP = 4 * (NKS / 2);  // partial maxima per column
    __shared__ double red[NP][32];
    const int q = threadIdx.x & 3, cl = (threadIdx.x >> 2) & 31, kh = threadIdx.x >> 7;
    const int G = blockIdx.x * 32 + cl;
    const int chunk = blockIdx.y;
    const long long tb = (c0 + chunk) * SKP;
    const bool col = G < ng;
    double2 m[2][4];  // [k-step i][pair j]
    double mx = 0.0;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long long t = tb + (2 * kh + i) * KSP + 4 * q + j;
            m[i][j] = (t < K && col) ? M[t * ng + G] : make_double2(0.0, 0.0);
            mx = fmax(mx, fmax(fabs(m[i][j].x), fabs(m[i][j].y)));
        }
    red[4 * kh + q][cl] = mx;
    __syncthreads();
    mx = 0.0;
#pragma unroll
    for (int k = 0; k < NP; ++k) mx = fmax(mx, red[k][cl]);
    const size_t slice_stride = (size_t)nchunk * NKS * gpad * KS;
    const int e = chunk_exp(mx);
    if (q == 0 && kh == 0) E[(size_t)chunk * gpad + G] = e;
    const double up = pow2(8 - e);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int ks = 2 * kh + i;
        unsigned short d[NSL][8];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int part = 0; part < 2; ++part) {
                const double y = (part ? m[i][j].y : m[i][j].x) * up;
                const double d1 = rint(y);
                double r = (y - d1) * 512.0;
                const double d2 = rint(r);
                r = (r - d2) * 512.0;
                const double d3 = rint(r);
                r = (r - d3) * 512.0;
                const double d4 = rint(r);
                const int qq = 4 * part + j;  // real parts first, then imaginary parts
                d[0][qq] = bf16_bits_exact(d1);
                d[1][qq] = bf16_bits_exact(d2);
                d[2][qq] = bf16_bits_exact(d3);
                d[3][qq] = bf16_bits_exact(d4);
            }
        const size_t dst = (((size_t)chunk * NKS + ks) * gpad + G) * KS + 8 * q;
#pragma unroll
        for (int sl = 0; sl < NSL; ++sl) {
            uint4 pk;
            pk.x = d[sl][0] | ((unsigned)d[sl][1] << 16);
            pk.y = d[sl][2] | ((unsigned)d[sl][3] << 16);
            pk.z = d[sl][4] | ((unsigned)d[sl][5] << 16);
            pk.w = d[sl][6] | ((unsigned)d[sl][7] << 16);
            *reinterpret_cast<uint4 *>(S + sl * slice_stride + dst) = pk;
        }
    }
    // weighted side: the same products fl(w x) the GEMM forms, so 2^EA bounds them
    double mr[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) mr[i][j] = fmax(fabs(m[i][j].x), fabs(m[i][j].y));
    for (int v = 0; v < nvec; ++v) {
        const double *wv = w + (size_t)v * wstride;
        double mw = 0.0;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const long long t = tb + (2 * kh + i) * KSP + 4 * q + j;
                if (t < K) mw = fmax(mw, fabs(wv[t]) * mr[i][j]);
            }
        __syncthreads();  // the previous vector's reduction has been read
        red[4 * kh + q][cl] = mw;
        __syncthreads();
        if (q == 0 && kh == 0) {
            mw = 0.0;
#pragma unroll
            for (int k = 0; k < NP; ++k) mw = fmax(mw, red[k][cl]);
            EA[((size_t)v * nchunk + chunk) * gpad + G] = (signed char)min(127, max(-128, chunk_exp(mw)));
        }
    }
}

namespace {
__device__ inline bf16x8_t as_bf16x8(uint4 u) {
    bf16x8_t r;
    __builtin_memcpy(&r, &u, 16);
    return r;
}
// A fragment holds four pairs as (Re t0..t3, Im t0..t3); the Y operand of the
// imaginary part is (Im t0..t3, -Re t0..t3): the two halves exchanged and the
// moved real parts negated (sign bits of both BF16 halves of a dword).
__device__ inline uint4 swap_neg(uint4 u) {
    uint4 r;
    r.x = u.z;
    r.y = u.w;
    r.z = u.x ^ 0x80008000u;
    r.w = u.y ^ 0x80008000u;
    return r;
}
#define MFMA(a, b, c) __builtin_amdgcn_mfma_f32_16x16x32_bf16((a), (b), (c), 0, 0, 0)

typedef __attribute__((address_space(3))) void lds_void_t;

// LDS stage of one k-step: the weighted side as FP64 complex, [16 pairs][64
// columns] (16 B each, 1 KB per pair row); the unweighted side's four digit
// slices, [slice][128 rows][64 B] with the four 16-B segments of row r stored
// in the order seg ^ ((r >> 1) & 3), so that the eight rows one 16-B read
// phase touches fall in distinct bank groups; the step's 16 weights.
// Besides the two stages, two exponent buffers hold a
// chunk's 128 column exponents (int32, bytes 0..511) and 64 row exponents of
// the weighted side (int8, bytes 512..575): chunk c in buffer c % 2, staged
// with the chunk's first step and read when the chunk starts and when it ends.
constexpr int A_LDS = KSP * TR * 16;          // 16 KB
constexpr int B_SLICE_LDS = TC * KS * 2;      // 8 KB
constexpr int W_OFF = A_LDS + NSL * B_SLICE_LDS;
constexpr int STG = W_OFF + 256;              // 48.25 KB
constexpr int E_LDS = 1024;
constexpr int NWAVE = XT / 64;
constexpr int PA = KSP / NWAVE;               // 1-KB pieces of the A part per wave: 2
constexpr int PB = NSL * B_SLICE_LDS / 1024 / NWAVE;  // of the B part: 4

// vmcnt(n) alone (expcnt and lgkmcnt left at their maxima); vmcnt is split
// over bits 3:0 and 15:14 of the immediate
#define BGW_WAIT_VM(n) __builtin_amdgcn_s_waitcnt(0x0F70 | ((n) & 0xF) | (((n) >> 4) << 14))

// Workgroup barrier for the stage pipeline: the wave's LDS reads are complete
// (lgkmcnt) and its direct-to-LDS loads have been waited for explicitly, so no
// fence is needed; __syncthreads() would also wait for the loads still in
// flight for later stages.
__device__ __forceinline__ void stage_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Per-lane sources of one item's stage loads.  A piece i of wave w is pair
// row j = 2w + i of the k-step: lane L loads M[t][G0 + L] (clamped into M;
// the slicing zeroes what lies outside).  B piece i of wave w is slice w/2,
// rows 64 (w%2) + 16 i .. +16: lane L loads row 64 (w%2) + 16 i + L/4 at
// stored segment L%4, i.e. source segment (L%4) ^ ((L/4) & 3), one per-lane
// address plus i KB.
// Wave 1 loads the step's weights (lanes 0..7, two each): the weight
// vectors are padded by 128 entries, and the slicing zeroes pairs past K.
struct StageSrc {
    const char *a_base;      // M + G(lane) (bytes), pair rows added per step
    long long a_row_bytes;   // ng * 16
    long long kmax;          // last valid pair
    const char *b_base;      // slice wave/2, row 64 (wave%2) + L/4 and segment of this lane (bytes), k-step added
    size_t b_step_bytes;     // gpad * KS * 2
    const double *w;         // weights of this vector
    const int *eb;           // EB: chunk-column exponents of the slices, [nch][gpad]
    const signed char *ea;   // EA of this vector: chunk-column exponents of the weighted side, [nch][gpad]
    int gpad, G0, H0;
};

__device__ __forceinline__ void stage_issue(unsigned char *__restrict__ stage, unsigned char *__restrict__ ebuf,
                                            const StageSrc &S, long long t0, long long step, int wave, int lane) {
#pragma unroll
    for (int i = 0; i < PA; ++i) {
        const long long t = min(t0 + PA * wave + i, S.kmax);
        __builtin_amdgcn_global_load_lds((const void *)(S.a_base + t * S.a_row_bytes),
                                         (lds_void_t *)(stage + (PA * wave + i) * 1024), 16, 0, 0);
    }
    const char *b = S.b_base + step * S.b_step_bytes;
#pragma unroll
    for (int i = 0; i < PB; ++i)
        __builtin_amdgcn_global_load_lds((const void *)(b + i * 1024),
                                         (lds_void_t *)(stage + A_LDS + (wave >> 1) * B_SLICE_LDS +
                                                        (wave & 1) * 4096 + i * 1024),
                                         16, 0, 0);
    if (wave == 1 && lane < 8)
        __builtin_amdgcn_global_load_lds((const void *)(S.w + t0 + 2 * lane), (lds_void_t *)(stage + W_OFF), 16, 0,
                                         0);
    if (wave == 0 && step % NKS == 0) {
        const long long ch = step / NKS;
        const int *er = S.eb + ch * S.gpad;
        if (lane < 32)
            __builtin_amdgcn_global_load_lds((const void *)(er + S.H0 + 4 * lane), (lds_void_t *)ebuf, 16, 0, 0);
        if (lane < 4)
            __builtin_amdgcn_global_load_lds((const void *)(S.ea + ch * S.gpad + S.G0 + 16 * lane),
                                             (lds_void_t *)(ebuf + 512), 16, 0, 0);
    }
}


__device__ __forceinline__ uint4 bfrag(const unsigned char *slice, int row, int lq) {
    return *reinterpret_cast<const uint4 *>(slice + row * 64 + 16 * (lq ^ ((row >> 1) & 3)));
}

constexpr int NCB = TC / 32;  // column blocks of a wave (each wave spans 64 of the 128 columns)

struct SplitAcc {
    float4_t g[NCB][NGR][2];  // [col block][group][re/im]
    double re[NCB][4], im[NCB][4];
};

// Digits of two values as the BF16 pairs (low half first) of each slice, and
// the same digits times 2^-9.
__device__ __forceinline__ void digits2(double y0, double y1, unsigned (&d)[NSL], unsigned (&ds)[NSL]) {
    double r0 = y0, r1 = y1;
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) {
        const double a = rint(r0), b = rint(r1);
        if (sl + 1 < NSL) {
            r0 = (r0 - a) * 512.0;
            r1 = (r1 - b) * 512.0;
        }
        const float fa = (float)a, fb = (float)b;
        d[sl] = __builtin_amdgcn_perm(__float_as_uint(fb), __float_as_uint(fa), 0x07060302u);
        ds[sl] = __builtin_amdgcn_perm(__float_as_uint(fb * 0.001953125f), __float_as_uint(fa * 0.001953125f),
                                       0x07060302u);
    }
}

// The four slice fragments f of this lane's 8 values (Re t0..t3, Im t0..t3)
// y = w_t M_t(G) 2^(8 - eA), and fs = f times 2^-9.  The values of pairs
// (t0, t1) are read and sliced before those of (t2, t3).
__device__ __forceinline__ void slice_frags(const unsigned char *src, const double (&sw)[4], uint4 (&f)[NSL],
                                            uint4 (&fs)[NSL]) {
    unsigned d[NSL], ds[NSL];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const double2 m0 = *reinterpret_cast<const double2 *>(src + (2 * h) * 1024);
        const double2 m1 = *reinterpret_cast<const double2 *>(src + (2 * h + 1) * 1024);
        digits2(m0.x * sw[2 * h], m1.x * sw[2 * h + 1], d, ds);
#pragma unroll
        for (int sl = 0; sl < NSL; ++sl) {
            if (h == 0) f[sl].x = d[sl], fs[sl].x = ds[sl];
            else f[sl].y = d[sl], fs[sl].y = ds[sl];
        }
        digits2(m0.y * sw[2 * h], m1.y * sw[2 * h + 1], d, ds);
#pragma unroll
        for (int sl = 0; sl < NSL; ++sl) {
            if (h == 0) f[sl].z = d[sl], fs[sl].z = ds[sl];
            else f[sl].w = d[sl], fs[sl].w = ds[sl];
        }
    }
}

// Ten BF16 products per (Re, Im) of the wave's row block and one column block.
__device__ __forceinline__ void split_mfma(const uint4 (&af)[NSL], const uint4 (&as)[NSL], const uint4 (&bf)[NSL],
                                           float4_t (&g)[NGR][2]) {
    const bf16x8_t a1 = as_bf16x8(af[0]), a2 = as_bf16x8(af[1]), a3 = as_bf16x8(af[2]);
    const bf16x8_t s1 = as_bf16x8(as[0]), s2 = as_bf16x8(as[1]), s3 = as_bf16x8(as[2]), s4 = as_bf16x8(as[3]);
    const bf16x8_t b1 = as_bf16x8(bf[0]), b2 = as_bf16x8(bf[1]), b3 = as_bf16x8(bf[2]), b4 = as_bf16x8(bf[3]);
    const bf16x8_t y1 = as_bf16x8(swap_neg(bf[0])), y2 = as_bf16x8(swap_neg(bf[1]));
    const bf16x8_t y3 = as_bf16x8(swap_neg(bf[2])), y4 = as_bf16x8(swap_neg(bf[3]));
    g[0][0] = MFMA(a1, b1, g[0][0]);
    g[0][1] = MFMA(a1, y1, g[0][1]);
    g[1][0] = MFMA(a1, b2, g[1][0]);
    g[1][1] = MFMA(a1, y2, g[1][1]);
    g[1][0] = MFMA(a2, b1, g[1][0]);
    g[1][1] = MFMA(a2, y1, g[1][1]);
    g[2][0] = MFMA(a1, b3, g[2][0]);
    g[2][1] = MFMA(a1, y3, g[2][1]);
    g[2][0] = MFMA(a2, b2, g[2][0]);
    g[2][1] = MFMA(a2, y2, g[2][1]);
    g[2][0] = MFMA(a3, b1, g[2][0]);
    g[2][1] = MFMA(a3, y1, g[2][1]);
    g[2][0] = MFMA(s1, b4, g[2][0]);
    g[2][1] = MFMA(s1, y4, g[2][1]);
    g[2][0] = MFMA(s2, b3, g[2][0]);
    g[2][1] = MFMA(s2, y3, g[2][1]);
    g[2][0] = MFMA(s3, b2, g[2][0]);
    g[2][1] = MFMA(s3, y2, g[2][1]);
    g[2][0] = MFMA(s4, b1, g[2][0]);
    g[2][1] = MFMA(s4, y1, g[2][1]);
}

// Chunk end: the three FP32 groups combined in FP64 with the chunk scales
// 2^(eA + eB - 16) into the FP64 accumulators.  D layout of 16x16x32: lane
// l, register r -> row 4 (l/16) + r, col l % 16.  E: the chunk's exponent
// buffer.
__device__ __forceinline__ void split_flush(SplitAcc &acc, const int *E, int wave, int li, int lq) {
    const signed char *Ea = reinterpret_cast<const signed char *>(E) + 512;
    int era[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) era[r] = (int)Ea[16 * (wave >> 1) + 4 * lq + r] - 16;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int ec = E[64 * (wave & 1) + 16 * cb + li];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double sc = pow2(era[r] + ec);
            const float4_t(&g)[NGR][2] = acc.g[cb];
            const double vre =
                (double)g[0][0][r] + ((double)g[1][0][r] + (double)g[2][0][r] * 0.001953125) * 0.001953125;
            const double vim =
                (double)g[0][1][r] + ((double)g[1][1][r] + (double)g[2][1][r] * 0.001953125) * 0.001953125;
            acc.re[cb][r] = fma(vre, sc, acc.re[cb][r]);
            acc.im[cb][r] = fma(vim, sc, acc.im[cb][r]);
        }
        __builtin_amdgcn_sched_barrier(0);  // one column block at a time
    }
}

// Upper tiles of the 64-row x 128-column tiling of an ng x ng matrix: tile
// (I, J) holds some G <= H iff 64 I <= 128 J + 127, i.e. I <= 2 J + 1.
}  // namespace

// One k-step x: stage step x + 1 into `nxt`, slice this lane's row of the
// weighted side from `cur`, 80 MFMAs over the four column blocks, then wait
// for step x + 1's loads and meet the block at the barrier.  The two stages
// are distinct restrict-qualified buffers, so the compiler knows that the
// loads in flight into one do not alias the reads of the other.
__device__ __forceinline__ void split_step(const unsigned char *__restrict__ cur, unsigned char *__restrict__ nxt,
                                           unsigned char *__restrict__ ebuf1, const StageSrc &S, long long x,
                                           long long s1, long long tbase, long long K, double up, int wave, int lane,
                                           int li, int lq, SplitAcc &acc) {
    __builtin_amdgcn_sched_barrier(0);
    if (x + 1 < s1) stage_issue(nxt, ebuf1, S, tbase + (x + 1) * KSP, x + 1, wave, lane);
    __builtin_amdgcn_sched_barrier(0);
    // the weighted side of this lane's row, sliced into digits (pairs >= K weigh 0)
    uint4 af[NSL], as[NSL];
    {
        const long long tp = tbase + x * KSP + 4 * lq;
        const double *wl = reinterpret_cast<const double *>(cur + W_OFF) + 4 * lq;
        double sw[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) sw[j] = tp + j < K ? wl[j] * up : 0.0;
        slice_frags(cur + (4 * lq) * 1024 + (16 * (wave >> 1) + li) * 16, sw, af, as);
    }
    const unsigned char *Bs = cur + A_LDS;
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        uint4 bf[NSL];
#pragma unroll
        for (int sl = 0; sl < NSL; ++sl) bf[sl] = bfrag(Bs + sl * B_SLICE_LDS, 64 * (wave & 1) + 16 * cb + li, lq);
        split_mfma(af, as, bf, acc.g[cb]);
    }
    BGW_WAIT_VM(0);
    stage_barrier();
}

// Persistent split-precision chi sum over every (q, weight vector, tile, K
// split) item of a launch.  Entry q owns the items q.item0 .. q.item0 +
// q.nitems (a multiple of 8); item i always runs on XCD i % 8 (a grid that
// is a multiple of 8, workgroups dealt to the XCDs round-robin), and XCD x
// takes the x-th contiguous eighth of the entry's (split, tile, vector)
// sequence, vector fastest: the blocks resident on one XCD work on the same
// tile for consecutive weight vectors (frequencies), reading the same rows of
// M and the same slices, which their L2 then serves.  With one weight vector
// the sequence walks the tiles in bands of eight row tiles.
// Block: 8 waves, two per SIMD; wave w owns rows 16 (w/2) .. +16 and columns
// 64 (w%2) .. +64 (four column blocks) of the 64 x 128 tile, so each row is
// sliced by the two waves that share it, and one wave's slicing and LDS
// reads run under the MFMAs of the other wave on its SIMD.
// Every k-step (16 pairs) the block stages 16 pair rows of M (the tile's 64
// columns), the four digit slices of the unweighted side (128 columns) and
// the 16 weights into LDS with direct global->LDS loads, one step ahead
// through two stages; each wave slices its 16 rows of w_t M_t(G) into BF16
// digits in registers and issues 80 MFMAs.
// out (+)= raw sums (no prefactor) of every element of the tile inside ng x ng.
__global__ __launch_bounds__(XT, 1) void k_chi_split(const SplitQ *__restrict__ qs, int nq, long long i0,
                                                     long long i1) {
    __shared__ __attribute__((aligned(1024))) unsigned char stage0[STG];
    __shared__ __attribute__((aligned(1024))) unsigned char stage1[STG];
    __shared__ __attribute__((aligned(1024))) unsigned char ebufs[2][E_LDS];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lq = lane >> 4;

    for (long long item = i0 + blockIdx.x; item < i1; item += gridDim.x) {
        int lo = 0, hi = nq - 1;  // last entry with item0 <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (qs[mid].item0 <= item) lo = mid;
            else hi = mid - 1;
        }
        const SplitQ &Q = qs[lo];
        const long long local = item - Q.item0;
        const long long per = Q.nitems / 8;  // items per XCD
        const long long u = (local % 8) * per + local / 8;
        const long long total = (long long)Q.ntiles * Q.ns * Q.nvec;
        if (u >= total) continue;  // padding item
        const int v = (int)(u % Q.nvec);
        const long long r0 = u / Q.nvec;
        const int tile = (int)(r0 % Q.ntiles);
        const int split = (int)(r0 / Q.ntiles);
        const unsigned tw = Q.tiles[tile];
        const int G0 = (int)(tw & 0xffff) * TR, H0 = (int)(tw >> 16) * TC;
        const int c0 = (int)((long long)split * Q.nch / Q.ns);
        const int c1 = (int)((long long)(split + 1) * Q.nch / Q.ns);
        const int ng = Q.ng, gpad = Q.gpad;
        const size_t slice_stride = (size_t)Q.nch * NKS * gpad * KS;

        StageSrc S;
        S.a_base = reinterpret_cast<const char *>(Q.M + min(G0 + lane, ng - 1));
        S.a_row_bytes = (long long)ng * 16;
        S.kmax = Q.K - 1;
        {
            const int row = 64 * (wave & 1) + (lane >> 2);
            const int seg = (lane & 3) ^ ((row >> 1) & 3);
            S.b_base = reinterpret_cast<const char *>(Q.SB + (wave >> 1) * slice_stride) +
                       ((size_t)(H0 + row) * KS * 2 + seg * 16);
        }
        S.b_step_bytes = (size_t)gpad * KS * 2;
        S.w = Q.w + (size_t)v * Q.wstride;
        S.eb = Q.EB;
        S.ea = Q.EA + (size_t)v * Q.nch * gpad;
        S.gpad = gpad;
        S.G0 = G0;
        S.H0 = H0;

        SplitAcc acc;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc.re[cb][r] = acc.im[cb][r] = 0.0;

        // k-steps [s0, s1) of the launch's chunk range; pair of step x: (chunk0 * 8 + x) * 16
        const long long s0 = (long long)c0 * NKS, s1 = (long long)c1 * NKS;
        const long long tbase = (long long)Q.chunk0 * SKP;
        const long long K = Q.K;
        const bool in = G0 + 16 * (wave >> 1) + li < ng;  // this lane's slicing row is inside the matrix

        stage_issue(stage0, ebufs[c0 & 1], S, tbase + s0 * KSP, s0, wave, lane);
        BGW_WAIT_VM(0);
        stage_barrier();

        for (int ch = c0; ch < c1; ++ch) {
            const int *E = reinterpret_cast<const int *>(ebufs[ch & 1]);
            unsigned char *En = ebufs[(ch + 1) & 1];
            // slicing scale of this lane's row: 2^(8 - eA)
            const double up =
                in ? pow2(8 - (int)reinterpret_cast<const signed char *>(E)[512 + 16 * (wave >> 1) + li]) : 0.0;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int p = 0; p < NGR; ++p)
#pragma unroll
                    for (int ri = 0; ri < 2; ++ri) acc.g[cb][p][ri] = (float4_t){0.f, 0.f, 0.f, 0.f};
            const long long xb = (long long)ch * NKS;  // even: step xb uses stage0
#pragma unroll 1
            for (int ks = 0; ks < NKS; ks += 2) {
                split_step(stage0, stage1, En, S, xb + ks, s1, tbase, K, up, wave, lane, li, lq, acc);
                split_step(stage1, stage0, En, S, xb + ks + 1, s1, tbase, K, up, wave, lane, li, lq, acc);
            }
            split_flush(acc, E, wave, li, lq);
        }

        double2 *o = Q.out + (size_t)v * Q.vstride + (size_t)split * ng * ng;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int G = G0 + 16 * (wave >> 1) + 4 * lq + r;
                const int H = H0 + 64 * (wave & 1) + 16 * cb + li;
                if (G < ng && H < ng) {
                    double2 val = make_double2(acc.re[cb][r], acc.im[cb][r]);
                    if (Q.add) val = cadd(val, o[(size_t)G * ng + H]);
                    o[(size_t)G * ng + H] = val;
                }
            }
        __syncthreads();  // the stages and exponent buffers are reused by the block's next item
    }
}

// FP64 head rows of every weight vector of one q in one pass over M:
// hw[s][v][H] = sum_{t in K range s} w_v[t] conj(M_t(head)) M_t(H), for the
// vectors [v0, v0 + nv) (at most kHeadVec).  grid: (ng / 256, ranges).
constexpr int kHeadVec = 16;
__global__ __launch_bounds__(256) void k_headwing(const double2 *__restrict__ M, long long K, int ng, int head,
                                                  const double *__restrict__ w, long long wstride, int v0, int nv,
                                                  long long kper, double2 *__restrict__ hw, int nvec) {
    const int H = blockIdx.x * blockDim.x + threadIdx.x;
    if (H >= ng) return;
    const long long k0 = blockIdx.y * kper, k1 = min(K, k0 + kper);
    double sr[kHeadVec], si[kHeadVec];
#pragma unroll
    for (int v = 0; v < kHeadVec; ++v) sr[v] = si[v] = 0.0;
    // four pairs' loads in flight at a time; every sum keeps the order of t
    constexpr int U = 4;
    for (long long t0 = k0; t0 < k1; t0 += U) {
        double2 p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long t = t0 + u;
            if (t < k1) {
                const double2 a = M[t * ng + head], b = M[t * ng + H];
                p[u] = make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);  // conj(a) b
            } else {
                p[u] = make_double2(0.0, 0.0);
            }
        }
#pragma unroll
        for (int v = 0; v < kHeadVec; ++v) {
            if (v < nv) {
                const double *wv = w + (size_t)(v0 + v) * wstride;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const double wt = t0 + u < k1 ? wv[t0 + u] : 0.0;
                    sr[v] = fma(wt, p[u].x, sr[v]);
                    si[v] = fma(wt, p[u].y, si[v]);
                }
            }
        }
    }
#pragma unroll
    for (int v = 0; v < kHeadVec; ++v)
        if (v < nv) hw[((size_t)blockIdx.y * nvec + v0 + v) * ng + H] = make_double2(sr[v], si[v]);
}

// Row and column `head` of every output matrix of one q: with A from vector
// va and (real frequency axis) B from vector vb = va + 1,
// chi[head][H] (+)= pf (A_H + i B_H), chi[H][head] (+)= pf (conj A_H + i conj B_H),
// where A_H = sum_s hw[s][va][H]; without B, chi is Hermitian and its head
// diagonal exactly real.  grid: (ng / 256, output matrices).
__global__ void k_headwing_write(const double2 *__restrict__ hw, int nsplit, int nvec, int ng, int head, double pf,
                                 double2 *__restrict__ chi, int two, int accumulate) {
    const int H = blockIdx.x * blockDim.x + threadIdx.x;
    if (H >= ng) return;
    const int f = blockIdx.y;
    const int va = two ? 2 * f : f;
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    for (int p = 0; p < nsplit; ++p) a = cadd(a, hw[((size_t)p * nvec + va) * ng + H]);
    if (two)
        for (int p = 0; p < nsplit; ++p) b = cadd(b, hw[((size_t)p * nvec + va + 1) * ng + H]);
    if (H == head) {
        a.y = 0.0;
        b.y = 0.0;
    }
    // row: A_H + i B_H; column: conj(A_H) + i conj(B_H)
    const double2 vr = make_double2(pf * (a.x - b.y), pf * (a.y + b.x));
    const double2 vc = make_double2(pf * (a.x + b.y), pf * (-a.y + b.x));
    double2 *cm = chi + (size_t)f * ng * ng;
    const size_t rowi = (size_t)head * ng + H, coli = (size_t)H * ng + head;
    if (accumulate) {
        cm[rowi] = cadd(cm[rowi], vr);
        if (H != head) cm[coli] = cadd(cm[coli], vc);
    } else {
        cm[rowi] = vr;
        if (H != head) cm[coli] = vc;
    }
}

// ---------------------------------------------------------------- host side

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
            cus = v;
        else
            cus = 256;
    }
    return cus;
}

int split_gpad(int ng) { return (ng + TC - 1) / TC * TC; }

long long split_chunks(long long K) { return (K + SKP - 1) / SKP; }

size_t split_slices_only_bytes(long long nch, int ng) { return (size_t)nch * NSL * SK * split_gpad(ng) * 2; }

size_t split_slice_bytes(long long nch, int ng) {
    return split_slices_only_bytes(nch, ng) + sizeof(int) * (size_t)nch * split_gpad(ng);
}

// Upper tiles in walk order: bands of eight row tiles, each band walked
// column tile by column tile.
void split_tiles(int ng, std::vector<unsigned> &out) {
    const int nti = (ng + TR - 1) / TR, ntj = (ng + TC - 1) / TC;
    out.clear();
    for (int b0 = 0; b0 < nti; b0 += 8)
        for (int J = 0; J < ntj; ++J)
            for (int I = b0; I < std::min(nti, b0 + 8); ++I)
                if (I <= 2 * J + 1) out.push_back((unsigned)I | ((unsigned)J << 16));
}

int split_grid() { return device_cus() / 8 * 8; }

int launch_split_slices(const double2 *M, long long K, int ng, long long c0, int nch, unsigned short *S, int *E,
                        const double *w, long long wstride, int nvec, signed char *EA, hipStream_t st) {
    const int gpad = split_gpad(ng);
    hipLaunchKernelGGL(k_split_slice, dim3(gpad / 32, nch), dim3(SLICE_T), 0, st, M, K, ng, gpad, c0, nch, S, E, w,
                       wstride, nvec, EA);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int launch_chi_split(const SplitQ *qs, int nq, long long nitems, hipStream_t st) {
    if (nitems <= 0) return BGW_OK;
    const long long g = std::max<long long>(8, std::min<long long>(nitems, split_grid()));
    hipLaunchKernelGGL(k_chi_split, dim3((unsigned)g), dim3(XT), 0, st, qs, nq, 0ll, nitems);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int launch_headwing(const double2 *M, long long K, int ng, int head, const double *w, long long wstride, int nvec,
                    int nsplit, double2 *hw, hipStream_t st) {
    const long long kper = (K + nsplit - 1) / nsplit;
    for (int v0 = 0; v0 < nvec; v0 += kHeadVec) {
        const int nv = std::min(kHeadVec, nvec - v0);
        hipLaunchKernelGGL(k_headwing, dim3((ng + 255) / 256, nsplit), dim3(256), 0, st, M, K, ng, head, w, wstride,
                           v0, nv, kper, hw, nvec);
    }
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int launch_headwing_write(const double2 *hw, int nsplit, int nvec, int ng, int head, double pf, double2 *chi, int nout,
                          int two, int accumulate, hipStream_t st) {
    hipLaunchKernelGGL(k_headwing_write, dim3((ng + 255) / 256, nout), dim3(256), 0, st, hw, nsplit, nvec, ng, head,
                       pf, chi, two, accumulate);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

}  // namespace bgw
