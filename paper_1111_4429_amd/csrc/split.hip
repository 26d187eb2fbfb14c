// Split-precision chi sum: chi = pf * X_w^T (X + iY) (real embedding of
// M^H diag(w) M, see chi.hip) computed from BF16 digit slices on MFMA with
// FP32 accumulation, recombined in FP64.
//
// Slicing (k_split_slice).  The real contraction index k' = 2t + part is cut
// into chunks of 256 (128 pairs).  Within a chunk every column G gets its own
// power-of-two scale 2^e (e = exponent of the chunk-column max), and each
// value is written as four signed base-256 digits:
//     x = 2^(e-8) (d1 + d2 2^-8 + d3 2^-16 + d4 2^-24 + r),  |d1| <= 256,
//     |d2|,|d3|,|d4| <= 128, |r| <= 2^-25,
// all exact in BF16.  Stored slices: d1, d2, d3, d4 (8 bytes per value).
//
// Products (k_herk_split), grouped by weight 2^-8p, one FP32 sum per group:
//     p = 0: a1 b1                                   (FP32-exact: |sum| <= 2^24)
//     p = 1: a1 b2 + a2 b1                           (FP32-exact: |sum| <= 2^24)
//     p = 2: a1 b3 + a2 b2 + a3 b1                   (rounded at 2^-24 of the group)
//     p = 3: a1 b4 + a2 b3 + a3 b2 + a4 b1
// Ten BF16 MFMA products per (Re, Im); at each chunk end the four FP32 sums
// are combined in FP64 with the chunk scales 2^(eA + eB - 16) and added to
// FP64 accumulators.  Terms with weight <= 2^-32 are dropped; the rounding of
// the last two groups is at 2^-40 and below.  Expected relative error ~1e-10.
//
// The head row/column (G = 0) is recomputed in FP64 from M (k_headwing)
// because v(q+G) ~ 1/q^2 amplifies it in epsilon.
#include <algorithm>
#include <cstdlib>

#include "common.h"

namespace bgw {

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef double double4_t __attribute__((ext_vector_type(4)));

namespace {
constexpr int SK = 256;      // real contraction rows per exact chunk
constexpr int SKP = SK / 2;  // pairs per chunk
constexpr int KS = 32;       // real rows per MFMA k-step (16x16x32)
constexpr int NKS = SK / KS; // k-steps per chunk
constexpr int NSL = 4;       // stored slices
constexpr int NGR = 4;       // FP32 product groups
constexpr int TT = 64;       // output tile (G and G')

__device__ inline double pow2(int e) { return __longlong_as_double((long long)(e + 1023) << 52); }

__device__ inline unsigned short bf16_bits_exact(double v) {
    // v is an integer of at most 9 significant bits times a power of two: exact in BF16
    const float f = (float)v;
    return (unsigned short)(__float_as_uint(f) >> 16);
}
}  // namespace

// Block = one chunk x 32 columns.  Thread t owns column G = 32 blockIdx.x +
// (t/4) % 32 and, in each of the k-steps 4 (t/128) .. +3, the four pairs
// 4 (t%4) .. +3; it keeps its 16 pairs in registers, so M is read once for
// both sides.  With this assignment every 16-byte store instruction of a wave
// writes 1 KB of contiguous slice memory.  Side A (X_w, weighted by w) and
// side B (X) are written when their slice pointer is non-null.
// S: [NSL][nchunk][NKS][gpad][KS] bf16 bits, each group of 8 values holding four
// pairs as (Re t0..t3, Im t0..t3); E: [nchunk][gpad].
// Rows t0 .. t0 + nchunk*128 of M (zero beyond K).
__global__ __launch_bounds__(256) void k_split_slice(const double2 *__restrict__ M, long long K, int ng, int gpad,
                                                     const double *__restrict__ w, long long t0, int nchunk,
                                                     unsigned short *__restrict__ SA, int *__restrict__ EA,
                                                     unsigned short *__restrict__ SB, int *__restrict__ EB) {
    __shared__ double red[2][8][32];
    const int q = threadIdx.x & 3, cl = (threadIdx.x >> 2) & 31, kh = threadIdx.x >> 7;
    const int G = blockIdx.x * 32 + cl;
    const int chunk = blockIdx.y;
    const long long tb = t0 + (long long)chunk * SKP;
    const bool col = G < ng;
    double2 m[4][4];  // [k-step i][pair j]
    double s[4][4];
    double mxa = 0.0, mxb = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long long t = tb + (4 * kh + i) * (KS / 2) + 4 * q + j;
            m[i][j] = make_double2(0.0, 0.0);
            s[i][j] = 0.0;
            if (t < K) {
                s[i][j] = w ? w[t] : 1.0;
                if (col) m[i][j] = M[t * ng + G];
            }
            mxa = fmax(mxa, fabs(s[i][j]) * fmax(fabs(m[i][j].x), fabs(m[i][j].y)));
            mxb = fmax(mxb, fmax(fabs(m[i][j].x), fabs(m[i][j].y)));
        }
    red[0][4 * kh + q][cl] = mxa;
    red[1][4 * kh + q][cl] = mxb;
    __syncthreads();
    mxa = 0.0;
    mxb = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        mxa = fmax(mxa, red[0][k][cl]);
        mxb = fmax(mxb, red[1][k][cl]);
    }
    if (G >= gpad) return;
    const size_t slice_stride = (size_t)nchunk * NKS * gpad * KS;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        unsigned short *S = side ? SB : SA;
        int *E = side ? EB : EA;
        if (!S) continue;
        const double mx = side ? mxb : mxa;
        int e = 0;
        if (mx > 0.0) (void)frexp(mx, &e);  // mx < 2^e
        if (q == 0 && kh == 0) E[(size_t)chunk * gpad + G] = e;
        const double up = pow2(8 - e);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int ks = 4 * kh + i;
            unsigned short d[NSL][8];
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int part = 0; part < 2; ++part) {
                    const double v = part ? m[i][j].y : m[i][j].x;
                    const double y = (side ? v : s[i][j] * v) * up;
                    const double d1 = rint(y);
                    double r = (y - d1) * 256.0;
                    const double d2 = rint(r);
                    r = (r - d2) * 256.0;
                    const double d3 = rint(r);
                    r = (r - d3) * 256.0;
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

// LDS stage: [side][slice][64 rows][64 B], the four 16-B segments of row r
// stored in the order seg ^ (r & 3) (conflict-free 16-B fragment reads).
constexpr int SLICE_LDS = TT * KS * 2;          // 4096 B
constexpr int STAGE_LDS = 2 * NSL * SLICE_LDS;  // 32768 B
constexpr int PIECES = 2 * NSL * 4 / 8;         // 1-KB pieces of a stage per wave

typedef __attribute__((address_space(3))) void lds_void_t;

// Block: 8 waves (512 threads) in a 2 x 4 layout over the 64 x 64 tile; wave
// (wr, wc) owns rows wr*32 .. +32 (two 16-row MFMA blocks a) and columns
// wc*16 .. +16.  Two waves per SIMD let one wave's LDS reads and VALU work
// run under the other's MFMAs.
constexpr int HT = 512;  // threads per block

struct HerkAcc {
    float4_t g[NGR][2][2];      // [group][re/im][a]
    double re[2][4], im[2][4];  // FP64 sums of the chunks done so far
};

constexpr int NSTAGE = 4;  // LDS stages: k-steps are loaded NSTAGE - 1 ahead

// vmcnt(n) alone (expcnt and lgkmcnt left at their maxima); vmcnt is split
// over bits 3:0 and 15:14 of the immediate
#define BGW_WAIT_VM(n) __builtin_amdgcn_s_waitcnt(0x0F70 | ((n) & 0xF) | (((n) >> 4) << 14))

// Workgroup barrier for the stage pipeline: the wave's LDS reads are complete
// (lgkmcnt) and its direct-to-LDS loads have been waited for explicitly, so no
// fence is needed; __syncthreads() would also wait for the loads still in
// flight for later stages.
__device__ __forceinline__ void stage_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Copy k-step `step` of the A (rows G0..) and B (rows H0..) slices into a
// stage with direct global->LDS loads.  The stage is 32 pieces of 1 KB
// (slice-side q/4, rows 16 (q%4) .. +16); wave w issues pieces 4w .. 4w+3,
// lane L the 16 B of row 16 (q%4) + L/4 at stored segment L%4.  Addresses: a
// wave-uniform base plus this lane's 32-bit byte offset.
__device__ __forceinline__ void herk_issue(unsigned char *stage, const unsigned short *SA,
                                           const unsigned short *SB, const unsigned (&off)[PIECES],
                                           size_t slice_stride, long long step, int gpad, int wave) {
    const size_t so = (size_t)step * gpad * KS;
#pragma unroll
    for (int i = 0; i < PIECES; ++i) {
        const int q = PIECES * wave + i;
        const int idx = q >> 2;  // 0..3: A slices, 4..7: B slices
        const unsigned short *base = idx < NSL ? SA + idx * slice_stride : SB + (idx - NSL) * slice_stride;
        __builtin_amdgcn_global_load_lds((const void *)(reinterpret_cast<const char *>(base + so) + off[i]),
                                         (lds_void_t *)(stage + idx * SLICE_LDS + (q & 3) * 1024), 16, 0, 0);
    }
}

__device__ __forceinline__ uint4 frag(const unsigned char *slice, int row, int lq) {
    return *reinterpret_cast<const uint4 *>(slice + row * 64 + 16 * (lq ^ (row & 3)));
}

// The wave's fragments of one k-step: the slices of the B column block and of
// the two A row blocks.
struct HerkFrags {
    uint4 b[NSL], a[2][NSL];
};

__device__ __forceinline__ void herk_frags(const unsigned char *stage, HerkFrags &f, int wr, int wc, int li,
                                           int lq) {
    const unsigned char *As = stage, *Bs = stage + NSL * SLICE_LDS;
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) f.b[sl] = frag(Bs + sl * SLICE_LDS, wc * 16 + li, lq);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int sl = 0; sl < NSL; ++sl) f.a[a][sl] = frag(As + sl * SLICE_LDS, wr * 32 + 16 * a + li, lq);
}

// Ten BF16 products per (Re, Im) for the wave's 32 x 16 block of one k-step.
__device__ __forceinline__ void herk_mfma(const HerkFrags &f, HerkAcc &acc) {
    // slice indices: 0 = d1, 1 = d2, 2 = d3, 3 = d4
    const bf16x8_t b1 = as_bf16x8(f.b[0]), b2 = as_bf16x8(f.b[1]), b3 = as_bf16x8(f.b[2]);
    const bf16x8_t b4 = as_bf16x8(f.b[3]);
    const bf16x8_t y1 = as_bf16x8(swap_neg(f.b[0])), y2 = as_bf16x8(swap_neg(f.b[1]));
    const bf16x8_t y3 = as_bf16x8(swap_neg(f.b[2])), y4 = as_bf16x8(swap_neg(f.b[3]));
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const bf16x8_t a1 = as_bf16x8(f.a[a][0]), a2 = as_bf16x8(f.a[a][1]), a3 = as_bf16x8(f.a[a][2]);
        const bf16x8_t a4 = as_bf16x8(f.a[a][3]);
        float4_t(&g0)[2][2] = acc.g[0];
        float4_t(&g1)[2][2] = acc.g[1];
        float4_t(&g2)[2][2] = acc.g[2];
        float4_t(&g3)[2][2] = acc.g[3];
        g0[0][a] = MFMA(a1, b1, g0[0][a]);
        g0[1][a] = MFMA(a1, y1, g0[1][a]);
        g1[0][a] = MFMA(a1, b2, g1[0][a]);
        g1[1][a] = MFMA(a1, y2, g1[1][a]);
        g1[0][a] = MFMA(a2, b1, g1[0][a]);
        g1[1][a] = MFMA(a2, y1, g1[1][a]);
        g2[0][a] = MFMA(a1, b3, g2[0][a]);
        g2[1][a] = MFMA(a1, y3, g2[1][a]);
        g2[0][a] = MFMA(a2, b2, g2[0][a]);
        g2[1][a] = MFMA(a2, y2, g2[1][a]);
        g2[0][a] = MFMA(a3, b1, g2[0][a]);
        g2[1][a] = MFMA(a3, y1, g2[1][a]);
        g3[0][a] = MFMA(a1, b4, g3[0][a]);
        g3[1][a] = MFMA(a1, y4, g3[1][a]);
        g3[0][a] = MFMA(a2, b3, g3[0][a]);
        g3[1][a] = MFMA(a2, y3, g3[1][a]);
        g3[0][a] = MFMA(a3, b2, g3[0][a]);
        g3[1][a] = MFMA(a3, y2, g3[1][a]);
        g3[0][a] = MFMA(a4, b1, g3[0][a]);
        g3[1][a] = MFMA(a4, y1, g3[1][a]);
    }
}

// Chunk-column exponents of this lane's output rows and column, loaded when
// the chunk starts and used when it is flushed.
struct ChunkExp {
    int ea[2][4], eb;
};

__device__ __forceinline__ void herk_exp_load(ChunkExp &E, const int *__restrict__ EA, const int *__restrict__ EB,
                                              long long ch, int gpad, int G0, int H0, int wr, int wc, int li, int lq) {
    E.eb = EB[(size_t)ch * gpad + H0 + wc * 16 + li];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) E.ea[a][r] = EA[(size_t)ch * gpad + G0 + wr * 32 + 16 * a + 4 * lq + r];
}

// Chunk end: combine the four FP32 groups in FP64 with the chunk-column
// scales into the FP64 accumulators and clear them.  D layout of 16x16x32:
// lane l, register r -> row 4 (l/16) + r, col l % 16.
__device__ __forceinline__ void herk_flush(HerkAcc &acc, const ChunkExp &E) {
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double sc = pow2(E.ea[a][r] + E.eb - 16);
            const double vre = (double)acc.g[0][0][a][r] +
                               ((double)acc.g[1][0][a][r] +
                                ((double)acc.g[2][0][a][r] + (double)acc.g[3][0][a][r] * 0.00390625) * 0.00390625) *
                                   0.00390625;
            const double vim = (double)acc.g[0][1][a][r] +
                               ((double)acc.g[1][1][a][r] +
                                ((double)acc.g[2][1][a][r] + (double)acc.g[3][1][a][r] * 0.00390625) * 0.00390625) *
                                   0.00390625;
            acc.re[a][r] += vre * sc;
            acc.im[a][r] += vim * sc;
        }
#pragma unroll
        for (int p = 0; p < NGR; ++p)
#pragma unroll
            for (int ri = 0; ri < 2; ++ri) acc.g[p][ri][a] = (float4_t){0.f, 0.f, 0.f, 0.f};
    }
}
// The k-step loop over [s0, s1) (a whole number of chunks).  The four stages
// are distinct restrict-qualified buffers, which tells the compiler that the
// loads in flight into one stage do not alias the reads of another, so it
// inserts no wait for them before those reads.
__device__ __forceinline__ void herk_pipeline(unsigned char *__restrict__ stage0, unsigned char *__restrict__ stage1,
                                              unsigned char *__restrict__ stage2, unsigned char *__restrict__ stage3,
                                              const unsigned short *__restrict__ SA,
                                              const unsigned short *__restrict__ SB, const int *__restrict__ EA,
                                              const int *__restrict__ EB, const unsigned (&off)[PIECES],
                                              size_t slice_stride, long long s0, long long s1, int gpad, int G0,
                                              int H0, int wave, int wr, int wc, int li, int lq, HerkAcc &acc) {
    // Each issue is PIECES loads per wave.  Before step x+1 is read, the loads
    // of steps x+2 and x+3 (2 PIECES, when both were issued) may be in flight.
    // The fragments of the current step are read before the loads into the
    // free stage are issued, so no wait on those loads is needed for them.
#define BGW_STEP(cur, nxt_stage, x)                                              \
    {                                                                             \
        HerkFrags f_;                                                             \
        herk_frags(cur, f_, wr, wc, li, lq);                                      \
        __builtin_amdgcn_sched_barrier(0);                                        \
        if ((x) + 3 < s1) herk_issue(nxt_stage, SA, SB, off, slice_stride, (x) + 3, gpad, wave); \
        __builtin_amdgcn_sched_barrier(0);                                        \
        herk_mfma(f_, acc);                                                       \
        if (((x) % NKS) == NKS - 1) herk_flush(acc, E);                           \
        if ((x) + 3 < s1) BGW_WAIT_VM(2 * PIECES);                                \
        else BGW_WAIT_VM(0);                                                      \
        stage_barrier();                                                          \
    }
    herk_issue(stage0, SA, SB, off, slice_stride, s0, gpad, wave);
    herk_issue(stage1, SA, SB, off, slice_stride, s0 + 1, gpad, wave);
    herk_issue(stage2, SA, SB, off, slice_stride, s0 + 2, gpad, wave);
    BGW_WAIT_VM(2 * PIECES);
    stage_barrier();
    ChunkExp E;
    for (long long s = s0; s < s1; s += NSTAGE) {
        if (s % NKS == 0) herk_exp_load(E, EA, EB, s / NKS, gpad, G0, H0, wr, wc, li, lq);
        BGW_STEP(stage0, stage3, s);
        BGW_STEP(stage1, stage0, s + 1);
        BGW_STEP(stage2, stage1, s + 2);
        BGW_STEP(stage3, stage2, s + 3);
    }
#undef BGW_STEP
}
}  // namespace

// Blocks are dealt to the 8 XCDs round-robin (block b runs on XCD b % 8).
// With nsplit a multiple of 8, XCD x works through splits x, x + 8, ... one
// after another, and within a split through the tiles in grouped order, so
// the blocks resident on an XCD stream one range of chunks through its L2
// and share most of their rows.  Otherwise block b takes split b % nsplit and
// grouped tile b / nsplit.
// The k-steps run through four LDS stages filled by direct global->LDS
// loads: the slices of the next three steps stream in while the current one
// feeds the MFMAs.
// part[split][ng][ng] (+)= chunk sums in FP64 (no prefactor).
__global__ __launch_bounds__(HT) void k_herk_split(const unsigned short *__restrict__ SA,
                                                   const int *__restrict__ EA,
                                                   const unsigned short *__restrict__ SB,
                                                   const int *__restrict__ EB, int ng, int gpad, int nt,
                                                   int nchunk, int nsplit, int chunks_per_split,
                                                   double2 *__restrict__ part, int add) {
    __shared__ __attribute__((aligned(1024))) unsigned char stage0[STAGE_LDS];
    __shared__ __attribute__((aligned(1024))) unsigned char stage1[STAGE_LDS];
    __shared__ __attribute__((aligned(1024))) unsigned char stage2[STAGE_LDS];
    __shared__ __attribute__((aligned(1024))) unsigned char stage3[STAGE_LDS];

    const int ntiles = nt * (nt + 1) / 2;
    int split, u;
    if (nsplit % 8 == 0) {
        const int x = blockIdx.x % 8, j = blockIdx.x / 8;
        split = x + 8 * (j / ntiles);
        u = j % ntiles;
    } else {
        split = blockIdx.x % nsplit;
        u = blockIdx.x / nsplit;
    }
    int ti, tj;
    grouped_tile(u, nt, ti, tj);
    const int G0 = ti * TT, H0 = tj * TT;
    const int c0 = split * chunks_per_split;
    const int c1 = min(nchunk, c0 + chunks_per_split);
    const size_t slice_stride = (size_t)nchunk * NKS * gpad * KS;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wr = wave >> 2, wc = wave & 3;
    const int li = lane & 15, lq = lane >> 4;

    // this lane's source offsets (bytes) for its pieces of a stage
    unsigned off[PIECES];
#pragma unroll
    for (int i = 0; i < PIECES; ++i) {
        const int q = PIECES * wave + i;
        const int row = 16 * (q & 3) + (lane >> 2);
        const int seg = (lane & 3) ^ (row & 3);
        off[i] = (unsigned)((((q >> 2) < NSL ? G0 : H0) + row) * KS * 2 + seg * 16);
    }

    HerkAcc acc;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc.re[a][r] = acc.im[a][r] = 0.0;
#pragma unroll
        for (int p = 0; p < NGR; ++p)
#pragma unroll
            for (int ri = 0; ri < 2; ++ri) acc.g[p][ri][a] = (float4_t){0.f, 0.f, 0.f, 0.f};
    }

    const long long s0 = (long long)c0 * NKS, s1 = (long long)c1 * NKS;  // s1 - s0: a multiple of NKS (8)
    herk_pipeline(stage0, stage1, stage2, stage3, SA, SB, EA, EB, off, slice_stride, s0, s1, gpad, G0, H0, wave, wr,
                  wc, li, lq, acc);
    double2 *o = part + (size_t)split * ng * ng;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int G = G0 + wr * 32 + 16 * a + 4 * lq + r;
            const int H = H0 + wc * 16 + li;
            if (G < ng && H < ng) {
                double2 v = make_double2(acc.re[a][r], acc.im[a][r]);
                if (add) v = cadd(v, o[(size_t)G * ng + H]);
                o[(size_t)G * ng + H] = v;
            }
        }
}

// FP64 head row: hw[s][H] = sum_{t in split s} w_t conj(M_t(head)) M_t(H)
__global__ void k_headwing(const double2 *__restrict__ M, long long K, int ng, int head,
                           const double *__restrict__ w, long long kper, double2 *__restrict__ hw) {
    const int H = blockIdx.x * blockDim.x + threadIdx.x;
    if (H >= ng) return;
    const long long k0 = blockIdx.y * kper, k1 = min(K, k0 + kper);
    double2 s = make_double2(0.0, 0.0);
    // eight pairs' loads in flight at a time; the sum keeps the order of t
    constexpr int U = 8;
    for (long long t0 = k0; t0 < k1; t0 += U) {
        double2 a[U], b[U];
        double wt[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long t = t0 + u;
            const bool in = t < k1;
            a[u] = in ? M[t * ng + head] : make_double2(0.0, 0.0);
            b[u] = in ? M[t * ng + H] : make_double2(0.0, 0.0);
            wt[u] = in ? w[t] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s.x += wt[u] * (a[u].x * b[u].x + a[u].y * b[u].y);
            s.y += wt[u] * (a[u].x * b[u].y - a[u].y * b[u].x);
        }
    }
    hw[(size_t)blockIdx.y * ng + H] = s;
}

// chi[head][H] (+)= pf sum_s hw[s][H]; chi[H][head] (+)= conj of it; chi[head][head] real.
__global__ void k_headwing_write(const double2 *__restrict__ hw, int nsplit, int ng, int head, double pf,
                                 double2 *__restrict__ chi, int accumulate) {
    const int H = blockIdx.x * blockDim.x + threadIdx.x;
    if (H >= ng) return;
    double2 s = make_double2(0.0, 0.0);
    for (int p = 0; p < nsplit; ++p) s = cadd(s, hw[(size_t)p * ng + H]);
    double2 v = make_double2(pf * s.x, pf * s.y);
    if (H == head) v.y = 0.0;
    const size_t rowi = (size_t)head * ng + H, coli = (size_t)H * ng + head;
    if (accumulate) {
        chi[rowi] = cadd(chi[rowi], v);
        if (H != head) chi[coli] = cadd(chi[coli], make_double2(v.x, -v.y));
    } else {
        chi[rowi] = v;
        if (H != head) chi[coli] = make_double2(v.x, -v.y);
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

namespace {
struct SplitPlan {
    int gpad, nt;
    long long tiles;
    long long sc_pairs;  // pairs per super-chunk (multiple of 128)
    int nsplit;
    size_t slice_bytes;  // one side, one super-chunk
};

// Splits of the chunk range: a multiple of the XCD count (8) when there are
// enough chunks, chosen so that tiles * nsplit fills whole waves of one block
// per CU as evenly as possible.
int choose_nsplit(long long tiles, long long nch) {
    const long long cus = device_cus();
    if (nch < 8) return (int)std::max<long long>(1, nch);
    int best = 8;
    double best_eff = 0.0;
    for (int ns = 8; ns <= 64 && ns <= nch; ns += 8) {
        const long long cps = (nch + ns - 1) / ns;
        const long long used = (nch + cps - 1) / cps;
        if (used != ns) continue;  // keep the XCD-aligned mapping
        const long long blocks = tiles * used;
        const long long rounds = (blocks + cus - 1) / cus;
        // useful chunk-steps over issued block-rounds of the longest block
        const double eff = (double)(tiles * nch) / (double)(rounds * cus * cps);
        if (eff > best_eff * 1.02) {
            best = ns;
            best_eff = eff;
        }
    }
    return best;
}

SplitPlan make_plan(long long K, int ng, int nsplit_override) {
    SplitPlan p;
    p.gpad = (ng + TT - 1) / TT * TT;
    p.nt = p.gpad / TT;
    p.tiles = (long long)p.nt * (p.nt + 1) / 2;
    const long long nch_total = (K + SKP - 1) / SKP;
    // slices of one side for a super-chunk: NSL * SK * gpad * 2 bytes per chunk
    const size_t per_chunk = (size_t)NSL * SK * p.gpad * 2;
    size_t cap = (size_t)6 << 30;  // 6 GiB per side (BGW_SPLIT_SLICE_BYTES overrides)
    if (const char *env = std::getenv("BGW_SPLIT_SLICE_BYTES")) cap = std::max<size_t>(1, std::strtoull(env, nullptr, 10));
    long long nch = std::max<long long>(1, std::min<long long>(nch_total, cap / per_chunk));
    p.sc_pairs = nch * SKP;
    p.slice_bytes = per_chunk * nch;
    p.nsplit = nsplit_override > 0 ? (int)std::min<long long>(nsplit_override, nch) : choose_nsplit(p.tiles, nch);
    return p;
}

constexpr int kHeadSplits = 512;  // K ranges of the FP64 head row (enough blocks to stream M at full rate)

size_t al(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

int split_workspace_bytes(long long K, int ng, int nsplit_override, size_t *bytes) {
    const SplitPlan p = make_plan(K, ng, nsplit_override);
    const long long nch = p.sc_pairs / SKP;
    size_t b = 0;
    b += 2 * al(p.slice_bytes);                                     // SA, SB
    b += 2 * al(sizeof(int) * (size_t)nch * p.gpad);               // EA, EB
    b += al(sizeof(double2) * (size_t)p.nsplit * ng * ng);          // partial sums
    b += al(sizeof(double2) * (size_t)kHeadSplits * ng);            // head row partials
    *bytes = b + 1024;
    return BGW_OK;
}

// Phase launchers used by the API (each phase is timed separately there).
SplitLayout split_layout(long long K, int ng, int nsplit_override, void *ws) {
    const SplitPlan p = make_plan(K, ng, nsplit_override);
    SplitLayout L;
    L.gpad = p.gpad;
    L.nt = p.nt;
    L.tiles = p.tiles;
    L.sc_pairs = p.sc_pairs;
    L.nsplit = p.nsplit;
    const long long nch_sc = p.sc_pairs / SKP;
    char *q = (char *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    L.SA = (unsigned short *)q; q += al(p.slice_bytes);
    L.SB = (unsigned short *)q; q += al(p.slice_bytes);
    L.EA = (int *)q; q += al(sizeof(int) * (size_t)nch_sc * p.gpad);
    L.EB = (int *)q; q += al(sizeof(int) * (size_t)nch_sc * p.gpad);
    L.part = (double2 *)q; q += al(sizeof(double2) * (size_t)p.nsplit * ng * ng);
    L.hw = (double2 *)q;
    return L;
}

int launch_split_slices(const SplitLayout &L, const double2 *M, long long K, int ng, const double *w, long long t0,
                        int nch, bool with_b, hipStream_t st) {
    dim3 sg(L.gpad / 32, nch);
    hipLaunchKernelGGL(k_split_slice, sg, dim3(256), 0, st, M, K, ng, L.gpad, w, t0, nch, L.SA, L.EA,
                       with_b ? L.SB : (unsigned short *)nullptr, with_b ? L.EB : (int *)nullptr);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

// Writes split slots [0, *used).  With add != 0 the slots [0, add) hold the
// sums of earlier super-chunks and at most that many are used.
int launch_split_gemm(const SplitLayout &L, int ng, int nch, int add, int *used, hipStream_t st) {
    int ns = std::min(L.nsplit, nch);
    if (nch < L.sc_pairs / SKP) ns = choose_nsplit(L.tiles, nch);  // short last super-chunk
    ns = std::min(ns, add > 0 ? add : L.nsplit);
    const int cps = (nch + ns - 1) / ns;
    const int nsplit_used = (nch + cps - 1) / cps;
    hipLaunchKernelGGL(k_herk_split, dim3((unsigned)(L.tiles * nsplit_used)), dim3(HT), 0, st, L.SA, L.EA,
                       L.SB, L.EB, ng, L.gpad, L.nt, nch, nsplit_used, cps, L.part, add > 0 ? 1 : 0);
    BGW_HIP(hipGetLastError());
    *used = nsplit_used;
    return BGW_OK;
}

int launch_split_headwing(const SplitLayout &L, const double2 *M, long long K, int ng, int head, const double *w,
                          double pf, double2 *chi, int accumulate, hipStream_t st) {
    const long long kper = (K + kHeadSplits - 1) / kHeadSplits;
    hipLaunchKernelGGL(k_headwing, dim3((ng + 255) / 256, kHeadSplits), dim3(256), 0, st, M, K, ng, head, w, kper,
                       L.hw);
    hipLaunchKernelGGL(k_headwing_write, dim3((ng + 255) / 256), dim3(256), 0, st, L.hw, kHeadSplits, ng, head, pf,
                       chi, accumulate);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

}  // namespace bgw
