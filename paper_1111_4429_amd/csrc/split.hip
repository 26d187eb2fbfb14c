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
// all exact in BF16.  Stored slices: d1, d2, d3, d3*2^-8, d4*2^-8.
//
// Products (k_herk_split), grouped by weight 2^-8p:
//     p = 0: a1 b1                                   (FP32-exact: |sum| <= 2^24)
//     p = 1: a1 b2 + a2 b1                           (FP32-exact: |sum| <= 2^24)
//     p = 2,3 together, pre-scaled: a1 b3 + a2 b2 + a3 b1
//                       + a1 b4' + a2 b3' + a3' b2 + a4' b1
// Ten BF16 MFMA products per (Re, Im); at each chunk end the three FP32 sums
// are combined in FP64 with the chunk scales 2^(eA + eB - 16) and added to
// FP64 accumulators.  Terms with weight <= 2^-32 are dropped; the rounding of
// the third group is at 2^-40.  Expected relative error ~1e-10.
//
// The head row/column (G = 0) is recomputed in FP64 from M (k_headwing)
// because v(q+G) ~ 1/q^2 amplifies it in epsilon.
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
constexpr int NSL = 5;       // stored slices
constexpr int TT = 64;       // output tile (G and G')
constexpr int ROWB = 80;     // LDS row stride in bytes (64 data + 16 pad: conflict-free 16-B reads)

__device__ inline double pow2(int e) { return __longlong_as_double((long long)(e + 1023) << 52); }

__device__ inline unsigned short bf16_bits_exact(double v) {
    // v is an integer of at most 9 significant bits times a power of two: exact in BF16
    const float f = (float)v;
    return (unsigned short)(__float_as_uint(f) >> 16);
}
}  // namespace

// One thread per (chunk, column).  S: [NSL][nchunk][NKS][gpad][KS] bf16 bits;
// E: [nchunk][gpad].  Rows t0 .. t0 + nchunk*128 of M (zero beyond K).
__global__ void k_split_slice(const double2 *__restrict__ M, long long K, int ng, int gpad,
                              const double *__restrict__ w, long long t0, int nchunk, unsigned short *__restrict__ S,
                              int *__restrict__ E) {
    const int G = blockIdx.x * blockDim.x + threadIdx.x;
    const int chunk = blockIdx.y;
    if (G >= gpad || chunk >= nchunk) return;
    const long long tb = t0 + (long long)chunk * SKP;
    const bool col = G < ng;
    double mx = 0.0;
    if (col)
        for (int i = 0; i < SKP; ++i) {
            const long long t = tb + i;
            if (t >= K) break;
            const double2 m = M[t * ng + G];
            const double s = w ? w[t] : 1.0;
            mx = fmax(mx, fmax(fabs(s * m.x), fabs(s * m.y)));
        }
    int e = 0;
    if (mx > 0.0) (void)frexp(mx, &e);  // mx < 2^e
    E[(size_t)chunk * gpad + G] = e;
    const double up = pow2(8 - e);
    const size_t slice_stride = (size_t)nchunk * NKS * gpad * KS;
    for (int i4 = 0; i4 < SKP; i4 += 4) {
        // 4 pairs -> 8 consecutive k' values
        unsigned short d[NSL][8];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const long long t = tb + i4 + j;
            double2 m = make_double2(0.0, 0.0);
            double s = 0.0;
            if (col && t < K) {
                m = M[t * ng + G];
                s = w ? w[t] : 1.0;
            }
#pragma unroll
            for (int part = 0; part < 2; ++part) {
                const double x = s * (part ? m.y : m.x);
                const double y = x * up;
                const double d1 = rint(y);
                double r = (y - d1) * 256.0;
                const double d2 = rint(r);
                r = (r - d2) * 256.0;
                const double d3 = rint(r);
                r = (r - d3) * 256.0;
                const double d4 = rint(r);
                const int q = 2 * j + part;
                d[0][q] = bf16_bits_exact(d1);
                d[1][q] = bf16_bits_exact(d2);
                d[2][q] = bf16_bits_exact(d3);
                d[3][q] = bf16_bits_exact(d3 * 0.00390625);
                d[4][q] = bf16_bits_exact(d4 * 0.00390625);
            }
        }
        const int kp = 2 * i4;  // first k' of the group
        const int ks = kp / KS, kk = kp % KS;
#pragma unroll
        for (int sl = 0; sl < NSL; ++sl) {
            uint4 pk;
            pk.x = d[sl][0] | ((unsigned)d[sl][1] << 16);
            pk.y = d[sl][2] | ((unsigned)d[sl][3] << 16);
            pk.z = d[sl][4] | ((unsigned)d[sl][5] << 16);
            pk.w = d[sl][6] | ((unsigned)d[sl][7] << 16);
            unsigned short *dst =
                S + sl * slice_stride + (((size_t)chunk * NKS + ks) * gpad + G) * KS + kk;
            *reinterpret_cast<uint4 *>(dst) = pk;
        }
    }
}

namespace {
__device__ inline bf16x8_t as_bf16x8(uint4 u) {
    bf16x8_t r;
    __builtin_memcpy(&r, &u, 16);
    return r;
}
// (x[2m], x[2m+1]) -> (x[2m+1], -x[2m]) for the four pairs of a fragment
__device__ inline uint4 swap_neg(uint4 u) {
    uint4 r;
    r.x = (u.x >> 16) | (((u.x & 0xffffu) ^ 0x8000u) << 16);
    r.y = (u.y >> 16) | (((u.y & 0xffffu) ^ 0x8000u) << 16);
    r.z = (u.z >> 16) | (((u.z & 0xffffu) ^ 0x8000u) << 16);
    r.w = (u.w >> 16) | (((u.w & 0xffffu) ^ 0x8000u) << 16);
    return r;
}
#define MFMA(a, b, c) __builtin_amdgcn_mfma_f32_16x16x32_bf16((a), (b), (c), 0, 0, 0)
}  // namespace

// grid.x: upper-triangle 64x64 tiles, grid.y: splits of the chunk range.
// part[split][ng][ng] (+)= chunk sums in FP64 (no prefactor).
__global__ __launch_bounds__(256) void k_herk_split(const unsigned short *__restrict__ SA,
                                                    const int *__restrict__ EA,
                                                    const unsigned short *__restrict__ SB,
                                                    const int *__restrict__ EB, int ng, int gpad, int nt,
                                                    int nchunk, int chunks_per_split, double2 *__restrict__ part,
                                                    int add) {
    __shared__ __attribute__((aligned(16))) unsigned char As[NSL][TT][ROWB];
    __shared__ __attribute__((aligned(16))) unsigned char Bs[NSL][TT][ROWB];

    int u = blockIdx.x, ti = 0;
    while (u >= nt - ti) {
        u -= nt - ti;
        ++ti;
    }
    const int tj = ti + u;
    const int G0 = ti * TT, H0 = tj * TT;
    const int c0 = blockIdx.y * chunks_per_split;
    const int c1 = min(nchunk, c0 + chunks_per_split);
    const size_t slice_stride = (size_t)nchunk * NKS * gpad * KS;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int li = lane & 15, lq = lane >> 4;

    double4_t are[2][2], aim[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            are[a][b] = (double4_t){0.0, 0.0, 0.0, 0.0};
            aim[a][b] = (double4_t){0.0, 0.0, 0.0, 0.0};
        }

    for (int ch = c0; ch < c1; ++ch) {
        float4_t g[3][2][2][2];  // [group][re/im][a][b]
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int ri = 0; ri < 2; ++ri)
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) g[p][ri][a][b] = (float4_t){0.f, 0.f, 0.f, 0.f};

        for (int ks = 0; ks < NKS; ++ks) {
            __syncthreads();
            // stage 5 slices x 64 rows x 64 B for A and B: 1280 16-byte pieces each
            for (int e = tid; e < NSL * TT * 4; e += 256) {
                const int sl = e / (TT * 4), rem = e % (TT * 4), row = rem >> 2, seg = rem & 3;
                const size_t off = sl * slice_stride + (((size_t)ch * NKS + ks) * gpad) * KS;
                const uint4 va = *reinterpret_cast<const uint4 *>(SA + off + (size_t)(G0 + row) * KS + seg * 8);
                const uint4 vb = *reinterpret_cast<const uint4 *>(SB + off + (size_t)(H0 + row) * KS + seg * 8);
                *reinterpret_cast<uint4 *>(&As[sl][row][seg * 16]) = va;
                *reinterpret_cast<uint4 *>(&Bs[sl][row][seg * 16]) = vb;
            }
            __syncthreads();
            uint4 af[NSL][2], bf[NSL][2];
#pragma unroll
            for (int sl = 0; sl < NSL; ++sl)
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    af[sl][a] = *reinterpret_cast<const uint4 *>(&As[sl][wr * 32 + 16 * a + li][lq * 16]);
                    bf[sl][a] = *reinterpret_cast<const uint4 *>(&Bs[sl][wc * 32 + 16 * a + li][lq * 16]);
                }
            // slice indices: 0 = d1, 1 = d2, 2 = d3, 3 = d3', 4 = d4'
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const bf16x8_t b1 = as_bf16x8(bf[0][b]), b2 = as_bf16x8(bf[1][b]), b3 = as_bf16x8(bf[2][b]);
                const bf16x8_t b3p = as_bf16x8(bf[3][b]), b4p = as_bf16x8(bf[4][b]);
                const bf16x8_t y1 = as_bf16x8(swap_neg(bf[0][b])), y2 = as_bf16x8(swap_neg(bf[1][b]));
                const bf16x8_t y3 = as_bf16x8(swap_neg(bf[2][b])), y3p = as_bf16x8(swap_neg(bf[3][b]));
                const bf16x8_t y4p = as_bf16x8(swap_neg(bf[4][b]));
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const bf16x8_t a1 = as_bf16x8(af[0][a]), a2 = as_bf16x8(af[1][a]), a3 = as_bf16x8(af[2][a]);
                    const bf16x8_t a3p = as_bf16x8(af[3][a]), a4p = as_bf16x8(af[4][a]);
                    g[0][0][a][b] = MFMA(a1, b1, g[0][0][a][b]);
                    g[0][1][a][b] = MFMA(a1, y1, g[0][1][a][b]);
                    g[1][0][a][b] = MFMA(a1, b2, g[1][0][a][b]);
                    g[1][0][a][b] = MFMA(a2, b1, g[1][0][a][b]);
                    g[1][1][a][b] = MFMA(a1, y2, g[1][1][a][b]);
                    g[1][1][a][b] = MFMA(a2, y1, g[1][1][a][b]);
                    g[2][0][a][b] = MFMA(a1, b3, g[2][0][a][b]);
                    g[2][0][a][b] = MFMA(a2, b2, g[2][0][a][b]);
                    g[2][0][a][b] = MFMA(a3, b1, g[2][0][a][b]);
                    g[2][0][a][b] = MFMA(a1, b4p, g[2][0][a][b]);
                    g[2][0][a][b] = MFMA(a2, b3p, g[2][0][a][b]);
                    g[2][0][a][b] = MFMA(a3p, b2, g[2][0][a][b]);
                    g[2][0][a][b] = MFMA(a4p, b1, g[2][0][a][b]);
                    g[2][1][a][b] = MFMA(a1, y3, g[2][1][a][b]);
                    g[2][1][a][b] = MFMA(a2, y2, g[2][1][a][b]);
                    g[2][1][a][b] = MFMA(a3, y1, g[2][1][a][b]);
                    g[2][1][a][b] = MFMA(a1, y4p, g[2][1][a][b]);
                    g[2][1][a][b] = MFMA(a2, y3p, g[2][1][a][b]);
                    g[2][1][a][b] = MFMA(a3p, y2, g[2][1][a][b]);
                    g[2][1][a][b] = MFMA(a4p, y1, g[2][1][a][b]);
                }
            }
        }
        // flush the chunk in FP64 with the chunk-column scales
        // D layout of 16x16x32: lane l, register r -> row 4 (l/16) + r, col l % 16
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int H = H0 + wc * 32 + 16 * b + li;
                const int eb = EB[(size_t)ch * gpad + H];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int G = G0 + wr * 32 + 16 * a + 4 * lq + r;
                    const double sc = pow2(EA[(size_t)ch * gpad + G] + eb - 16);
                    const double vre = (double)g[0][0][a][b][r] + (double)g[1][0][a][b][r] * 0.00390625 +
                                       (double)g[2][0][a][b][r] * 0.0000152587890625;
                    const double vim = (double)g[0][1][a][b][r] + (double)g[1][1][a][b][r] * 0.00390625 +
                                       (double)g[2][1][a][b][r] * 0.0000152587890625;
                    are[a][b][r] += vre * sc;
                    aim[a][b][r] += vim * sc;
                }
            }
    }
    double2 *o = part + (size_t)blockIdx.y * ng * ng;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int G = G0 + wr * 32 + 16 * a + 4 * lq + r;
                const int H = H0 + wc * 32 + 16 * b + li;
                if (G < ng && H < ng) {
                    double2 v = make_double2(are[a][b][r], aim[a][b][r]);
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
    for (long long t = k0; t < k1; ++t) {
        const double2 a = M[t * ng + head];
        const double2 b = M[t * ng + H];
        const double wt = w[t];
        s.x += wt * (a.x * b.x + a.y * b.y);
        s.y += wt * (a.x * b.y - a.y * b.x);
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

namespace {
struct SplitPlan {
    int gpad, nt;
    long long tiles;
    long long sc_pairs;  // pairs per super-chunk (multiple of 128)
    int nsplit;
    size_t slice_bytes;  // one side, one super-chunk
};

SplitPlan make_plan(long long K, int ng) {
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
    long long want = (2048 + p.tiles - 1) / p.tiles;
    want = std::min<long long>(want, nch);
    p.nsplit = (int)std::max<long long>(1, std::min<long long>(want, 64));
    return p;
}

constexpr int kHeadSplits = 64;

size_t al(size_t b) { return (b + 255) / 256 * 256; }
}  // namespace

int split_workspace_bytes(long long K, int ng, size_t *bytes) {
    const SplitPlan p = make_plan(K, ng);
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
SplitLayout split_layout(long long K, int ng, void *ws) {
    const SplitPlan p = make_plan(K, ng);
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
                        int nch, hipStream_t st) {
    dim3 sg((L.gpad + 255) / 256, nch);
    hipLaunchKernelGGL(k_split_slice, sg, dim3(256), 0, st, M, K, ng, L.gpad, w, t0, nch, L.SA, L.EA);
    hipLaunchKernelGGL(k_split_slice, sg, dim3(256), 0, st, M, K, ng, L.gpad, (const double *)nullptr, t0, nch, L.SB,
                       L.EB);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

// Returns the number of split slots written in *used.
int launch_split_gemm(const SplitLayout &L, int ng, int nch, int add, int *used, hipStream_t st) {
    const int ns = std::min(L.nsplit, nch);
    const int cps = (nch + ns - 1) / ns;
    const int nsplit_used = (nch + cps - 1) / cps;
    hipLaunchKernelGGL(k_herk_split, dim3((unsigned)L.tiles, nsplit_used), dim3(256), 0, st, L.SA, L.EA, L.SB, L.EB,
                       ng, L.gpad, L.nt, nch, cps, L.part, add);
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
