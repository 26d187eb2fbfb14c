// Real flavor (the paper's real and complex flavors): with inversion and
// time-reversal symmetry the plane-wave coefficients are real, the pair
// densities M_vc(G) are then real, and the chi sum is a real symmetric
// rank-K update, four times fewer flops than the complex one at the same K
// and half the memory for M and chi.
#include <algorithm>

#include "common.h"

namespace bgw {

typedef double double4_t __attribute__((ext_vector_type(4)));

__global__ void k_real_to_complex(const double *__restrict__ src, long long n, double2 *__restrict__ dst) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        dst[e] = make_double2(src[e], 0.0);
}

// Two real conduction bands as one complex band: dst[k][j] = src[k][2j] +
// i src[k][2j + 1] (the second zero past nc), ncp = ceil(nc / 2) per k.  M is
// linear in the conduction state and real for real coefficients, so the
// complex pair density of (v, j) is M_v,2j + i M_v,2j+1: one transform for two
// pairs.
__global__ void k_pack_band_pairs(const double *__restrict__ src, int nk, int nc, int ngw,
                                  double2 *__restrict__ dst) {
    const int ncp = (nc + 1) / 2;
    const long long n = (long long)nk * ncp * ngw;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const int g = (int)(e % ngw);
        const long long r = e / ngw;
        const int j = (int)(r % ncp), k = (int)(r / ncp);
        const double *sk = src + (size_t)k * nc * ngw;
        const double a = sk[(size_t)(2 * j) * ngw + g];
        const double b = 2 * j + 1 < nc ? sk[(size_t)(2 * j + 1) * ngw + g] : 0.0;
        dst[e] = make_double2(a, b);
    }
}

// The real pair densities from the packed ones: M[(k nv + v) nc + c][G] is
// the real part of Mp[(k nv + v) ncp + c / 2][G] for even c, the imaginary
// part for odd c.
__global__ void k_unpack_pair_halves(const double2 *__restrict__ Mp, int nkv, int nc, int ng, double *__restrict__ M) {
    const int ncp = (nc + 1) / 2;
    const long long n = (long long)nkv * nc * ng;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
        const int G = (int)(e % ng);
        const long long r = e / ng;
        const int c = (int)(r % nc);
        const long long kv = r / nc;
        const double2 z = Mp[((size_t)kv * ncp + c / 2) * ng + G];
        M[e] = (c & 1) ? z.y : z.x;
    }
}

namespace {
constexpr int RT = kSyrkTile;    // output tile edge (128)
constexpr int RKC = kSyrkK;      // contraction rows (pairs) per LDS stage
constexpr int RLDA = RT + 16;    // padded LDS row (doubles): rows 2 apart fall on opposite bank halves
constexpr int RTHREADS = 512;    // 8 waves: 4 x 2 wave blocks of 32 x 64
constexpr int WR = 32, WC = 64;  // wave block edges (rows G, columns H)

// One RT x RT tile of sum_t M[t][G] w_t M[t][H] over t in [k0, k1): 8 waves
// in a 4 x 2 layout, each a 32 x 64 block of 2 x 4 v_mfma_f64_16x16x4 tiles.
// A 128-wide tile gives the real product the same flops per loaded byte as
// the 64-wide complex tile; 8 waves of 64 accumulators each let two blocks
// share a CU (four waves per SIMD to cover the loads).  The next stage's
// values are loaded into registers while the current one feeds the MFMAs,
// then stored into the other of two LDS stages: one barrier per stage.
// Raw sums to o (rows/columns >= ng dropped).
__device__ __forceinline__ void syrk_tile(const double *__restrict__ M, int ng, const double *__restrict__ w,
                                          int G0, int H0, long long k0, long long k1, double *__restrict__ o,
                                          double (*As)[RKC][RLDA], double (*Bs)[RKC][RLDA]) {
    constexpr int NR = WR / 16, NC = WC / 16, LR = RTHREADS / RT, SL = RKC / LR;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int li = lane & 15, lk = lane >> 4;
    double4_t c[NR][NC];
#pragma unroll
    for (int a = 0; a < NR; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b) c[a][b] = (double4_t){0.0, 0.0, 0.0, 0.0};
    // a wave's 64 lanes share one loader row (RT >= 64): row index, bounds
    // and weight are wave-uniform scalars
    const int lcol = tid % RT, lrow = __builtin_amdgcn_readfirstlane(tid / RT);
    const bool gin = G0 + lcol < ng, hin = H0 + lcol < ng;
    double av[SL], bv[SL];
    auto load_stage = [&](long long kk) {
        const double *row = M + (kk + lrow) * ng;
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const long long t = kk + lrow + LR * s;
            const bool in = t < k1;
            const double wt = in ? w[t] : 0.0;
            const double *r = row + (size_t)(LR * s) * ng;
            av[s] = (in && gin) ? wt * r[G0 + lcol] : 0.0;
            bv[s] = (in && hin) ? r[H0 + lcol] : 0.0;
        }
    };
    auto store_stage = [&](int sb) {
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            As[sb][lrow + LR * s][lcol] = av[s];
            Bs[sb][lrow + LR * s][lcol] = bv[s];
        }
    };
    load_stage(k0);
    store_stage(0);
    __syncthreads();
    int cur = 0;
    for (long long kk = k0; kk < k1; kk += RKC) {
        const bool more = kk + RKC < k1;
        if (more) load_stage(kk + RKC);
#pragma unroll
        for (int s = 0; s < RKC / 4; ++s) {
            const int kr = 4 * s + lk;
            double x[NR], y[NC];
#pragma unroll
            for (int a = 0; a < NR; ++a) x[a] = As[cur][kr][wr * WR + 16 * a + li];
#pragma unroll
            for (int b = 0; b < NC; ++b) y[b] = Bs[cur][kr][wc * WC + 16 * b + li];
#pragma unroll
            for (int a = 0; a < NR; ++a)
#pragma unroll
                for (int b = 0; b < NC; ++b) c[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[a], y[b], c[a][b], 0, 0, 0);
        }
        // the other stage was last read before the previous barrier
        if (more) store_stage(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }
    // D layout of v_mfma_f64_16x16x4: lane l, register r -> row 4r + l/16, col l%16
#pragma unroll
    for (int a = 0; a < NR; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int G = G0 + wr * WR + 16 * a + 4 * r + lk;
                const int H = H0 + wc * WC + 16 * b + li;
                if (G < ng && H < ng) o[(size_t)G * ng + H] = c[a][b][r];
            }
}
}  // namespace

// Persistent batched real rank-K update over every (problem, K split, upper
// tile) item; item i on XCD i % 8, each XCD a contiguous eighth of a
// problem's (split, tile) sequence with tiles in grouped order, as the
// complex chi sum.
__global__ __launch_bounds__(512, 4) void k_syrk_f64(const SyrkProb *__restrict__ probs, int nprob, long long i0,
                                                  long long i1) {
    __shared__ double As[2][RKC][RLDA];
    __shared__ double Bs[2][RKC][RLDA];
    for (long long item = i0 + blockIdx.x; item < i1; item += gridDim.x) {
        int lo = 0, hi = nprob - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (probs[mid].item0 <= item) lo = mid;
            else hi = mid - 1;
        }
        const SyrkProb &P = probs[lo];
        const long long local = item - P.item0;
        const long long per = P.nitems / 8;
        const long long u = (local % 8) * per + local / 8;
        const long long ntile = (long long)P.nt * (P.nt + 1) / 2;
        if (u >= ntile * P.ns) continue;  // padding item
        const int split = (int)(u / ntile);
        int ti, tj;
        grouped_tile((int)(u % ntile), P.nt, ti, tj);
        const long long k0 = split * P.kper, k1 = min(P.K, k0 + P.kper);
        syrk_tile(P.M, P.ng, P.w, ti * RT, tj * RT, k0, k1, P.out + (size_t)split * P.ng * P.ng, As, Bs);
    }
}

// chi[G][H] (+)= pf sum over splits of the raw upper sums at (min, max):
// the symmetric mirror.  In place (ns == 1, part == chi, no accumulation):
// each upper element is read once and written to both positions.
// grid.y: output matrix.
__global__ void k_syrk_finalize(const SyrkFin *__restrict__ probs) {
    const SyrkFin P = probs[blockIdx.y];
    const int ng = P.ng;
    const size_t total = (size_t)ng * ng;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int G = (int)(e / ng), H = (int)(e % ng);
        if (P.inplace) {
            if (G > H) continue;
            const double val = P.pf * P.chi[e];
            P.chi[e] = val;
            P.chi[(size_t)H * ng + G] = val;
            continue;
        }
        const size_t src = G <= H ? e : (size_t)H * ng + G;
        double a = 0.0;
        for (int p = 0; p < P.ns; ++p) a += P.part[p * total + src];
        const double val = P.pf * a;
        P.chi[e] = P.accumulate ? P.chi[e] + val : val;
    }
}

// ---------------------------------------------------------------- launchers

int launch_real_to_complex(const double *src, long long n, double2 *dst, hipStream_t st) {
    hipLaunchKernelGGL(k_real_to_complex, dim3((unsigned)std::min<long long>((n + 255) / 256, 8192)), dim3(256), 0,
                       st, src, n, dst);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int launch_pack_band_pairs(const double *src, int nk, int nc, int ngw, double2 *dst, hipStream_t st) {
    const long long n = (long long)nk * ((nc + 1) / 2) * ngw;
    hipLaunchKernelGGL(k_pack_band_pairs, dim3((unsigned)std::min<long long>((n + 255) / 256, 8192)), dim3(256), 0,
                       st, src, nk, nc, ngw, dst);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int launch_unpack_pair_halves(const double2 *Mp, int nkv, int nc, int ng, double *M, hipStream_t st) {
    const long long n = (long long)nkv * nc * ng;
    hipLaunchKernelGGL(k_unpack_pair_halves, dim3((unsigned)std::min<long long>((n + 255) / 256, 8192)), dim3(256), 0,
                       st, Mp, nkv, nc, ng, M);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int launch_syrk_batch(const SyrkProb *probs, int nprob, long long nitems, int grid, hipStream_t st) {
    if (nitems <= 0) return BGW_OK;
    const long long g = std::max<long long>(1, std::min<long long>(nitems, grid));
    hipLaunchKernelGGL(k_syrk_f64, dim3((unsigned)g), dim3(RTHREADS), 0, st, probs, nprob, 0ll, nitems);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int syrk_blocks_per_cu() {
    static int n = 0;
    if (!n) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_syrk_f64, RTHREADS, 0) != hipSuccess || n < 1) n = 1;
    }
    return n;
}

int launch_syrk_finalize(const SyrkFin *probs, int nprob, int maxng, hipStream_t st) {
    const size_t total = (size_t)maxng * maxng;
    const int blocks = (int)std::max<size_t>(1, std::min<size_t>((total + 255) / 256, 16384 / std::max(1, nprob) + 1));
    hipLaunchKernelGGL(k_syrk_finalize, dim3(blocks, nprob), dim3(256), 0, st, probs);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

}  // namespace bgw
