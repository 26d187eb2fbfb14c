// The chi sum (epsilon section, static chi equation and its compact matrix
// form): chi(omega) = pf * M^H diag(w(omega)) M over the composite pair index
// t = (k*nv + v)*nc + c, on FP64 MFMA, for a whole batch of (q, omega)
// problems in one persistent launch.
//
// Complex arithmetic uses a real embedding along the contraction index: with
// M = A + iB and X = [A; B] interleaved per pair (k = 2t + part, which is the
// memory order of interleaved complex), Re chi = X_w^T X and
// Im chi = X_w^T Y with Y_{2t} = B_t, Y_{2t+1} = -A_t and X_w = diag(w) X.
// Only tiles on or above the diagonal are computed; the finalize kernel
// reduces the K-splits in a fixed order (bitwise reproducible), applies the
// prefactor and mirrors the lower triangle as the conjugate transpose.
#include <algorithm>

#include "common.h"

namespace bgw {

typedef double double4_t __attribute__((ext_vector_type(4)));

// Energy weights of one vector, Delta_t = (E_v,k+q - E_c,k) / Ha (see WeightKind):
//   imaginary axis:  w = Delta / (Delta^2 + omega^2)
//   real axis:       the real or the imaginary part of
//                    (1/2) [1/(Delta - E -+ i delta) + 1/(Delta + E +- i delta)],
//                    with a = Delta - E, b = Delta + E:
//                    Re = (a / (a^2 + delta^2) + b / (b^2 + delta^2)) / 2,
//                    Im = +-(delta / (a^2 + delta^2) - delta / (b^2 + delta^2)) / 2.
// grid.y: vector; every block strides over that vector's pairs.
__global__ void k_weights(const WProb *__restrict__ probs) {
    const WProb P = probs[blockIdx.y];
    const long long K = (long long)P.nk * P.nv * P.nc;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < K;
         t += (long long)gridDim.x * blockDim.x) {
        const long long c = t % P.nc, kv = t / P.nc;
        const long long k = kv / P.nv;
        const double d = (P.ev[kv] - P.ec[k * P.nc + c]) / kHartreeEv;
        double w;
        if (P.kind == kWeightGiven) {
            w = P.ev[t];
        } else if (P.kind == kWeightImag) {
            w = d / (d * d + P.omega_ha * P.omega_ha);
        } else {
            const double a = d - P.omega_ha, b = d + P.omega_ha, dl = P.delta_ha;
            const double da = a * a + dl * dl, db = b * b + dl * dl;
            if (P.kind == kWeightRealRe) {
                w = 0.5 * (a / da + b / db);
            } else {
                const double im = 0.5 * (dl / da - dl / db);
                w = P.kind == kWeightRetIm ? im : -im;
            }
        }
        P.w[t] = w;
    }
}

namespace {
constexpr int KC = 16;       // complex pairs per LDS stage
constexpr int KR = 2 * KC;   // real contraction rows per stage
constexpr int LDA = 64 + 16; // padded LDS row (doubles): the two half-waves of a 64-bit MFMA operand
                             // read hit disjoint bank halves

// One T x T tile of sum_t conj(P[t][G]) w_t Q[t][H] over t in [k0, k1) (w_t
// = 1 without weights): 4 waves in a 2 x 2 layout, each owning a (T/2) x
// (T/2) block of 16 x 16 MFMA tiles.  P has rows of ldp values of which the
// first m are used, Q rows of ldq with n used.  Raw sums (no prefactor) are
// stored to o, rows of ldo (tile rows >= m or columns >= n are dropped).
template <int T, bool W>
__device__ __forceinline__ void pq_tile(const double2 *__restrict__ P, long long ldp, int m,
                                        const double2 *__restrict__ Q, long long ldq, int n,
                                        const double *__restrict__ w, int G0, int H0, long long k0, long long k1,
                                        double2 *__restrict__ o, long long ldo, double (*As)[LDA],
                                        double (*Bs)[LDA]) {
    constexpr int NB = T / 32;    // MFMA tiles per wave side
    constexpr int WT = T / 2;     // wave block edge
    constexpr int LR = 256 / T;   // loader rows per sweep
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int li = lane & 15, lk = lane >> 4;

    double4_t cre[NB][NB], cim[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            cre[a][b] = (double4_t){0.0, 0.0, 0.0, 0.0};
            cim[a][b] = (double4_t){0.0, 0.0, 0.0, 0.0};
        }

    const int lcol = tid % T, lrow = tid / T;
    constexpr int SL = KC / LR;  // pairs each thread stages per stage
    // the imaginary-part operand is +-B of the other part of the same pair
    // (row kr ^ 1), negated on imaginary rows: a sign, not a branch
    const double isign = (lk & 1) ? -1.0 : 1.0;
    // The stage's values are loaded into registers one stage ahead: the loads
    // of stage kk + KC are issued before the MFMAs of stage kk.
    double2 a[SL], b[SL];
    double wt[SL];
    auto load_stage = [&](long long kk) {
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const long long t = kk + lrow + LR * s;
            const bool in = t < k1;
            wt[s] = in ? (W ? w[t] : 1.0) : 0.0;
            a[s] = (in && G0 + lcol < m) ? P[t * ldp + G0 + lcol] : make_double2(0.0, 0.0);
            b[s] = (in && H0 + lcol < n) ? Q[t * ldq + H0 + lcol] : make_double2(0.0, 0.0);
        }
    };
    load_stage(k0);
    for (long long kk = k0; kk < k1; kk += KC) {
        __syncthreads();  // the previous stage's reads are done
#pragma unroll
        for (int s = 0; s < SL; ++s) {
            const int r = lrow + LR * s;
            As[2 * r][lcol] = wt[s] * a[s].x;
            As[2 * r + 1][lcol] = wt[s] * a[s].y;
            Bs[2 * r][lcol] = b[s].x;
            Bs[2 * r + 1][lcol] = b[s].y;
        }
        __syncthreads();
        if (kk + KC < k1) load_stage(kk + KC);
#pragma unroll
        for (int s = 0; s < KR / 4; ++s) {
            const int kr = 4 * s + lk;
            double av[NB], bre[NB], bim[NB];
#pragma unroll
            for (int a = 0; a < NB; ++a) av[a] = As[kr][wr * WT + 16 * a + li];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int col = wc * WT + 16 * b + li;
                bre[b] = Bs[kr][col];
                bim[b] = isign * Bs[kr ^ 1][col];
            }
#pragma unroll
            for (int a = 0; a < NB; ++a)
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    cre[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bre[b], cre[a][b], 0, 0, 0);
                    cim[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bim[b], cim[a][b], 0, 0, 0);
                }
        }
    }
    __syncthreads();  // the LDS tiles are reused by the block's next item
    // D layout of v_mfma_f64_16x16x4: lane l, register r -> row 4r + l/16, col l%16
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int G = G0 + wr * WT + 16 * a + 4 * r + lk;
                const int H = H0 + wc * WT + 16 * b + li;
                if (G < m && H < n) o[(size_t)G * ldo + H] = make_double2(cre[a][b][r], cim[a][b][r]);
            }
}

// The chi-sum tile: P = Q = M, rows of ng, weights w.
template <int T>
__device__ __forceinline__ void herk_tile(const double2 *__restrict__ M, int ng, const double *__restrict__ w,
                                          int G0, int H0, long long k0, long long k1, double2 *__restrict__ o,
                                          double (*As)[LDA], double (*Bs)[LDA]) {
    pq_tile<T, true>(M, ng, ng, M, ng, ng, w, G0, H0, k0, k1, o, ng, As, Bs);
}
}  // namespace

// Persistent batched rank-K update for one output-tile size T.  Problem p
// owns the items p.item0 .. p.item0 + p.nitems (a multiple of 8).  Blocks
// stride over the items of the whole batch with a grid that is a multiple of
// 8, so item i always runs on XCD i % 8 (workgroups are dealt to the XCDs
// round-robin).  Within a problem, XCD x takes the x-th contiguous eighth of
// the (K split, tile) sequence, split-major with tiles in grouped order:
// the blocks resident on one XCD then stream the same K range of nearby row
// and column blocks of M through its L2.  Uneven problems (many q with
// different ng, many omega) share one launch per tile size.
template <int T>
__global__ __launch_bounds__(256, 3) void k_herk_f64(const HerkProb *__restrict__ probs, int nprob, long long i0,
                                                  long long i1) {
    __shared__ double As[KR][LDA];
    __shared__ double Bs[KR][LDA];
    for (long long item = i0 + blockIdx.x; item < i1; item += gridDim.x) {
        int lo = 0, hi = nprob - 1;  // last problem with item0 <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (probs[mid].item0 <= item) lo = mid;
            else hi = mid - 1;
        }
        const HerkProb &P = probs[lo];
        const long long local = item - P.item0;
        const long long chunk = P.nitems / 8;  // items per XCD
        const long long u = (local % 8) * chunk + local / 8;
        const long long ntile = (long long)P.nt * (P.nt + 1) / 2;
        if (u >= ntile * P.ns) continue;  // padding item
        const int split = (int)(u / ntile);
        int ti, tj;
        grouped_tile((int)(u % ntile), P.nt, ti, tj);
        const long long k0 = split * P.kper;
        const long long k1 = min(P.K, k0 + P.kper);
        herk_tile<T>(P.M, P.ng, P.w, ti * T, tj * T, k0, k1, P.out + (size_t)split * P.ng * P.ng, As, Bs);
    }
}

// chi[G][H] (+)= pf * (A_GH + i B_GH), where A (and B, when part_im is set)
// are Hermitian with raw upper-triangle sums part[s][G][H], G <= H, reduced
// over the K splits s in fixed order; below the diagonal A_GH = conj(A_HG).
// Without B (imaginary axis) chi is Hermitian and its diagonal exactly real.
// In place (ns == 1, no B): chi's upper triangle holds the raw sums and each
// thread reads (G, H), G <= H, and writes (G, H) and (H, G).  Row and column
// `skip` (>= 0) are left untouched (written by the FP64 head kernel).
// grid.y: output matrix.
__global__ void k_chi_finalize(const FinProb *__restrict__ probs) {
    const FinProb P = probs[blockIdx.y];
    const int ng = P.ng;
    const size_t total = (size_t)ng * ng;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int G = (int)(e / ng), H = (int)(e % ng);
        if (G == P.skip || H == P.skip) continue;
        if (P.inplace) {
            if (G > H) continue;
            const double2 s = P.chi[e];
            double2 val = make_double2(P.pf * s.x, P.pf * s.y);
            if (G == H) {
                val.y = 0.0;
                P.chi[e] = val;
            } else {
                P.chi[e] = val;
                P.chi[(size_t)H * ng + G] = make_double2(val.x, -val.y);
            }
            continue;
        }
        const bool up = G <= H;
        const size_t src = up ? e : (size_t)H * ng + G;
        double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
#pragma unroll 8
        for (int p = 0; p < P.ns; ++p) a = cadd(a, P.part[p * total + src]);
        if (P.part_im) {
#pragma unroll 8
            for (int p = 0; p < P.ns; ++p) b = cadd(b, P.part_im[p * total + src]);
        }
        if (!up) {
            a.y = -a.y;
            b.y = -b.y;
        }
        if (G == H) {
            a.y = 0.0;
            b.y = 0.0;
        }
        double2 val = make_double2(P.pf * (a.x - b.y), P.pf * (a.y + b.x));
        if (P.accumulate) val = cadd(P.chi[e], val);
        P.chi[e] = val;
    }
}

// C = P^H Q (rows t of P and Q contracted) for one problem, all T x T tiles of
// the m x n result, the contraction cut into ns ranges: raw sums of range s
// to out + s m n.  A persistent grid strides over the (range, tile) items.
template <int T>
__global__ __launch_bounds__(256, 3) void k_gemm_phq(const GemmProb G) {
    __shared__ double As[KR][LDA];
    __shared__ double Bs[KR][LDA];
    const long long ntile = (long long)G.ntr * G.ntc;
    for (long long item = blockIdx.x; item < ntile * G.ns; item += gridDim.x) {
        const long long split = item / ntile, tile = item % ntile;
        const int tr = (int)(tile / G.ntc), tc = (int)(tile % G.ntc);
        const long long k0 = split * G.kper, k1 = min(G.K, k0 + G.kper);
        pq_tile<T, false>(G.P, G.ldp, G.m, G.Q, G.ldq, G.n, nullptr, tr * T, tc * T, k0, k1,
                          G.out + (size_t)split * G.m * G.n, G.n, As, Bs);
    }
}

// C (+)= scale * sum over s < ns of part[s] (m x n, complex).
__global__ void k_gemm_finalize(const double2 *__restrict__ part, int ns, long long mn, double scale,
                                double2 *__restrict__ C, int accumulate) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < mn; e += (long long)gridDim.x * blockDim.x) {
        double2 a = make_double2(0.0, 0.0);
        for (int p = 0; p < ns; ++p) a = cadd(a, part[p * mn + e]);
        a = make_double2(scale * a.x, scale * a.y);
        C[e] = accumulate ? cadd(C[e], a) : a;
    }
}

// MT[G][t] = M[t][G] for the K x ng matrix M (pairs x G), row `head` of MT
// zeroed (head < 0: none): the contraction over G of the Bethe-Salpeter
// exchange kernel becomes the contraction over the leading index that the
// chi-sum kernels perform.  grid.z batches: matrix z starts at M + z K ng and
// MT + z ng K.  32 x 32 tiles through LDS, both sides coalesced; grid
// (ceil(ng / 32), ceil(K / 32), batches), block (32, 8).
__global__ __launch_bounds__(256) void k_transpose_pairs(const double2 *__restrict__ M, long long K, int ng,
                                                         int head, double2 *__restrict__ MT) {
    __shared__ double2 tile[32][33];
    M += (size_t)blockIdx.z * K * ng;
    MT += (size_t)blockIdx.z * K * ng;
    const int g0 = blockIdx.x * 32;
    const long long t0 = (long long)blockIdx.y * 32;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const long long t = t0 + threadIdx.y + 8 * r;
        const int g = g0 + threadIdx.x;
        tile[threadIdx.y + 8 * r][threadIdx.x] = (t < K && g < ng) ? M[t * ng + g] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int g = g0 + threadIdx.y + 8 * r;
        const long long t = t0 + threadIdx.x;
        if (g < ng && t < K)
            MT[(size_t)g * K + t] = g == head ? make_double2(0.0, 0.0) : tile[threadIdx.x][threadIdx.y + 8 * r];
    }
}

// Self-energy operands.  w[i ng + G] = v[G] for i < ninner (the bare
// exchange's weights along the contraction index (i, G)).
__global__ void k_sigma_weights(const double *__restrict__ v, int ng, int ninner, double *__restrict__ w) {
    const long long n = (long long)ng * ninner;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        w[e] = v[e % ng];
}

// WT[k][g] = conj(W[g][k]) with W[g][k] = (einv[g][k] - ch delta_gk) v[k]: the
// screened interaction (ch = 0) or its screening part (ch = 1), transposed
// and conjugated so that sum_k conj(WT[k][g]) A[k] = (W A)[g].  32 x 32 tiles
// through LDS; grid (ceil(ng / 32), ceil(ng / 32)), block (32, 8).
__global__ __launch_bounds__(256) void k_sigma_wt(const double2 *__restrict__ einv, const double *__restrict__ v,
                                                  int ng, int ch, double2 *__restrict__ WT) {
    __shared__ double2 tile[32][33];
    const int k0 = blockIdx.x * 32, g0 = blockIdx.y * 32;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int g = g0 + threadIdx.y + 8 * r, k = k0 + threadIdx.x;
        double2 e = make_double2(0.0, 0.0);
        if (g < ng && k < ng) {
            e = einv[(size_t)g * ng + k];
            if (ch && g == k) e.x -= 1.0;
            e = make_double2(e.x * v[k], -e.y * v[k]);
        }
        tile[threadIdx.y + 8 * r][threadIdx.x] = e;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int k = k0 + threadIdx.y + 8 * r, g = g0 + threadIdx.x;
        if (k < ng && g < ng) WT[(size_t)k * ng + g] = tile[threadIdx.x][threadIdx.y + 8 * r];
    }
}

// B2[i ng + G][n] = B[G][i nouter + n]: the rows of W M regrouped by inner
// state, so that the last contraction runs over (i, G).
__global__ void k_sigma_regroup(const double2 *__restrict__ B, int ng, int ninner, int nouter,
                                double2 *__restrict__ B2) {
    const long long total = (long long)ng * ninner * nouter;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int n = (int)(e % nouter);
        const long long r = e / nouter;
        const int G = (int)(r % ng), i = (int)(r / ng);
        B2[e] = B[((size_t)G * ninner + i) * nouter + n];
    }
}

// ---------------------------------------------------------------- launchers

int launch_transpose_pairs(const double2 *M, long long K, int ng, int head, double2 *MT, hipStream_t st,
                           int batches) {
    hipLaunchKernelGGL(k_transpose_pairs, dim3((ng + 31) / 32, (unsigned)((K + 31) / 32), batches), dim3(32, 8), 0,
                       st, M, K, ng, head, MT);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int launch_weights_batch(const WProb *probs, int nprob, long long maxK, hipStream_t st) {
    const int blocks = (int)std::max<long long>(1, std::min<long long>((maxK + 255) / 256, 1024));
    hipLaunchKernelGGL(k_weights, dim3(blocks, nprob), dim3(256), 0, st, probs);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int herk_blocks_per_cu() {
    static int n = 0;
    if (!n) {
        int a = 0, b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k_herk_f64<64>, 256, 0) != hipSuccess || a < 1) a = 1;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_herk_f64<32>, 256, 0) != hipSuccess || b < 1) b = 1;
        n = std::min(a, b);
    }
    return n;
}

// Items [i0, i1) all have output tile `tile`.
int launch_herk_batch(const HerkProb *probs, int nprob, long long i0, long long i1, int tile, int grid,
                      hipStream_t st) {
    if (i1 <= i0) return BGW_OK;
    const long long g = std::max<long long>(1, std::min<long long>(i1 - i0, grid));
    if (tile == 64) hipLaunchKernelGGL(k_herk_f64<64>, dim3((unsigned)g), dim3(256), 0, st, probs, nprob, i0, i1);
    else hipLaunchKernelGGL(k_herk_f64<32>, dim3((unsigned)g), dim3(256), 0, st, probs, nprob, i0, i1);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int device_cus();

int launch_gemm_phq(const GemmProb &G, int tile, hipStream_t st) {
    const long long items = (long long)G.ntr * G.ntc * G.ns;
    const long long g = std::max<long long>(1, std::min<long long>(items, (long long)device_cus() * 3));
    if (tile == 64) hipLaunchKernelGGL(k_gemm_phq<64>, dim3((unsigned)g), dim3(256), 0, st, G);
    else hipLaunchKernelGGL(k_gemm_phq<32>, dim3((unsigned)g), dim3(256), 0, st, G);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int launch_gemm_finalize(const double2 *part, int ns, long long mn, double scale, double2 *C, int accumulate,
                         hipStream_t st) {
    const int blocks = (int)std::max<long long>(1, std::min<long long>((mn + 255) / 256, 8192));
    hipLaunchKernelGGL(k_gemm_finalize, dim3(blocks), dim3(256), 0, st, part, ns, mn, scale, C, accumulate);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int launch_sigma_weights(const double *v, int ng, int ninner, double *w, hipStream_t st) {
    const long long n = (long long)ng * ninner;
    hipLaunchKernelGGL(k_sigma_weights, dim3((unsigned)std::min<long long>((n + 255) / 256, 4096)), dim3(256), 0, st,
                       v, ng, ninner, w);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int launch_sigma_wt(const double2 *einv, const double *v, int ng, int ch, double2 *WT, hipStream_t st) {
    hipLaunchKernelGGL(k_sigma_wt, dim3((ng + 31) / 32, (ng + 31) / 32), dim3(32, 8), 0, st, einv, v, ng, ch, WT);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int launch_sigma_regroup(const double2 *B, int ng, int ninner, int nouter, double2 *B2, hipStream_t st) {
    const long long n = (long long)ng * ninner * nouter;
    hipLaunchKernelGGL(k_sigma_regroup, dim3((unsigned)std::min<long long>((n + 255) / 256, 8192)), dim3(256), 0, st,
                       B, ng, ninner, nouter, B2);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int launch_finalize_batch(const FinProb *probs, int nprob, int maxng, hipStream_t st) {
    const size_t total = (size_t)maxng * maxng;
    const int blocks = (int)std::max<size_t>(1, std::min<size_t>((total + 255) / 256, 16384 / std::max(1, nprob) + 1));
    hipLaunchKernelGGL(k_chi_finalize, dim3(blocks, nprob), dim3(256), 0, st, probs);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

}  // namespace bgw
