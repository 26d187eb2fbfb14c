// The chi sum (epsilon section, static chi equation and its compact matrix
// form): chi(omega) = pf * M^H diag(w(omega)) M over the composite pair index
// t = (k*nv + v)*nc + c, on FP64 MFMA.
//
// Complex arithmetic uses a real embedding along the contraction index: with
// M = A + iB and X = [A; B] interleaved per pair (k = 2t + part, which is the
// memory order of interleaved complex), Re chi = X_w^T X and
// Im chi = X_w^T Y with Y_{2t} = B_t, Y_{2t+1} = -A_t and X_w = diag(w) X.
// Only tiles on or above the diagonal are computed; the finalize kernel
// reduces the K-splits in a fixed order (bitwise reproducible), applies the
// prefactor and mirrors the lower triangle as the conjugate transpose.
#include "common.h"

namespace bgw {

typedef double double4_t __attribute__((ext_vector_type(4)));

// w[t] = Delta_t / (Delta_t^2 + omega^2), Delta_t = (E_v,k+q - E_c,k) / Ha  (omega in Ha)
__global__ void k_weights(const double *__restrict__ ev, const double *__restrict__ ec, int nk, int nv, int nc,
                          double omega_ha, double *__restrict__ w) {
    const long long K = (long long)nk * nv * nc;
    for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < K;
         t += (long long)gridDim.x * blockDim.x) {
        const long long c = t % nc, kv = t / nc;
        const long long k = kv / nv;
        const double d = (ev[kv] - ec[k * nc + c]) / kHartreeEv;
        w[t] = d / (d * d + omega_ha * omega_ha);
    }
}

namespace {
constexpr int TM = 64;       // tile rows (G)
constexpr int TN = 64;       // tile cols (G')
constexpr int KC = 16;       // complex pairs per LDS stage
constexpr int KR = 2 * KC;   // real contraction rows per stage
constexpr int LDA = TM + 16; // padded LDS row: 640 B = 128 B mod 256 B, so the two half-waves of a
                             // 64-bit MFMA operand read hit disjoint bank halves
}  // namespace

// grid.x: upper-triangle tiles (ti <= tj) of an nt x nt tile grid, grid.y: K splits.
// out: [split][ng][ng] partial sums (no prefactor).
__global__ __launch_bounds__(256) void k_herk_f64(const double2 *__restrict__ M, long long K, int ng, int nt,
                                                  const double *__restrict__ w, long long kper,
                                                  double2 *__restrict__ out) {
    __shared__ double As[KR][LDA];
    __shared__ double Bs[KR][LDA];

    int u = blockIdx.x, ti = 0;
    while (u >= nt - ti) {
        u -= nt - ti;
        ++ti;
    }
    const int tj = ti + u;
    const int G0 = ti * TM, H0 = tj * TN;
    const long long k0 = blockIdx.y * kper;
    const long long k1 = min(K, k0 + kper);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int li = lane & 15, lk = lane >> 4;

    double4_t cre[2][2], cim[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            cre[a][b] = (double4_t){0.0, 0.0, 0.0, 0.0};
            cim[a][b] = (double4_t){0.0, 0.0, 0.0, 0.0};
        }

    const int lcol = tid & 63, lrow = tid >> 6;  // loader: 4 rows x 64 cols per sweep
    for (long long kk = k0; kk < k1; kk += KC) {
#pragma unroll
        for (int s = 0; s < KC / 4; ++s) {
            const int r = lrow + 4 * s;
            const long long t = kk + r;
            double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
            double wt = 0.0;
            if (t < k1) {
                wt = w[t];
                if (G0 + lcol < ng) a = M[t * ng + G0 + lcol];
                if (H0 + lcol < ng) b = M[t * ng + H0 + lcol];
            }
            As[2 * r][lcol] = wt * a.x;
            As[2 * r + 1][lcol] = wt * a.y;
            Bs[2 * r][lcol] = b.x;
            Bs[2 * r + 1][lcol] = b.y;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < KR / 4; ++s) {
            const int kr = 4 * s + lk;
            double av[2], bre[2], bim[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = As[kr][wr * 32 + 16 * a + li];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int col = wc * 32 + 16 * b + li;
                bre[b] = Bs[kr][col];
                bim[b] = (kr & 1) ? -Bs[kr - 1][col] : Bs[kr + 1][col];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    cre[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bre[b], cre[a][b], 0, 0, 0);
                    cim[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bim[b], cim[a][b], 0, 0, 0);
                }
        }
        __syncthreads();
    }
    // D layout of v_mfma_f64_16x16x4: lane l, register r -> row 4r + l/16, col l%16
    double2 *o = out + (size_t)blockIdx.y * ng * ng;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int G = G0 + wr * 32 + 16 * a + 4 * r + lk;
                const int H = H0 + wc * 32 + 16 * b + li;
                if (G < ng && H < ng) o[(size_t)G * ng + H] = make_double2(cre[a][b][r], cim[a][b][r]);
            }
}

// chi[G][H] (+)= pf * sum_s part[s][G][H] for G <= H, conjugate mirror below the
// diagonal, diagonal made exactly real.  The split sum runs in fixed order.
// Row and column `skip` (>= 0) are left untouched (written by the FP64 head kernel).
__global__ void k_chi_finalize(const double2 *__restrict__ part, int nsplit, int ng, double pf,
                               double2 *__restrict__ chi, int accumulate, int skip) {
    const size_t total = (size_t)ng * ng;
    const size_t pstride = total;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int G = (int)(e / ng), H = (int)(e % ng);
        if (G == skip || H == skip) continue;
        const bool up = G <= H;
        const size_t src = up ? e : (size_t)H * ng + G;
        double2 s = make_double2(0.0, 0.0);
        for (int p = 0; p < nsplit; ++p) s = cadd(s, part[p * pstride + src]);
        double2 val = make_double2(pf * s.x, up ? pf * s.y : -pf * s.y);
        if (G == H) val.y = 0.0;
        if (accumulate) val = cadd(chi[e], val);
        chi[e] = val;
    }
}

// ---------------------------------------------------------------- launchers

int launch_weights(const double *ev, const double *ec, int nk, int nv, int nc, double omega_ev, double *w,
                   hipStream_t st) {
    const long long K = (long long)nk * nv * nc;
    const int blocks = (int)std::min<long long>((K + 255) / 256, 4096);
    hipLaunchKernelGGL(k_weights, dim3(blocks), dim3(256), 0, st, ev, ec, nk, nv, nc, omega_ev / kHartreeEv, w);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int herk_f64_splits(long long K, int ng) {
    const int nt = (ng + TM - 1) / TM;
    const long long tiles = (long long)nt * (nt + 1) / 2;
    long long want = (2048 + tiles - 1) / tiles;
    const long long maxs = std::max<long long>(1, K / (8 * KC));
    want = std::min(want, maxs);
    return (int)std::max<long long>(1, std::min<long long>(want, 64));
}

int launch_herk_f64(const double2 *M, long long K, int ng, const double *w, int nsplit, double2 *part,
                    hipStream_t st) {
    const int nt = (ng + TM - 1) / TM;
    const long long tiles = (long long)nt * (nt + 1) / 2;
    long long kper = (K + nsplit - 1) / nsplit;
    kper = (kper + KC - 1) / KC * KC;
    hipLaunchKernelGGL(k_herk_f64, dim3((unsigned)tiles, nsplit), dim3(256), 0, st, M, K, ng, nt, w, kper, part);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int launch_chi_finalize_skip(const double2 *part, int nsplit, int ng, double pf, double2 *chi, int accumulate,
                             int skip, hipStream_t st) {
    const size_t total = (size_t)ng * ng;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_chi_finalize, dim3(blocks), dim3(256), 0, st, part, nsplit, ng, pf, chi, accumulate, skip);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int launch_chi_finalize(const double2 *part, int nsplit, int ng, double pf, double2 *chi, int accumulate,
                        hipStream_t st) {
    return launch_chi_finalize_skip(part, nsplit, ng, pf, chi, accumulate, -1, st);
}

}  // namespace bgw
