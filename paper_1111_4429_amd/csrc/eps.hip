// Dielectric matrix epsilon = 1 - v chi (epsilon section, dielectric-matrix
// equation, asymmetric Coulomb form) and its inverse.
//
// The paper inverts with LU + solve (ZGESV).  Here the inverse is formed by
// blocked Gauss-Jordan elimination with partial pivoting, in place: it uses
// the same pivot sequence as LU with partial pivoting (largest |Re|+|Im| in
// the current column among the rows not yet pivoted, first index on ties),
// costs the same 8 n^3 real flops as getrf+getri, and puts nearly all of
// them into rank-nbo updates (FP64 MFMA GEMMs).
//
// Columns are taken in outer blocks of nbo (64 or 128) columns, each
// factored as panels of nb (16 or 32) columns [ks, ks+nb):
//   k_gje_panel*     the panel's column steps (pivot search, interchange,
//                    elimination of every row: Gauss-Jordan) on its nb
//                    columns; the panel ends up holding its elimination
//                    transform.  One workgroup per matrix, or cooperative:
//                    R workgroups each holding a block of rows, one grid
//                    barrier per column.
//   k_gje_swap_save  applies the panel's row interchanges to the other
//                    columns of the outer block, saves their panel rows and
//                    zeroes them;
//   k_gje_update     A[:, those columns] += P * Rsaved  (complex, FP64 MFMA).
// When the outer block is done its columns hold the transform of all its nbo
// steps (the same numbers an nbo-wide panel would give), and the columns
// outside it take all its interchanges and one rank-nbo update: the matrix
// streams through HBM once per nbo columns instead of once per panel.
// At the end the row interchanges are undone as column interchanges in
// reverse order (k_gje_colperm).
//
// Barrier waits are bounded: a wait that exceeds its spin budget stores
// info = -1000 for that matrix and gives up, so the kernel always terminates.
#include <cfloat>
#include <cstdlib>
#include <cstring>
#include <utility>

#include "common.h"

namespace bgw {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kPanelMax = 32;
constexpr int kGjeMaxR = 48;                // workgroups per matrix (n <= 12288, 256 rows each; the narrow
                                            // panel's LDS, 256 x 33 + 64 + 48 x 32 complex, fits 160 KB)
constexpr int kInfoBarrierTimeout = -1000;  // info value when a grid barrier wait gave up

struct GjeScratch {
    double *cand_val;         // [nmat][2][R]
    int *cand_row;            // [nmat][2][R]
    double2 *cand_rows;       // [nmat][2][R][nb]
    double2 *rowbuf;          // [nmat][2][nb]
    unsigned int *bar;        // [nmat] barrier counters (zeroed before the first panel)
};

__global__ void k_eps_build(const double2 *__restrict__ chi, const double *__restrict__ v, int ng, int nw,
                            double2 *__restrict__ eps) {
    const size_t per = (size_t)ng * ng;
    const size_t total = per * nw;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const size_t r = e % per;
        const int G = (int)(r / ng), H = (int)(r % ng);
        const double2 x = chi[e];
        eps[e] = make_double2((G == H ? 1.0 : 0.0) - v[G] * x.x, -v[G] * x.y);
    }
}

__global__ void k_fill_u32(unsigned int *p, size_t n, unsigned int val) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = val;
}

__device__ inline double cabs1(double2 a) { return fabs(a.x) + fabs(a.y); }

// x - f p, complex, as four FMAs
__device__ __forceinline__ double2 cfms(double2 x, double2 f, double2 p) {
    return make_double2(fma(-f.x, p.x, fma(f.y, p.y, x.x)), fma(-f.x, p.y, fma(-f.y, p.x, x.y)));
}

__device__ inline double2 cdiv(double2 a, double2 b) {
    // a / b with scaling (Smith's method)
    if (fabs(b.x) >= fabs(b.y)) {
        const double r = b.y / b.x, d = b.x + b.y * r;
        return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
    }
    const double r = b.x / b.y, d = b.x * r + b.y;
    return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}

// grid barrier among the R workgroups of one matrix; `target` = R * (number of
// barriers passed including this one).  One release (the arrival) and one
// acquire fence after the wait: the spin itself uses relaxed loads, since an
// acquire load per iteration would invalidate the XCD's L2 every time.
__device__ inline void matrix_barrier(unsigned int *bar, unsigned int target, int *info) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1ull << 24)) {  // bounded wait: report and give up
                atomicExch(info, kInfoBarrierTimeout);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    // the exchanged values are then read with device-scope atomic loads
    __syncthreads();
}

__device__ inline double2 ld_agent(const double2 *p) {
    const double *d = reinterpret_cast<const double *>(p);
    return make_double2(__hip_atomic_load(d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                        __hip_atomic_load(d + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

__device__ inline void st_agent(double2 *p, double2 v) {
    double *d = reinterpret_cast<double *>(p);
    __hip_atomic_store(d, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(d + 1, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Largest |Re|+|Im| over a wavefront, first row on ties; every lane gets the result.
__device__ inline void wave_argmax(double &v, int &row) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off);
        const int orow = __shfl_xor(row, off);
        if (ov > v || (ov == v && orow < row)) {
            v = ov;
            row = orow;
        }
    }
}

// A: matrices of a group, [nmat][n][n]; each matrix is factored by R
// consecutive workgroups, workgroup r owning rows [r*rows, min(n, (r+1)*rows))
// (rows <= blockDim.x: one row per thread).  NB: panel width known at compile
// time (0: the runtime nb, for the last, narrower panel).
template <int NB>
__global__ __launch_bounds__(256) void k_gje_panel(double2 *__restrict__ A, int n, int k, int nb_rt, int rows, int R,
                                                   int *__restrict__ ipiv, int *__restrict__ info, GjeScratch sc,
                                                   unsigned int bar_done) {
    extern __shared__ double2 lds[];
    const int nb = NB ? NB : nb_rt;
    const int ps = nb + 1;                       // padded row stride of the panel in LDS
    double2 *P = lds;                            // [rows][ps]
    double2 *prow = P + rows * (kPanelMax + 1);  // scaled pivot row [nb]
    double2 *oldrow = prow + kPanelMax;          // row k+j before the swap [nb]
    double2 *cand = oldrow + kPanelMax;          // candidate rows of all workgroups [R][nb]
    __shared__ double wv[4], cv_s[kGjeMaxR];
    __shared__ int wrow[4], cr_s[kGjeMaxR];

    const int mat = blockIdx.x / R, r = blockIdx.x % R;
    double2 *Am = A + (size_t)mat * n * n;
    int *ip = ipiv + (size_t)mat * n;
    const int row0 = r * rows;
    const int nloc = max(0, min(rows, n - row0));
    double *cval = sc.cand_val + (size_t)mat * 2 * R;
    int *crow = sc.cand_row + (size_t)mat * 2 * R;
    double2 *crows = sc.cand_rows + (size_t)mat * 2 * R * nb;
    double2 *rbuf = sc.rowbuf + (size_t)mat * 2 * nb;
    unsigned int *bar = sc.bar + mat;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int gi = row0 + tid;  // this thread's row
    const bool mine = tid < nloc;
    double2 *pr = P + tid * ps;

    for (int e = tid; e < nloc * nb; e += blockDim.x) {
        const int i = e / nb, c = e % nb;
        P[i * ps + c] = Am[(size_t)(row0 + i) * n + k + c];
    }
    __syncthreads();

    for (int j = 0; j < nb; ++j) {
        const int col = k + j;
        const int slot = j & 1;
        // local pivot candidate among rows >= col
        double best = -1.0;
        int brow = 0x7fffffff;
        if (mine && gi >= col) {
            const double v = cabs1(pr[j]);
            if (v >= 0.0) {  // a NaN entry is never a pivot candidate
                best = v;
                brow = gi;
            }
        }
        wave_argmax(best, brow);
        if (lane == 0) {
            wv[wave] = best;
            wrow[wave] = brow;
        }
        __syncthreads();
        best = wv[0];
        brow = wrow[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            if (wv[w] > best || (wv[w] == best && wrow[w] < brow)) {
                best = wv[w];
                brow = wrow[w];
            }
        // publish the candidate (value, row, row contents) and, from the owner, row col
        if (tid == 0) {
            __hip_atomic_store(&cval[slot * R + r], best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&crow[slot * R + r], brow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (tid < nb)
            st_agent(&crows[((size_t)slot * R + r) * nb + tid],
                     best >= 0.0 ? P[(brow - row0) * ps + tid] : make_double2(0.0, 0.0));
        if (col >= row0 && col < row0 + nloc && tid < nb) st_agent(&rbuf[slot * nb + tid], P[(col - row0) * ps + tid]);

        matrix_barrier(bar, (bar_done + j + 1) * (unsigned)R, info + mat);

        // every workgroup fetches all candidates (values, rows, row contents) and row col in one round
        for (int e = tid; e < R * nb; e += blockDim.x) cand[e] = ld_agent(&crows[(size_t)slot * R * nb + e]);
        if (tid < R) {
            cv_s[tid] = __hip_atomic_load(&cval[slot * R + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            cr_s[tid] = __hip_atomic_load(&crow[slot * R + tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (tid >= 64 && tid < 64 + nb) oldrow[tid - 64] = ld_agent(&rbuf[slot * nb + tid - 64]);
        __syncthreads();
        // global pivot (every thread, same order): largest |Re|+|Im|, first row on ties
        double bv = cv_s[0];
        int p = cr_s[0], win = 0;
        for (int q = 1; q < R; ++q)
            if (cv_s[q] > bv || (cv_s[q] == bv && cr_s[q] < p)) {
                bv = cv_s[q];
                p = cr_s[q];
                win = q;
            }
        if (p >= n) p = col;  // no candidate (a column of NaNs): no interchange; info flags the matrix
        if (tid == 0 && r == 0) {
            if (!(bv > 0.0)) atomicCAS(info + mat, 0, col + 1);
            ip[col] = p;
        }
        const double2 *praw = cand + win * nb;
        if (tid < nb) {
            double2 piv = praw[j];
            if (piv.x == 0.0 && piv.y == 0.0) piv = make_double2(1.0, 0.0);
            const double2 ipv = cdiv(make_double2(1.0, 0.0), piv);
            prow[tid] = tid == j ? ipv : cmul(praw[tid], ipv);
            // row interchange col <-> p inside the panel
            if (p != col && p >= row0 && p < row0 + nloc) P[(p - row0) * ps + tid] = oldrow[tid];
        }
        __syncthreads();
        // eliminate: every row except col; row col becomes the scaled pivot row
        if (mine) {
            if (gi == col) {
#pragma unroll
                for (int c = 0; c < (NB ? NB : kPanelMax); ++c)
                    if (NB || c < nb) pr[c] = prow[c];
            } else {
                const double2 f = pr[j];
                const double2 pj = prow[j];
#pragma unroll
                for (int c = 0; c < (NB ? NB : kPanelMax); ++c)
                    if (NB || c < nb) {
                        const double2 pc = prow[c];
                        const double2 x = pr[c];
                        pr[c] = (c == j) ? make_double2(-(f.x * pj.x - f.y * pj.y), -(f.x * pj.y + f.y * pj.x))
                                         : cfms(x, f, pc);
                    }
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < nloc * nb; e += blockDim.x) {
        const int i = e / nb, c = e % nb;
        Am[(size_t)(row0 + i) * n + k + c] = P[i * ps + c];
    }
}

// Full-width panels (kPanelMax columns): the same column steps as
// k_gje_panel, with each thread's panel row held in registers.  The column
// steps are instantiated per column index, so every row element has a fixed
// register.  Every thread scales by the inverse pivot on the fly:
// row i -= (f / p) * (pivot row) and row col = (pivot row) / p, so the only
// shared data per column are the candidates fetched after the grid barrier.
struct GjeRegCtx {
    double2 *Am;
    int *ip, *info, *crow;
    double *cval;
    double2 *crows, *rbuf, *oldrow, *cand;
    unsigned int *bar;
    double *wv, *cv_s;
    int *wrow, *cr_s;
    int k, R, r, row0, nloc, gi, lane, wave, tid, mat;
    bool mine;
    unsigned int bar_done;
};

template <int J>
__device__ __forceinline__ void gje_reg_column(const GjeRegCtx &x, double2 (&rv)[kPanelMax]) {
    constexpr int nb = kPanelMax;
    const int col = x.k + J;
    constexpr int slot = J & 1;
    const int R = x.R;
    // local pivot candidate among rows >= col
    double best = -1.0;
    int brow = 0x7fffffff;
    if (x.mine && x.gi >= col) {
        const double v = cabs1(rv[J]);
        if (v >= 0.0) {  // a NaN entry is never a pivot candidate
            best = v;
            brow = x.gi;
        }
    }
    wave_argmax(best, brow);
    if (x.lane == 0) {
        x.wv[x.wave] = best;
        x.wrow[x.wave] = brow;
    }
    __syncthreads();
    best = x.wv[0];
    brow = x.wrow[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
        if (x.wv[w] > best || (x.wv[w] == best && x.wrow[w] < brow)) {
            best = x.wv[w];
            brow = x.wrow[w];
        }
    // publish the candidate (value, row, row contents) and, from its owner, row col
    if (x.tid == 0) {
        __hip_atomic_store(&x.cval[slot * R + x.r], best, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&x.crow[slot * R + x.r], brow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (x.mine && x.gi == brow) {
#pragma unroll
        for (int c = 0; c < nb; ++c) st_agent(&x.crows[((size_t)slot * R + x.r) * nb + c], rv[c]);
    }
    if (x.mine && x.gi == col) {
#pragma unroll
        for (int c = 0; c < nb; ++c) st_agent(&x.rbuf[slot * nb + c], rv[c]);
    }

    matrix_barrier(x.bar, (x.bar_done + J + 1) * (unsigned)R, x.info + x.mat);

    // every workgroup fetches all candidates and row col in one round
    for (int e = x.tid; e < R * nb; e += blockDim.x) x.cand[e] = ld_agent(&x.crows[(size_t)slot * R * nb + e]);
    if (x.tid < R) {
        x.cv_s[x.tid] = __hip_atomic_load(&x.cval[slot * R + x.tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x.cr_s[x.tid] = __hip_atomic_load(&x.crow[slot * R + x.tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (x.tid >= 64 && x.tid < 64 + nb) x.oldrow[x.tid - 64] = ld_agent(&x.rbuf[slot * nb + x.tid - 64]);
    __syncthreads();
    // global pivot (every thread, same order): largest |Re|+|Im|, first row on ties
    double bv = x.cv_s[0];
    int p = x.cr_s[0], win = 0;
    for (int q = 1; q < R; ++q)
        if (x.cv_s[q] > bv || (x.cv_s[q] == bv && x.cr_s[q] < p)) {
            bv = x.cv_s[q];
            p = x.cr_s[q];
            win = q;
        }
    if (p == 0x7fffffff) p = col;  // no candidate (a column of NaNs): no interchange; info flags the matrix
    if (x.tid == 0 && x.r == 0) {
        if (!(bv > 0.0)) atomicCAS(x.info + x.mat, 0, col + 1);
        x.ip[col] = p;
    }
    const double2 *praw = x.cand + win * nb;
    double2 piv = praw[J];
    if (piv.x == 0.0 && piv.y == 0.0) piv = make_double2(1.0, 0.0);
    const double2 ipv = cdiv(make_double2(1.0, 0.0), piv);
    if (x.mine) {
        if (x.gi == col) {
            // row col becomes the scaled pivot row
#pragma unroll
            for (int c = 0; c < nb; ++c) rv[c] = c == J ? ipv : cmul(praw[c], ipv);
        } else {
            if (p != col && x.gi == p) {
#pragma unroll
                for (int c = 0; c < nb; ++c) rv[c] = x.oldrow[c];  // row p receives row col
            }
            const double2 fs = cmul(rv[J], ipv);
#pragma unroll
            for (int c = 0; c < nb; ++c)
                rv[c] = c == J ? make_double2(-fs.x, -fs.y) : cfms(rv[c], fs, praw[c]);
        }
    }
}

template <int J>
struct GjeRegColumns {
    __device__ __forceinline__ static void run(const GjeRegCtx &x, double2 (&rv)[kPanelMax]) {
        gje_reg_column<J>(x, rv);
        GjeRegColumns<J + 1>::run(x, rv);
    }
};
template <>
struct GjeRegColumns<kPanelMax> {
    __device__ __forceinline__ static void run(const GjeRegCtx &, double2 (&)[kPanelMax]) {}
};

__global__ __launch_bounds__(256) void k_gje_panel_reg(double2 *__restrict__ A, int n, int k, int rows, int R,
                                                       int *__restrict__ ipiv, int *__restrict__ info,
                                                       GjeScratch sc, unsigned int bar_done) {
    extern __shared__ double2 lds[];
    __shared__ double wv[4], cv_s[kGjeMaxR];
    __shared__ int wrow[4], cr_s[kGjeMaxR];
    GjeRegCtx x;
    x.mat = blockIdx.x / R;
    x.r = blockIdx.x % R;
    x.Am = A + (size_t)x.mat * n * n;
    x.ip = ipiv + (size_t)x.mat * n;
    x.info = info;
    x.row0 = x.r * rows;
    x.nloc = max(0, min(rows, n - x.row0));
    x.cval = sc.cand_val + (size_t)x.mat * 2 * R;
    x.crow = sc.cand_row + (size_t)x.mat * 2 * R;
    x.crows = sc.cand_rows + (size_t)x.mat * 2 * R * kPanelMax;
    x.rbuf = sc.rowbuf + (size_t)x.mat * 2 * kPanelMax;
    x.bar = sc.bar + x.mat;
    x.oldrow = lds;                  // row k+j before the swap [kPanelMax]
    x.cand = lds + kPanelMax;        // candidate rows of all workgroups [R][kPanelMax]
    x.wv = wv;
    x.cv_s = cv_s;
    x.wrow = wrow;
    x.cr_s = cr_s;
    x.k = k;
    x.R = R;
    x.tid = threadIdx.x;
    x.lane = x.tid & 63;
    x.wave = x.tid >> 6;
    x.gi = x.row0 + x.tid;
    x.mine = x.tid < x.nloc;
    x.bar_done = bar_done;

    double2 rv[kPanelMax];
#pragma unroll
    for (int c = 0; c < kPanelMax; ++c) rv[c] = x.mine ? x.Am[(size_t)x.gi * n + k + c] : make_double2(0.0, 0.0);
    GjeRegColumns<0>::run(x, rv);
    if (x.mine) {
#pragma unroll
        for (int c = 0; c < kPanelMax; ++c) x.Am[(size_t)x.gi * n + k + c] = rv[c];
    }
}

// The columns an update touches: [lo, hi) without [ex0, ex1), numbered
// cp = 0 .. m-1 in increasing order.
struct GjeCols {
    int lo, hi, ex0, ex1;
    __host__ __device__ int count() const { return (hi - lo) - (ex1 - ex0); }
    __device__ int col(int cp) const {
        const int c = lo + cp;
        return c < ex0 ? c : c + (ex1 - ex0);
    }
};

// For every column of cs: apply the interchanges ipiv[r0 .. r0+nbr) in order
// (none when ipiv is null), copy rows r0 .. r0+nbr-1 to Rs [nbr][m] and zero
// them in A.
__global__ __launch_bounds__(64) void k_gje_swap_save(double2 *__restrict__ A, int n, int r0, int nbr, GjeCols cs,
                                                      const int *__restrict__ ipiv, double2 *__restrict__ Rs) {
    const int mat = blockIdx.y;
    double2 *Am = A + (size_t)mat * n * n;
    const int *ip = ipiv ? ipiv + (size_t)mat * n : nullptr;
    const int m = cs.count();
    double2 *R = Rs + (size_t)mat * nbr * m;
    for (int cp = blockIdx.x * blockDim.x + threadIdx.x; cp < m; cp += gridDim.x * blockDim.x) {
        const int c = cs.col(cp);
        for (int j = 0; ip && j < nbr; ++j) {
            const int p = ip[r0 + j];
            if (p > r0 + j && p < n) {
                const double2 t = Am[(size_t)(r0 + j) * n + c];
                Am[(size_t)(r0 + j) * n + c] = Am[(size_t)p * n + c];
                Am[(size_t)p * n + c] = t;
            }
        }
        for (int j = 0; j < nbr; ++j) {
            R[(size_t)j * m + cp] = Am[(size_t)(r0 + j) * n + c];
            Am[(size_t)(r0 + j) * n + c] = make_double2(0.0, 0.0);
        }
    }
}

namespace {
constexpr int UT = 64;            // update tile (rows and cols)
constexpr int ULD = UT + 4;       // padded LDS row
}  // namespace

// A[:, cs] += P * R with P = A[:, r0:r0+nbr] (n x nbr) and R = Rs (nbr x m),
// complex, as two real products over the interleaved index kk = 2j + part:
//   Re += sum_kk P'[i][kk] Bre[kk][c],  Bre[2j] = Re R, Bre[2j+1] = -Im R
//   Im += sum_kk P'[i][kk] Bim[kk][c],  Bim[2j] = Im R, Bim[2j+1] =  Re R
// The panel is staged kPanelMax columns at a time, the next chunk loaded
// into registers while the current one feeds the MFMAs.
__global__ __launch_bounds__(256, 2) void k_gje_update(double2 *__restrict__ A, int n, int r0, int nbr, GjeCols cs,
                                                    const double2 *__restrict__ Rs) {
    __shared__ double Ps[2 * kPanelMax][ULD];
    __shared__ double Rsh[2 * kPanelMax][ULD];
    const int mat = blockIdx.z;
    double2 *Am = A + (size_t)mat * n * n;
    const int m = cs.count();
    const double2 *R = Rs + (size_t)mat * nbr * m;
    const int I0 = blockIdx.x * UT, C0 = blockIdx.y * UT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1, li = lane & 15, lk = lane >> 4;

    double4_t cre[2][2], cim[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            cre[a][b] = (double4_t){0.0, 0.0, 0.0, 0.0};
            cim[a][b] = (double4_t){0.0, 0.0, 0.0, 0.0};
        }
    // P and R tiles of one chunk of kPanelMax panel columns, loaded into
    // registers one chunk ahead: the loads of chunk j0 + kPanelMax are issued
    // before the MFMAs of chunk j0
    constexpr int SIT = UT * kPanelMax / 256;
    double2 pv[SIT], rw[SIT];
    auto load_chunk = [&](int j0) {
        const int nbc = min(kPanelMax, nbr - j0);
#pragma unroll
        for (int it = 0; it < SIT; ++it) {
            const int e = tid + 256 * it;
            const int i = e / kPanelMax, j = e % kPanelMax;  // P tile: row i, panel col j
            pv[it] = (I0 + i < n && j < nbc) ? Am[(size_t)(I0 + i) * n + r0 + j0 + j] : make_double2(0.0, 0.0);
            const int jr = e / UT, c = e % UT;  // R tile: panel row jr, col c
            rw[it] = (jr < nbc && C0 + c < m) ? R[(size_t)(j0 + jr) * m + C0 + c] : make_double2(0.0, 0.0);
        }
    };
    // this lane's elements of the output tile, fetched during the last chunk
    double2 old[2][2][4];
    auto load_old = [&]() {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = I0 + wr * 32 + 16 * a + 4 * r + lk;
                    const int cp = C0 + wc * 32 + 16 * b + li;
                    old[a][b][r] = make_double2(0.0, 0.0);
                    if (i < n && cp < m) old[a][b][r] = Am[(size_t)i * n + cs.col(cp)];
                }
    };
    const double rsign = (lk & 1) ? -1.0 : 1.0;  // kr = 4 s + lk has the parity of lk
    auto stage_chunk = [&]() {
#pragma unroll
        for (int it = 0; it < SIT; ++it) {
            const int e = tid + 256 * it;
            const int i = e / kPanelMax, j = e % kPanelMax;
            Ps[2 * j][i] = pv[it].x;
            Ps[2 * j + 1][i] = pv[it].y;
            const int jr = e / UT, c = e % UT;
            Rsh[2 * jr][c] = rw[it].x;
            Rsh[2 * jr + 1][c] = rw[it].y;
        }
    };
    auto mfma_step = [&](int s) {
        const int kr = 4 * s + lk;
        double av[2], bre[2], bim[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = Ps[kr][wr * 32 + 16 * a + li];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int col = wc * 32 + 16 * b + li;
            // odd rows (imaginary parts): Bre = -Im R, Bim = Re R; even: Re R, Im R
            bre[b] = rsign * Rsh[kr][col];
            bim[b] = Rsh[kr ^ 1][col];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                cre[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bre[b], cre[a][b], 0, 0, 0);
                cim[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bim[b], cim[a][b], 0, 0, 0);
            }
    };
    // a full chunk has a compile-time step count; the last one may be narrower
    auto mfma_chunk = [&](int nbc) {
        if (nbc == kPanelMax) {
#pragma unroll 4
            for (int s = 0; s < 2 * kPanelMax / 4; ++s) mfma_step(s);
        } else {
            const int ksteps = (2 * nbc + 3) / 4;
            for (int s = 0; s < ksteps; ++s) mfma_step(s);
        }
    };
    load_chunk(0);
    int j0 = 0;
    for (; j0 + kPanelMax < nbr; j0 += kPanelMax) {
        stage_chunk();
        __syncthreads();
        load_chunk(j0 + kPanelMax);
        mfma_chunk(kPanelMax);
        __syncthreads();  // this chunk's LDS reads are done
    }
    // the last chunk: the output tile's old values are fetched under its MFMAs
    stage_chunk();
    __syncthreads();
    load_old();
    mfma_chunk(nbr - j0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = I0 + wr * 32 + 16 * a + 4 * r + lk;
                const int cp = C0 + wc * 32 + 16 * b + li;
                if (i < n && cp < m)
                    Am[(size_t)i * n + cs.col(cp)] =
                        make_double2(old[a][b][r].x + cre[a][b][r], old[a][b][r].y + cim[a][b][r]);
            }
}

// Column index map of the final column interchanges: start from the identity
// and swap entries j <-> ipiv[j] for j = n-1 down to 0.  One workgroup per
// matrix; the sequential swap chain runs on one thread over LDS copies.
__global__ void k_gje_perm(const int *__restrict__ ipiv, int n, int *__restrict__ idx) {
    extern __shared__ int perm_lds[];
    int *id = perm_lds, *ip = perm_lds + n;
    const int mat = blockIdx.x;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        id[j] = j;
        const int p = ipiv[(size_t)mat * n + j];
        ip[j] = (p >= j && p < n) ? p : j;  // an out-of-range pivot: no interchange
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int j = n - 1; j >= 0; --j) {
            const int p = ip[j];
            const int t = id[j];
            id[j] = id[p];
            id[p] = t;
        }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) idx[(size_t)mat * n + j] = id[j];
}

// out[i][c] = A[i][idx[c]], one workgroup per row, row staged in LDS (in place).
__global__ void k_gje_colperm(double2 *__restrict__ A, int n, const int *__restrict__ idx) {
    extern __shared__ double2 row[];
    const int mat = blockIdx.y;
    double2 *a = A + ((size_t)mat * n + blockIdx.x) * n;
    const int *id = idx + (size_t)mat * n;
    for (int c = threadIdx.x; c < n; c += blockDim.x) row[c] = a[c];
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += blockDim.x) a[c] = row[id[c]];
}

// The same for rows longer than LDS holds (n > 8192): every thread gathers
// its outputs' sources from the row in global memory into registers, waits
// for them, the block meets, then the row is overwritten.  n <= 256 * 48.
constexpr int kColPermPer = 48;
__global__ __launch_bounds__(256) void k_gje_colperm_reg(double2 *__restrict__ A, int n, const int *__restrict__ idx) {
    const int mat = blockIdx.y;
    double2 *a = A + ((size_t)mat * n + blockIdx.x) * n;
    const int *id = idx + (size_t)mat * n;
    double2 v[kColPermPer];
#pragma unroll
    for (int j = 0; j < kColPermPer; ++j) {
        const int c = threadIdx.x + 256 * j;
        v[j] = c < n ? a[id[c]] : make_double2(0.0, 0.0);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // every read of the row has returned
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kColPermPer; ++j) {
        const int c = threadIdx.x + 256 * j;
        if (c < n) a[c] = v[j];
    }
}

// ------------------------------------------------------- one-workgroup panels
//
// Matrices with n <= kWgThreads * kWgMaxRows take their panels from one
// workgroup each: thread t holds the panel rows that start at positions
// t, t + 512, t + 1024 (panel width kWgNb) in registers, so a column step needs
// two workgroup barriers and no grid barrier.  The column steps are those of
// k_gje_panel: pivot = largest |Re|+|Im| among positions >= col (first
// position on ties), positions col and p exchanged, every other row
// eliminated, the pivot row scaled.  A row stays in its thread's registers;
// an interchange only swaps the positions recorded for the two rows, and each
// row is stored at its final position when the panel ends.
constexpr int kWgNb = 16;
constexpr int kWgThreads = 512;
constexpr int kWgMaxRows = 3;

namespace {
template <int CTRL>
__device__ __forceinline__ void argmax_dpp(double &v, int &key) {
    const unsigned long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    const int ok = __builtin_amdgcn_mov_dpp(key, CTRL, 0xF, 0xF, false);
    const double ov = __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
    if (ov > v || (ov == v && ok < key)) {
        v = ov;
        key = ok;
    }
}

// Largest v over the wavefront, smallest key on ties; every lane gets the
// result.  Quad swaps and the half-row and row mirrors agree the 16 lanes of
// each row, then the four rows are compared.
__device__ __forceinline__ void wave_argmax_dpp(double &v, int &key) {
    argmax_dpp<0xB1>(v, key);   // quad_perm [1,0,3,2]
    argmax_dpp<0x4E>(v, key);   // quad_perm [2,3,0,1]
    argmax_dpp<0x141>(v, key);  // row_half_mirror
    argmax_dpp<0x140>(v, key);  // row_mirror
    const unsigned long long b = __double_as_longlong(v);
    double bv = 0.0;
    int bk = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int lo = __builtin_amdgcn_readlane((int)(unsigned)b, 16 * r);
        const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 16 * r);
        const int kk = __builtin_amdgcn_readlane(key, 16 * r);
        const double x = __longlong_as_double(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
        if (r == 0 || x > bv || (x == bv && kk < bk)) {
            bv = x;
            bk = kk;
        }
    }
    v = bv;
    key = bk;
}
}  // namespace

struct WgLds {
    double wv[kWgThreads / 64];
    int wk[kWgThreads / 64];
    double2 praw[kWgNb];
};

// Candidate of this thread for pivot column J (largest |Re|+|Im| among its
// rows at positions >= col, first position on ties), then of the wavefront,
// published in the LDS slots of the wavefront.
template <int ROWS, int J>
__device__ __forceinline__ void gje_wg_candidate(const double2 (&rv)[ROWS][kWgNb], const int (&pos)[ROWS], WgLds &L,
                                                 int n, int col) {
    double best = -1.0;
    int key = 0x7fffffff;
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        if (pos[r] >= col && pos[r] < n) {
            const double v = cabs1(rv[r][J]);
            if (v > best || (v == best && pos[r] < key)) {
                best = v;
                key = pos[r];
            }
        }
    }
    wave_argmax_dpp(best, key);
    if ((threadIdx.x & 63) == 0) {
        L.wv[threadIdx.x >> 6] = best;
        L.wk[threadIdx.x >> 6] = key;
    }
}

// 1 / z with one division: z is scaled by a power of two first, so that
// |z|^2 can neither overflow nor underflow.
__device__ __forceinline__ double2 crecip(double2 z) {
    int e = 0;
    (void)frexp(fmax(fabs(z.x), fabs(z.y)), &e);
    const double x = ldexp(z.x, -e), y = ldexp(z.y, -e);
    const double t = ldexp(1.0 / (x * x + y * y), -e);
    return make_double2(x * t, -y * t);
}

// Column step J (compile-time, so every row element keeps a fixed register).
// pos[r]: current position of row r of this thread (>= n: padding row of
// zeros).  The candidates of column J were published by step J - 1 (by the
// caller for J = 0): right after column J + 1 is eliminated, before the
// other columns, so their search overlaps the rest of the elimination.
template <int ROWS, int J>
__device__ __forceinline__ void gje_wg_column(double2 (&rv)[ROWS][kWgNb], int (&pos)[ROWS], WgLds &L, int n, int k,
                                              int jb, int nb, int *ip, int *info) {
    constexpr int NW = kWgThreads / 64;
    if (jb + J >= nb) return;  // uniform
    const int tid = threadIdx.x;
    const int col = k + jb + J;
    __syncthreads();
    double bv = L.wv[0];
    int p = L.wk[0];
#pragma unroll
    for (int w = 1; w < NW; ++w)
        if (L.wv[w] > bv || (L.wv[w] == bv && L.wk[w] < p)) {
            bv = L.wv[w];
            p = L.wk[w];
        }
    // p >= col; no candidate at all (a column of NaNs): no interchange, info flags the matrix
    if (p >= n) p = col;
    int piv_r = -1;  // which of this thread's rows is the pivot row
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
        if (pos[r] == p) piv_r = r;
    if (piv_r >= 0) {
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
            if (r == piv_r) {
#pragma unroll
                for (int c = 0; c < kWgNb; ++c) L.praw[c] = rv[r][c];
            }
    }
    if (tid == 0) {
        ip[col] = p;
        if (!(bv > 0.0)) atomicCAS(info, 0, col + 1);
    }
    // interchange of positions col and p
#pragma unroll
    for (int r = 0; r < ROWS; ++r) pos[r] = pos[r] == p ? col : (pos[r] == col ? p : pos[r]);
    __syncthreads();
    double2 piv = L.praw[J];
    if (piv.x == 0.0 && piv.y == 0.0) piv = make_double2(1.0, 0.0);
    const double2 ipv = crecip(piv);
    // every row is eliminated with the pivot row, read from LDS once per
    // column element by element (padding rows hold zeros and stay zero);
    // the pivot row's own result is replaced below
    double2 fs[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        fs[r] = cmul(rv[r][J], ipv);
        rv[r][J] = make_double2(-fs[r].x, -fs[r].y);
    }
    constexpr int JN = J + 1 < kWgNb ? J + 1 : J;  // next pivot column
    if (J + 1 < kWgNb) {
        const double2 pc = L.praw[JN];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) rv[r][JN] = cfms(rv[r][JN], fs[r], pc);
        if (jb + J + 1 < nb) gje_wg_candidate<ROWS, JN>(rv, pos, L, n, col + 1);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < kWgNb; ++c) {
        if (c == J || c == JN) continue;
        const double2 pc = L.praw[c];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) rv[r][c] = cfms(rv[r][c], fs[r], pc);
        __builtin_amdgcn_sched_barrier(0);  // keeps the pivot-row reads from piling up in registers
    }
    if (piv_r >= 0) {  // the pivot row, now at position col, becomes the scaled pivot row
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
            if (r == piv_r) {
#pragma unroll
                for (int c = 0; c < kWgNb; ++c) rv[r][c] = c == J ? ipv : cmul(L.praw[c], ipv);
            }
    }
    // the next step writes praw only after its first barrier, which every
    // thread reaches after these reads; its candidates were written after
    // this step's second barrier, which every thread passed after reading
    // this step's candidates
}

template <int ROWS, int... Js>
__device__ __forceinline__ void gje_wg_columns(double2 (&rv)[ROWS][kWgNb], int (&pos)[ROWS], WgLds &L, int n, int k,
                                               int jb, int nb, int *ip, int *info, std::integer_sequence<int, Js...>) {
    (gje_wg_column<ROWS, Js>(rv, pos, L, n, k, jb, nb, ip, info), ...);
}

// One workgroup per matrix (blockIdx.x), panel columns [k, k + nb), nb <= kWgNb.
// The panel moves between A and the registers through an LDS stage of 512
// rows (row stride kWgNb + 1 elements, conflict-free row reads), so the
// global accesses are whole 256-byte row segments.
constexpr int kWgStageLd = kWgNb + 1;
constexpr int kWgUnroll = 2;  // column steps per pass of the panel loop
static_assert(kWgNb % kWgUnroll == 0 && kWgUnroll >= 1, "whole passes");
constexpr size_t kWgStageBytes = sizeof(double2) * kWgThreads * kWgStageLd;

template <int ROWS>
__global__ __launch_bounds__(kWgThreads) void k_gje_panel_wg(double2 *__restrict__ A, int n, int k, int nb,
                                                             int *__restrict__ ipiv, int *__restrict__ info) {
    __shared__ WgLds L;
    extern __shared__ double2 wg_stage[];  // [kWgThreads][kWgStageLd]
    const int mat = blockIdx.x;
    double2 *Am = A + (size_t)mat * n * n;
    const int tid = threadIdx.x;
    double2 rv[ROWS][kWgNb];
    int pos[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int r0 = r * kWgThreads;
        const int cnt = min(kWgThreads, n - r0);  // >= 1
        pos[r] = r0 + tid;
        {
            // the block's 16 loads per thread in flight together
            double2 v[kWgNb];
#pragma unroll
            for (int it = 0; it < kWgNb; ++it) {
                const int e = tid + it * kWgThreads, i = e / kWgNb, c = e % kWgNb;
                v[it] = (i < cnt && c < nb) ? Am[(size_t)(r0 + i) * n + k + c] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int it = 0; it < kWgNb; ++it) {
                const int e = tid + it * kWgThreads, i = e / kWgNb, c = e % kWgNb;
                if (i < cnt) wg_stage[i * kWgStageLd + c] = v[it];
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < kWgNb; ++c) rv[r][c] = tid < cnt ? wg_stage[tid * kWgStageLd + c] : make_double2(0.0, 0.0);
        __syncthreads();
    }
    gje_wg_candidate<ROWS, 0>(rv, pos, L, n, k);
    // kWgUnroll column steps per pass on register columns 0 .. kWgUnroll-1,
    // then the columns rotate left by kWgUnroll, so that the next pass again
    // starts at register column 0; after kWgNb / kWgUnroll passes every
    // column is back in its own register.  The pass is a real loop: fully
    // unrolled, the three-row panel is about 100 KB of code, more than the
    // instruction cache holds, and each launch fetches all of it once.
#pragma unroll 1
    for (int jb = 0; jb < kWgNb; jb += kWgUnroll) {
        gje_wg_columns<ROWS>(rv, pos, L, n, k, jb, nb, ipiv + (size_t)mat * n, info + mat,
                             std::make_integer_sequence<int, kWgUnroll>{});
        if (kWgUnroll < kWgNb) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                double2 t[kWgNb];
#pragma unroll
                for (int c = 0; c < kWgNb; ++c) t[c] = rv[r][(c + kWgUnroll) % kWgNb];
#pragma unroll
                for (int c = 0; c < kWgNb; ++c) rv[r][c] = t[c];
            }
        }
    }
    // every row to its final position, one 512-position block at a time
#pragma unroll
    for (int b = 0; b < ROWS; ++b) {
        const int r0 = b * kWgThreads;
        const int cnt = min(kWgThreads, n - r0);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            if (pos[r] >= r0 && pos[r] < r0 + cnt) {
#pragma unroll
                for (int c = 0; c < kWgNb; ++c) wg_stage[(pos[r] - r0) * kWgStageLd + c] = rv[r][c];
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int it = 0; it < kWgNb; ++it) {
            const int e = tid + it * kWgThreads, i = e / kWgNb, c = e % kWgNb;
            if (i < cnt && c < nb) Am[(size_t)(r0 + i) * n + k + c] = wg_stage[i * kWgStageLd + c];
        }
    }
}

// ---------------------------------------------------------------- host side

int launch_eps_build(const double2 *chi, const double *v, int ng, int nw, double2 *eps, hipStream_t st) {
    const size_t total = (size_t)ng * ng * nw;
    const int blocks = (int)std::min<size_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(k_eps_build, dim3(blocks), dim3(256), 0, st, chi, v, ng, nw, eps);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

size_t gje_scratch_bytes(int nmat, int R) {
    size_t b = 0;
    b += sizeof(double) * nmat * 2 * R;
    b += sizeof(int) * nmat * 2 * R;
    b += sizeof(double2) * nmat * 2 * R * kPanelMax;
    b += sizeof(double2) * nmat * 2 * kPanelMax;
    b += sizeof(unsigned int) * nmat;
    return b + 6 * 256;
}

static char *align256(char *p) { return (char *)(((uintptr_t)p + 255) & ~(uintptr_t)255); }

// Width of the outer blocks: panels run kWgNb or kPanelMax columns at a time
// and update only the other columns of their outer block; the rest of the
// matrix takes one rank-(outer width) update per outer block.
static int gje_outer_nb(int n) { return n >= 3000 ? 4 * kPanelMax : 2 * kPanelMax; }

// Row interchanges and rank-nbr update of the panel [r0, r0 + nbr) applied to
// the columns cs: A[:, cs] = swapped, panel rows saved and zeroed, += P Rs.
static int gje_apply(double2 *A, int n, int nmat, int r0, int nbr, GjeCols cs, const int *ipiv, double2 *Rs,
                     hipStream_t st) {
    const int m = cs.count();
    if (m <= 0) return BGW_OK;
    hipLaunchKernelGGL(k_gje_swap_save, dim3((m + 63) / 64, nmat), dim3(64), 0, st, A, n, r0, nbr, cs, ipiv, Rs);
    hipLaunchKernelGGL(k_gje_update, dim3((n + UT - 1) / UT, (m + UT - 1) / UT, nmat), dim3(256), 0, st, A, n, r0,
                       nbr, cs, (const double2 *)Rs);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

// In-place inversion of `nmat` matrices A[nmat][n][n].  ws: device workspace of
// at least gje_workspace_bytes(n, nmat, R) bytes.  info: [nmat], zeroed here.
size_t gje_workspace_bytes(int n, int nmat, int R) {
    return gje_scratch_bytes(nmat, R) + sizeof(double2) * (size_t)nmat * gje_outer_nb(n) * n + 256 +
           sizeof(int) * (size_t)nmat * n * 2 + 512;
}

static size_t gje_panel_lds(int rows, int R) {
    return sizeof(double2) * ((size_t)rows * (kPanelMax + 1) + 2 * kPanelMax + (size_t)R * kPanelMax);
}

static size_t gje_panel_reg_lds(int R) { return sizeof(double2) * (kPanelMax + (size_t)R * kPanelMax); }

// rows of the panel held by one workgroup (one per thread): few workgroups per
// matrix keep the per-column grid barrier cheap
int gje_rows_per_wg(int n) { return std::min(256, n); }

// One workgroup per matrix panel for n <= 1536, unless BGW_GJE_PATH=coop asks
// for the cooperative multi-workgroup panels.
static bool gje_one_wg(int n) {
    if (n > kWgThreads * kWgMaxRows) return false;
    const char *e = std::getenv("BGW_GJE_PATH");
    return !(e && std::strcmp(e, "coop") == 0);
}

static int launch_gje_invert_wg(double2 *A, int n, int nmat, int *ipiv, int *info, double2 *Rs, hipStream_t st) {
    const int rows = (n + kWgThreads - 1) / kWgThreads;
    const void *kern = rows == 1 ? (const void *)k_gje_panel_wg<1>
                     : rows == 2 ? (const void *)k_gje_panel_wg<2>
                                 : (const void *)k_gje_panel_wg<3>;
    BGW_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kWgStageBytes));
    const int nbo = gje_outer_nb(n);
    for (int k = 0; k < n; k += nbo) {
        const int ke = std::min(n, k + nbo);
        for (int ks = k; ks < ke; ks += kWgNb) {
            const int nb = std::min(kWgNb, ke - ks);
            void *args[] = {&A, (void *)&n, &ks, (void *)&nb, &ipiv, &info};
            BGW_HIP(hipLaunchKernel(kern, dim3(nmat), dim3(kWgThreads), args, kWgStageBytes, st));
            BGW_TRY(gje_apply(A, n, nmat, ks, nb, GjeCols{k, ke, ks, ks + nb}, ipiv, Rs, st));
        }
        BGW_TRY(gje_apply(A, n, nmat, k, ke - k, GjeCols{0, n, k, ke}, ipiv, Rs, st));
    }
    return BGW_OK;
}

static int launch_gje_invert_coop(double2 *A, int n, int nmat, int *info, GjeScratch sc, double2 *Rs, int *ipiv,
                                  int rows, int R, hipStream_t st);
static int launch_gje_unpermute(double2 *A, int n, int nmat, const int *ipiv, int *idx, hipStream_t st);

int launch_gje_invert(double2 *A, int n, int nmat, int *info, void *ws, int *ipiv_ws, hipStream_t st) {
    const int rows = gje_rows_per_wg(n);
    const int R = (n + rows - 1) / rows;
    char *p = align256((char *)ws);
    GjeScratch sc;
    sc.cand_val = (double *)p; p = align256(p + sizeof(double) * nmat * 2 * R);
    sc.cand_row = (int *)p; p = align256(p + sizeof(int) * nmat * 2 * R);
    sc.cand_rows = (double2 *)p; p = align256(p + sizeof(double2) * nmat * 2 * R * kPanelMax);
    sc.rowbuf = (double2 *)p; p = align256(p + sizeof(double2) * nmat * 2 * kPanelMax);
    sc.bar = (unsigned int *)p; p = align256(p + sizeof(unsigned int) * nmat);
    double2 *Rs = (double2 *)p; p = align256(p + sizeof(double2) * (size_t)nmat * gje_outer_nb(n) * n);
    int *ipiv = ipiv_ws;
    int *idx = ipiv + (size_t)nmat * n;

    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, sc.bar, (size_t)nmat, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (unsigned int *)info, (size_t)nmat, 0u);
    BGW_HIP(hipGetLastError());

    if (gje_one_wg(n)) {
        BGW_TRY(launch_gje_invert_wg(A, n, nmat, ipiv, info, Rs, st));
    } else {
        BGW_TRY(launch_gje_invert_coop(A, n, nmat, info, sc, Rs, ipiv, rows, R, st));
    }
    return launch_gje_unpermute(A, n, nmat, ipiv, idx, st);
}

static int launch_gje_invert_coop(double2 *A, int n, int nmat, int *info, GjeScratch sc, double2 *Rs, int *ipiv,
                                  int rows, int R, hipStream_t st) {
    if (R > kGjeMaxR) return BGW_ERR_UNSUPPORTED;
    const size_t lds = gje_panel_lds(rows, R);
    BGW_HIP(hipFuncSetAttribute((const void *)k_gje_panel<kPanelMax>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    BGW_HIP(hipFuncSetAttribute((const void *)k_gje_panel<0>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const size_t rlds_panel = gje_panel_reg_lds(R);
    unsigned int bar_done = 0;
    const int nbo = gje_outer_nb(n);
    for (int k = 0; k < n; k += nbo) {
        const int ke = std::min(n, k + nbo);
        for (int ks = k; ks < ke; ks += kPanelMax) {
            const int nb = std::min(kPanelMax, ke - ks);
            void *args[] = {&A, (void *)&n, &ks, (void *)&nb, (void *)&rows, (void *)&R, &ipiv, &info, &sc, &bar_done};
            if (nb == kPanelMax) {
                void *rargs[] = {&A, (void *)&n, &ks, (void *)&rows, (void *)&R, &ipiv, &info, &sc, &bar_done};
                BGW_HIP(hipLaunchCooperativeKernel((const void *)k_gje_panel_reg, dim3(R * nmat), dim3(256), rargs,
                                                   rlds_panel, st));
            } else {
                BGW_HIP(hipLaunchCooperativeKernel((const void *)k_gje_panel<0>, dim3(R * nmat), dim3(256), args, lds,
                                                   st));
            }
            bar_done += nb;
            BGW_TRY(gje_apply(A, n, nmat, ks, nb, GjeCols{k, ke, ks, ks + nb}, ipiv, Rs, st));
        }
        BGW_TRY(gje_apply(A, n, nmat, k, ke - k, GjeCols{0, n, k, ke}, ipiv, Rs, st));
    }
    return BGW_OK;
}

static int launch_gje_unpermute(double2 *A, int n, int nmat, const int *ipiv, int *idx, hipStream_t st) {
    const size_t plds = sizeof(int) * 2 * (size_t)n;
    BGW_HIP(hipFuncSetAttribute((const void *)k_gje_perm, hipFuncAttributeMaxDynamicSharedMemorySize, (int)plds));
    hipLaunchKernelGGL(k_gje_perm, dim3(nmat), dim3(256), plds, st, ipiv, n, idx);
    if (n > 8192) {
        if (n > 256 * kColPermPer) return BGW_ERR_UNSUPPORTED;
        hipLaunchKernelGGL(k_gje_colperm_reg, dim3(n, nmat), dim3(256), 0, st, A, n, idx);
        BGW_HIP(hipGetLastError());
        return BGW_OK;
    }
    const size_t rlds = sizeof(double2) * (size_t)n;
    BGW_HIP(hipFuncSetAttribute((const void *)k_gje_colperm, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rlds));
    hipLaunchKernelGGL(k_gje_colperm, dim3(n, nmat), dim3(256), rlds, st, A, n, idx);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

// Largest group of matrices inverted together: for cooperative panels, the
// matrices whose panel workgroups can be co-resident; one-workgroup panels
// need no co-residency (the cap bounds the workspace).
int gje_max_group(int n) {
    if (gje_one_wg(n)) return 64;
    const int rows = gje_rows_per_wg(n);
    const int R = (n + rows - 1) / rows;
    const size_t lds = gje_panel_lds(rows, R);
    int per_cu = 0;
    if (hipFuncSetAttribute((const void *)k_gje_panel<kPanelMax>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
        return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_gje_panel<kPanelMax>, 256, lds) !=
            hipSuccess ||
        per_cu <= 0)
        return 1;
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const long long slots = (long long)per_cu * cus;
    return (int)std::max<long long>(1, slots / R);
}


// ---------------------------------------------------------------------------
// Inversion without row interchanges, for chi Hermitian and negative
// semidefinite: chi0 at zero and at imaginary frequency, where every weight
// of the chi sum is negative.  With S = diag(v^1/2) (v > 0),
//   eps = 1 - v chi = S epst S^-1,   epst = 1 - S chi S,
// and epst is Hermitian with every eigenvalue >= 1.  Every leading principal
// block of epst is then >= 1 as well, so each elimination pivot (the ratio
// of consecutive leading minors, the same for eps and epst because a
// diagonal similarity keeps every principal minor) is real and >= 1:
// elimination needs no interchanges, and without them Gauss-Jordan is
// exactly as stable as on the Hermitian positive definite epst.  The column
// steps then need no search over the rows, and only the diagonal block of a
// panel is eliminated step by step:
//   k_nsd_check  max over (G, G') of sqrt(v_G v_G') |chi_GG' - conj chi_G'G|
//                and of sqrt(v_G v_G') |chi_GG'| (read before epsilon is
//                built in place), +inf when some v <= 0 or a value is not
//                finite;
//   k_nsd_diag   one workgroup per matrix inverts the panel's diagonal block
//                D (kNsdNb x kNsdNb, registers, one barrier per step) in
//                place and into Dinv, watching every pivot;
//   k_nsd_rows   the panel's other rows become -A[i, K] D^-1, all rows in
//                parallel;
//   k_nsd_save   the panel rows of the other columns copied and zeroed, one
//                workgroup row per panel row;
// then the pivoted path's rank update (k_gje_update), in the same two-level
// outer blocks.  A
// matrix whose chi is not Hermitian to 1e-8 (relative, on the symmetrised
// scale) or has v <= 0 gets info = -2; one with a pivot whose real part is
// below 1/2, or that is not real to half of it, gets info = -3 (chi not
// negative semidefinite).  Either way epsinv is unspecified.
constexpr int kNsdNb = 64;        // panel width (diagonal block size)
constexpr int kNsdDiagThreads = 512;
constexpr int kNsdRowsPer = 16;   // rows of one k_nsd_rows workgroup
constexpr int kNsdTile = 32;      // tile of the Hermitian check
constexpr double kNsdHermTol = 1e-8;

__device__ __forceinline__ void atomic_max_nonneg(double *p, double x) {
    // non-negative doubles order like their bit patterns
    atomicMax((unsigned long long *)p, (unsigned long long)__double_as_longlong(x));
}

// Upper tile pairs (I <= J) of each matrix; chk[mat] = {non-Hermiticity, max}.
__global__ __launch_bounds__(256) void k_nsd_check(const double2 *__restrict__ chi, const double *__restrict__ v,
                                                   int n, int tiles, double *__restrict__ chk) {
    __shared__ double2 T[kNsdTile][kNsdTile + 1];
    __shared__ double red[2][4];
    const int mat = blockIdx.y;
    // blockIdx.x enumerates the pairs I <= J row by row
    int I = 0, rem = blockIdx.x;
    while (rem >= tiles - I) {
        rem -= tiles - I;
        ++I;
    }
    const int J = I + rem;
    const double2 *C = chi + (size_t)mat * n * n;
    const int tid = threadIdx.x, tx = tid & 31, ty = tid >> 5;
    const int I0 = I * kNsdTile, J0 = J * kNsdTile;
#pragma unroll
    for (int r = 0; r < kNsdTile; r += 8) {  // T[a][b] = chi[J0 + a][I0 + b]
        const int a = ty + r, row = J0 + a, col = I0 + tx;
        T[a][tx] = (row < n && col < n) ? C[(size_t)row * n + col] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    double nh = 0.0, mx = 0.0;
    const int j = J0 + tx;
    const double vj = j < n ? v[j] : 1.0;
#pragma unroll
    for (int r = 0; r < kNsdTile; r += 8) {
        const int i = I0 + ty + r;
        if (i < n && j < n) {
            const double vi = v[i];
            const double2 x = C[(size_t)i * n + j];
            const double2 y = T[tx][ty + r];  // chi[j][i]
            const double sc = sqrt(vi * vj);
            double d = sc * sqrt((x.x - y.x) * (x.x - y.x) + (x.y + y.y) * (x.y + y.y));
            double m = sc * fmax(sqrt(x.x * x.x + x.y * x.y), sqrt(y.x * y.x + y.y * y.y));
            if (!(vi > 0.0) || !(vj > 0.0) || !(d <= DBL_MAX) || !(m <= DBL_MAX)) d = m = INFINITY;
            nh = fmax(nh, d);
            mx = fmax(mx, m);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        nh = fmax(nh, __shfl_xor(nh, off, 64));
        mx = fmax(mx, __shfl_xor(mx, off, 64));
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = nh;
        red[1][tid >> 6] = mx;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < 4; ++w) {
            nh = fmax(nh, red[0][w]);
            mx = fmax(mx, red[1][w]);
        }
        atomic_max_nonneg(chk + 2 * mat, nh);
        atomic_max_nonneg(chk + 2 * mat + 1, mx);
    }
}

// Gauss-Jordan without interchanges on D = A[K, K], K = [ks, ks + nb),
// padded to kNsdNb with the identity.  Thread t holds column t / 8 of the
// rows 8 (t % 8) + r, so the eight threads of the pivot column sit in one
// wavefront and, with the steps unrolled by eight, the pivot row's register
// is known at compile time.  A step is one complex FMA per entry,
// d -= f_i s_j with f the old pivot column and s the new pivot row
// (inv * old row); the pivot row and column are then set exactly: row c to
// s, column c to -f inv, (c, c) to inv.  The pivot row and column go
// through LDS, double-buffered (one barrier per step), and every LDS read of
// a step is issued before its arithmetic.
__global__ __launch_bounds__(kNsdDiagThreads) void k_nsd_diag(double2 *__restrict__ A, int n, int ks, int nb,
                                                              double2 *__restrict__ Dinv,
                                                              const double *__restrict__ chk, int *__restrict__ info) {
    constexpr int CPT = kNsdDiagThreads / kNsdNb;  // threads per column
    constexpr int RPT = kNsdNb / CPT;              // rows per thread
    __shared__ double2 rowb[2][kNsdNb], colb[2][kNsdNb];
    const int mat = blockIdx.x;
    double2 *Am = A + (size_t)mat * n * n;
    const int t = threadIdx.x, j = t / CPT, rg = t % CPT;  // rows RPT rg + r
    double2 d[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int i = RPT * rg + r;
        d[r] = (i < nb && j < nb) ? Am[(size_t)(ks + i) * n + ks + j] : make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    bool bad = false;
    for (int cb = 0; cb * RPT < nb; ++cb) {
        const bool holder = rg == cb;  // this thread holds the pivot rows of these RPT steps
#pragma unroll
        for (int cr = 0; cr < RPT; ++cr) {
            const int c = cb * RPT + cr;
            if (c >= nb) break;
            const int b = c & 1;
            if (holder) rowb[b][j] = d[cr];
            if (j == c) {
#pragma unroll
                for (int r = 0; r < RPT; ++r) colb[b][RPT * rg + r] = d[r];
            }
            __syncthreads();
            const double2 p = rowb[b][c];
            const double2 rj = rowb[b][j];
            double2 f[RPT];
#pragma unroll
            for (int r = 0; r < RPT; ++r) f[r] = colb[b][RPT * rg + r];
            __builtin_amdgcn_sched_barrier(0);
            bad |= !(p.x >= 0.5 && fabs(p.y) <= 0.5 * p.x);
            const double rden = 1.0 / (p.x * p.x + p.y * p.y);
            const double2 inv = make_double2(p.x * rden, -p.y * rden);
            const double2 sj = cmul(inv, rj);
#pragma unroll
            for (int r = 0; r < RPT; ++r) d[r] = cfms(d[r], f[r], sj);
            if (holder) d[cr] = sj;
            if (j == c) {
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    const double2 fi = cmul(f[r], inv);
                    d[r] = make_double2(-fi.x, -fi.y);
                }
                if (holder) d[cr] = inv;
            }
        }
    }
    double2 *Dm = Dinv + (size_t)mat * kNsdNb * kNsdNb;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int i = RPT * rg + r;
        if (i < nb && j < nb) {
            Am[(size_t)(ks + i) * n + ks + j] = d[r];
            Dm[i * kNsdNb + j] = d[r];
        }
    }
    if (t == 0) {
        if (ks == 0) {
            const double nh = chk[2 * mat], mx = chk[2 * mat + 1];
            if (!(mx <= DBL_MAX && nh <= kNsdHermTol * mx)) info[mat] = -2;
        }
        if (bad && info[mat] == 0) info[mat] = -3;
    }
}

// A[i, K] = -A[i, K] Dinv for the rows i outside K of one block of kNsdRowsPer
// rows.  Thread t: row t / 16, columns t % 16 + 16 q.
__global__ __launch_bounds__(256) void k_nsd_rows(double2 *__restrict__ A, int n, int ks, int nb,
                                                  const double2 *__restrict__ Dinv) {
    extern __shared__ double2 nsd_lds[];
    constexpr int ALD = kNsdNb + 1;
    constexpr int CG = 256 / kNsdRowsPer;  // column groups
    constexpr int NQ = kNsdNb / CG;
    double2 *Ds = nsd_lds;                        // [kNsdNb][kNsdNb]
    double2 *As = nsd_lds + kNsdNb * kNsdNb;      // [kNsdRowsPer][ALD]
    const int mat = blockIdx.y;
    double2 *Am = A + (size_t)mat * n * n;
    const double2 *Dm = Dinv + (size_t)mat * kNsdNb * kNsdNb;
    const int i0 = blockIdx.x * kNsdRowsPer, tid = threadIdx.x;
    for (int e = tid; e < kNsdNb * kNsdNb; e += 256) {
        const int k = e / kNsdNb, jj = e % kNsdNb;
        Ds[e] = (k < nb && jj < nb) ? Dm[e] : make_double2(0.0, 0.0);
    }
    for (int e = tid; e < kNsdRowsPer * kNsdNb; e += 256) {
        const int il = e / kNsdNb, k = e % kNsdNb, i = i0 + il;
        As[il * ALD + k] = (i < n && k < nb) ? Am[(size_t)i * n + ks + k] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int il = tid / CG, cg = tid % CG;
    double2 acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = make_double2(0.0, 0.0);
    for (int k = 0; k < nb; ++k) {
        const double2 a = As[il * ALD + k];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const double2 x = Ds[k * kNsdNb + cg + CG * q];
            acc[q].x = fma(a.x, x.x, fma(-a.y, x.y, acc[q].x));
            acc[q].y = fma(a.x, x.y, fma(a.y, x.x, acc[q].y));
        }
    }
    const int i = i0 + il;
    if (i < n && (i < ks || i >= ks + nb)) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int jj = cg + CG * q;
            if (jj < nb) Am[(size_t)i * n + ks + jj] = make_double2(-acc[q].x, -acc[q].y);
        }
    }
}

// Rows r0 .. r0 + nbr of the columns cs copied to Rs [nbr][m] and zeroed in A
// (the save of k_gje_swap_save without interchanges), one row per blockIdx.y.
__global__ __launch_bounds__(256) void k_nsd_save(double2 *__restrict__ A, int n, int r0, int nbr, GjeCols cs,
                                                  double2 *__restrict__ Rs) {
    const int mat = blockIdx.z, jr = blockIdx.y;
    const int m = cs.count();
    const int cp = blockIdx.x * 256 + threadIdx.x;
    if (cp >= m) return;
    double2 *a = A + (size_t)mat * n * n + (size_t)(r0 + jr) * n + cs.col(cp);
    Rs[(size_t)mat * nbr * m + (size_t)jr * m + cp] = *a;
    *a = make_double2(0.0, 0.0);
}

namespace {
struct NsdWs {
    double2 *Rs, *Dinv;
    double *chk;
};
NsdWs nsd_layout(void *ws, int n, int nmat, int nall) {
    char *p = align256((char *)ws);
    NsdWs w;
    w.chk = (double *)p; p = align256(p + sizeof(double) * 2 * (size_t)nall);
    w.Dinv = (double2 *)p; p = align256(p + sizeof(double2) * (size_t)nmat * kNsdNb * kNsdNb);
    w.Rs = (double2 *)p;
    return w;
}
}  // namespace

// Workspace of the interchange-free inversion: nmat matrices per group,
// nall matrices checked at once.
size_t nsd_workspace_bytes(int n, int nmat, int nall) {
    return 256 + ((sizeof(double) * 2 * (size_t)nall + 255) / 256) * 256 +
           ((sizeof(double2) * (size_t)nmat * kNsdNb * kNsdNb + 255) / 256) * 256 +
           sizeof(double2) * (size_t)nmat * gje_outer_nb(n) * n + 256;
}

int launch_nsd_check(const double2 *chi, const double *v, int n, int nall, int nmat, void *ws, hipStream_t st) {
    NsdWs w = nsd_layout(ws, n, nmat, nall);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, (unsigned int *)w.chk, (size_t)4 * nall, 0u);
    const int tiles = (n + kNsdTile - 1) / kNsdTile;
    const long long pairs = (long long)tiles * (tiles + 1) / 2;
    for (int m0 = 0; m0 < nall; m0 += 65535) {
        const int mm = std::min(65535, nall - m0);
        hipLaunchKernelGGL(k_nsd_check, dim3((unsigned)pairs, mm), dim3(256), 0, st, chi + (size_t)m0 * n * n, v, n,
                           tiles, w.chk + 2 * (size_t)m0);
    }
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

// Rank-nbr update of the columns cs by the panel [r0, r0 + nbr), no interchanges.
static int nsd_apply(double2 *A, int n, int nmat, int r0, int nbr, GjeCols cs, double2 *Rs, hipStream_t st) {
    const int m = cs.count();
    if (m <= 0) return BGW_OK;
    hipLaunchKernelGGL(k_nsd_save, dim3((m + 255) / 256, nbr, nmat), dim3(256), 0, st, A, n, r0, nbr, cs, Rs);
    hipLaunchKernelGGL(k_gje_update, dim3((n + UT - 1) / UT, (m + UT - 1) / UT, nmat), dim3(256), 0, st, A, n, r0,
                       nbr, cs, (const double2 *)Rs);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

// In place: A[nmat][n][n] (matrices m0 .. m0 + nmat of the checked set).
int launch_nsd_invert(double2 *A, int n, int nmat, int m0, int nall, int *info, void *ws, hipStream_t st) {
    NsdWs w = nsd_layout(ws, n, nmat, nall);
    const double *chk = w.chk + 2 * (size_t)m0;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (unsigned int *)info, (size_t)nmat, 0u);
    const size_t rlds = sizeof(double2) * ((size_t)kNsdNb * kNsdNb + (size_t)kNsdRowsPer * (kNsdNb + 1));
    BGW_HIP(hipFuncSetAttribute((const void *)k_nsd_rows, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rlds));
    const int nbo = gje_outer_nb(n);
    for (int k = 0; k < n; k += nbo) {
        const int ke = std::min(n, k + nbo);
        for (int ks = k; ks < ke; ks += kNsdNb) {
            const int nb = std::min(kNsdNb, ke - ks);
            hipLaunchKernelGGL(k_nsd_diag, dim3(nmat), dim3(kNsdDiagThreads), 0, st, A, n, ks, nb, w.Dinv, chk, info);
            hipLaunchKernelGGL(k_nsd_rows, dim3((n + kNsdRowsPer - 1) / kNsdRowsPer, nmat), dim3(256), rlds, st, A, n,
                               ks, nb, (const double2 *)w.Dinv);
            BGW_TRY(nsd_apply(A, n, nmat, ks, nb, GjeCols{k, ke, ks, ks + nb}, w.Rs, st));
        }
        BGW_TRY(nsd_apply(A, n, nmat, k, ke - k, GjeCols{0, n, k, ke}, w.Rs, st));
    }
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

}  // namespace bgw
