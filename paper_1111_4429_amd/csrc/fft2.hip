// Fast paths of the pair-density transforms for grids whose y and z lengths
// are 16 x r or 8 x r (r small): compile-time sizes, register-resident radix-16
// (or radix-8) FFT passes, pruned output combination, L2-friendly work order.
//
// Pair kernel, per x-plane of one pair:
//   1. product conj(u_v) u_c loaded with coalesced 16-byte accesses into an LDS
//      plane (row stride padded so the strided radix reads are bank-conflict free);
//   2. z: each thread takes one line's elements z = za + R2*zb (zb = 0..R1-1),
//      does the R1-point DFT in registers, applies the twiddle w_n^{za*kb} and
//      writes the results back in place; only the bez dielectric-box outputs
//      are then combined (R2-point sums);
//   3. y: the same two steps on the bez pruned columns;
//   4. x: every sphere point accumulates w_{n1}^{mx x} R[my][mz] in registers.
// Band kernel (u_n(r) from the sphere): the x stage sums each x-stick, the y
// stage is a direct sum over the box rows, the z stage a direct sum over the
// box columns evaluated by a thread that owns a fixed z (its twiddles live in
// registers) and stored with coalesced writes.
#include <cstdlib>

#include "common.h"

namespace bgw {

namespace {

constexpr double kC8 = 0.92387953251128675613;   // cos(pi/8)
constexpr double kS8 = 0.38268343236508977173;   // sin(pi/8)
constexpr double kR2 = 0.70710678118654752440;   // sqrt(2)/2
constexpr double kS60 = 0.86602540378443864676;  // sin(2 pi/3)

__device__ inline double2 mul_i(double2 a) { return make_double2(-a.y, a.x); }
// a * (r + i r)
__device__ inline double2 mul_rr(double2 a, double r) { return make_double2(r * (a.x - a.y), r * (a.x + a.y)); }
// a * (-r + i r)
__device__ inline double2 mul_mrr(double2 a, double r) { return make_double2(-r * (a.x + a.y), r * (a.x - a.y)); }

__device__ inline void d2(double2 &a, double2 &b) {
    const double2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}
__device__ inline void d4(double2 &a, double2 &b, double2 &c, double2 &d) {
    const double2 t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), t3 = csub(b, d);
    const double2 it3 = mul_i(t3);
    a = cadd(t0, t2);
    c = csub(t0, t2);
    b = cadd(t1, it3);
    d = csub(t1, it3);
}

// In-register DFT, kernel exp(+2 pi i j k / R), natural order in and out.
template <int R>
struct RegDFT;

template <>
struct RegDFT<1> {
    __device__ static void run(double2 *) {}
};
template <>
struct RegDFT<2> {
    __device__ static void run(double2 *v) { d2(v[0], v[1]); }
};
template <>
struct RegDFT<4> {
    __device__ static void run(double2 *v) { d4(v[0], v[1], v[2], v[3]); }
};
template <>
struct RegDFT<8> {
    __device__ static void run(double2 *v) {
        // x[a + 2b]: DFT4 over b, twiddle w8^{a c}, DFT2 over a
        d4(v[0], v[2], v[4], v[6]);
        d4(v[1], v[3], v[5], v[7]);
        v[3] = mul_rr(v[3], kR2);
        v[5] = mul_i(v[5]);
        v[7] = mul_mrr(v[7], kR2);
        d2(v[0], v[1]);
        d2(v[2], v[3]);
        d2(v[4], v[5]);
        d2(v[6], v[7]);
        // X[c + 4d] sits at v[2c + d]
        double2 t[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) t[i] = v[i];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int d = 0; d < 2; ++d) v[c + 4 * d] = t[2 * c + d];
    }
};
template <>
struct RegDFT<16> {
    __device__ static void run(double2 *v) {
        // x[a + 4b]: DFT4 over b, twiddle w16^{a c}, DFT4 over a
#pragma unroll
        for (int a = 0; a < 4; ++a) d4(v[a], v[a + 4], v[a + 8], v[a + 12]);
        const double2 w1 = make_double2(kC8, kS8), w3 = make_double2(kS8, kC8);
        const double2 w9 = make_double2(-kC8, -kS8);
        v[5] = cmul(v[5], w1);
        v[9] = mul_rr(v[9], kR2);
        v[13] = cmul(v[13], w3);
        v[6] = mul_rr(v[6], kR2);
        v[10] = mul_i(v[10]);
        v[14] = mul_mrr(v[14], kR2);
        v[7] = cmul(v[7], w3);
        v[11] = mul_mrr(v[11], kR2);
        v[15] = cmul(v[15], w9);
#pragma unroll
        for (int c = 0; c < 4; ++c) d4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
        // X[c + 4d] sits at v[4c + d]
        double2 t[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) t[i] = v[i];
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int d = 0; d < 4; ++d) v[c + 4 * d] = t[4 * c + d];
    }
};

template <>
struct RegDFT<3> {
    __device__ static void run(double2 *v) {
        const double2 s = v[0], t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
        const double2 m = make_double2(s.x - 0.5 * t1.x, s.y - 0.5 * t1.y);
        const double2 is = make_double2(-kS60 * t2.y, kS60 * t2.x);
        v[0] = cadd(s, t1);
        v[1] = cadd(m, is);
        v[2] = csub(m, is);
    }
};

// cos(2 pi j / 96), j = 0..24, rounded to the nearest double; every twiddle
// exp(2 pi i j / N) of the lengths 16, 24, 32, 48 and 96 is one of these
// values up to sign (quarter-wave symmetry).
constexpr double kCos96[25] = {1.0,
                               0.9978589232386035,
                               0.9914448613738104,
                               0.9807852804032304,
                               0.9659258262890683,
                               0.9469301294951057,
                               0.9238795325112867,
                               0.8968727415326883,
                               0.8660254037844386,
                               0.8314696123025452,
                               0.7933533402912352,
                               0.7518398074789774,
                               0.7071067811865476,
                               0.6593458151000688,
                               0.6087614290087207,
                               0.5555702330196022,
                               0.5,
                               0.4422886902190013,
                               0.3826834323650898,
                               0.3214394653031616,
                               0.25881904510252074,
                               0.19509032201612828,
                               0.1305261922200516,
                               0.06540312923014306,
                               0.0};
__host__ __device__ constexpr double cos96(int j) {
    j = ((j % 96) + 96) % 96;
    return j <= 24 ? kCos96[j] : (j <= 48 ? -kCos96[48 - j] : (j <= 72 ? -kCos96[j - 48] : kCos96[96 - j]));
}
__host__ __device__ constexpr double sin96(int j) { return cos96(24 - j); }

// Whole-line DFT in registers, kernel exp(+2 pi i j k / N), natural order in
// and out, N = R1 * R2: R2 DFTs of length R1 over x[a + R2 b], twiddles
// w_N^{a kb}, then R1 DFTs of length R2 (output kb + R1 ka).
template <int R1, int R2>
struct RegFFT2 {
    static constexpr int N = R1 * R2;
    __device__ static void run(double2 *v) {
        double2 y[R2][R1];
#pragma unroll
        for (int a = 0; a < R2; ++a) {
#pragma unroll
            for (int b = 0; b < R1; ++b) y[a][b] = v[a + R2 * b];
            RegDFT<R1>::run(y[a]);
#pragma unroll
            for (int kb = 1; kb < R1; ++kb)
                if (a) y[a][kb] = cmul(y[a][kb], make_double2(cos96(a * kb * (96 / N)), sin96(a * kb * (96 / N))));
            // one sub-transform at a time keeps the live registers near the line itself
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int kb = 0; kb < R1; ++kb) {
            double2 z[R2];
#pragma unroll
            for (int a = 0; a < R2; ++a) z[a] = y[a][kb];
            RegDFT<R2>::run(z);
#pragma unroll
            for (int ka = 0; ka < R2; ++ka) v[kb + R1 * ka] = z[ka];
            __builtin_amdgcn_sched_barrier(0);
        }
    }
};

template <int N>
struct LineDFT;
template <>
struct LineDFT<16> : RegDFT<16> {};
template <>
struct LineDFT<24> : RegFFT2<8, 3> {};
template <>
struct LineDFT<32> : RegFFT2<8, 4> {};

// n = R1 * R2; element z of a line at line[z * es].  Stage 1 (in place): for
// each za < R2, Y_za = DFT_R1 over x[za + R2 zb], times w_n^{za kb}, stored at
// position za + R2 kb.  Output k = kb + R1 ka is then
// sum_za w_R2^{za ka} Y_za[kb].
template <int R1, int R2>
struct LineFFT {
    static constexpr int N = R1 * R2;

    __device__ static void stage1(double2 *buf, int nlines, int ls, int es, const double2 *twN) {
        for (int item = threadIdx.x; item < nlines * R2; item += blockDim.x) {
            const int line = item / R2;
            const int za = item - line * R2;
            double2 *b = buf + line * ls + za * es;
            double2 v[R1];
#pragma unroll
            for (int zb = 0; zb < R1; ++zb) v[zb] = b[zb * R2 * es];
            RegDFT<R1>::run(v);
            if (za) {
#pragma unroll
                for (int kb = 1; kb < R1; ++kb) v[kb] = cmul(v[kb], twN[za * kb]);
            }
#pragma unroll
            for (int kb = 0; kb < R1; ++kb) b[kb * R2 * es] = v[kb];
        }
    }

    __device__ static double2 output(const double2 *line, int es, int k, const double2 *twN) {
        const int kb = k % R1, ka = k / R1;
        const double2 *p = line + R2 * kb * es;
        double2 s = p[0];
        if (R2 == 3) {
            // exact radix-3 weights: w3^{ka} for ka = 0, 1, 2
            const double2 a = p[es], b = p[2 * es];
            if (ka == 0) return cadd(s, cadd(a, b));
            const double2 t1 = cadd(a, b), t2 = csub(a, b);
            const double2 m = make_double2(s.x - 0.5 * t1.x, s.y - 0.5 * t1.y);
            const double2 is = make_double2(-kS60 * t2.y, kS60 * t2.x);
            return ka == 1 ? cadd(m, is) : csub(m, is);
        }
#pragma unroll
        for (int za = 1; za < R2; ++za) s = cadd(s, cmul(twN[((za * ka) % R2) * R1], p[za * es]));
        return s;
    }
};

__device__ inline int wrap(int m, int n) { return m < 0 ? m + n : m; }

}  // namespace

// ------------------------------------------------------------------ pair kernel

// LDS row strides: plane row padded so that stride == R2 (mod 16) when R2 < 16
template <int Z1, int Z2>
__host__ __device__ constexpr int plane_stride() {
    return Z1 * Z2 + ((Z2 % 16) - (Z1 * Z2) % 16 + 16) % 16;
}

// ------------------------------------------------------------------ two-pass pair transform
//
// Pass A (k_pair_yz): one workgroup per (k, c, block of x-planes); for every x of
// the block and every valence band v: product conj(u_v) u_c on the plane, z FFT
// pruned to the dielectric box, y FFT pruned likewise; the bey x bez values are
// written to T[t][x][iy][iz] (no per-pair accumulators).  Concurrent
// workgroups (same k and x-block, consecutive c) share the u_v planes in L2.
// Pass B (k_pair_x): one workgroup per pair; T[t] is staged through LDS a few
// planes at a time and every sphere point accumulates w_{n1}^{mx x} T[x][iy][iz].
template <int Z1, int Z2, int NT, int LC>
__global__ __launch_bounds__(NT) void k_pair_yz(const double2 *__restrict__ gv, const double2 *__restrict__ gc,
                                                int nkb, int nv, int nc, int c0, int ncb, int n1,
                                                const double2 *__restrict__ tw2g, const double2 *__restrict__ tw3g,
                                                int rey, int rez, int xblk, double2 *__restrict__ T) {
    constexpr int n3 = Z1 * Z2, n2 = n3;
    constexpr int PS = plane_stride<Z1, Z2>();
    constexpr int CH = LC * n3;
    constexpr int PER = (CH + NT - 1) / NT;
    constexpr int NCHUNK = (n2 + LC - 1) / LC;
    const int bez = 2 * rez + 1, bey = 2 * rey + 1;
    const int QS = bez;
    const int nbox = bey * bez;
    const unsigned mdiv = (1u << 20) / (unsigned)bez + 1u;
    extern __shared__ double2 lds[];
    double2 *tw2 = lds, *tw3 = tw2 + n2;
    double2 *P = tw3 + n3;     // [LC][PS]
    double2 *Q = P + LC * PS;  // [n2][QS]
    for (int i = threadIdx.x; i < n2; i += NT) tw2[i] = tw2g[i];
    for (int i = threadIdx.x; i < n3; i += NT) tw3[i] = tw3g[i];

    // c-batch [c0, c0 + ncb) of the k-batch; T is indexed by the batch-local
    // pair (k * nv + v) * ncb + cl
    const int nxb = (n1 + xblk - 1) / xblk;
    const int cl = blockIdx.x % ncb;
    const int c = c0 + cl;
    const int rest = blockIdx.x / ncb;
    const int xb = rest % nxb;
    const int k = rest / nxb;
    const int x0 = xb * xblk, x1 = min(n1, x0 + xblk);
    const size_t N = (size_t)n1 * n2 * n3;
    const double2 *uc = gc + (size_t)(k * nc + c) * N;
    const double2 *uvk = gv + (size_t)k * nv * N;

    double2 fv[PER], fc[PER];
    auto fetch = [&](int x, int v, int ci) {
        const int y0 = ci * LC;
        const int Lc = min(LC, n2 - y0);
        const size_t off = ((size_t)x * n2 + y0) * n3;
        const double2 *pv = uvk + (size_t)v * N + off;
        const double2 *pc = uc + off;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int e = threadIdx.x + j * NT;
            if (e < Lc * n3) {
                fv[j] = pv[e];
                fc[j] = pc[e];
            }
        }
    };
    __syncthreads();
    for (int x = x0; x < x1; ++x) {
#pragma unroll 1
        for (int v = 0; v < nv; ++v) {
#pragma unroll 1
            for (int ci = 0; ci < NCHUNK; ++ci) {
                const int y0 = ci * LC;
                const int Lc = min(LC, n2 - y0);
                fetch(x, v, ci);
#pragma unroll
                for (int j = 0; j < PER; ++j) {
                    const int e = threadIdx.x + j * NT;
                    if (e < Lc * n3) {
                        const int yy = e / n3, z = e - yy * n3;
                        P[yy * PS + z] = cconjmul(fv[j], fc[j]);
                    }
                }
                __syncthreads();
                LineFFT<Z1, Z2>::stage1(P, Lc, PS, 1, tw3);
                __syncthreads();
                for (int e = threadIdx.x; e < Lc * bez; e += NT) {
                    const int yy = (int)(((unsigned long long)e * mdiv) >> 20), iz = e - yy * bez;
                    Q[(y0 + yy) * QS + iz] = LineFFT<Z1, Z2>::output(P + yy * PS, 1, wrap(iz - rez, n3), tw3);
                }
                __syncthreads();
            }
            LineFFT<Z1, Z2>::stage1(Q, bez, 1, QS, tw2);
            __syncthreads();
            const long long tl = ((long long)k * nv + v) * ncb + cl;
            double2 *o = T + ((size_t)tl * n1 + x) * nbox;
            for (int e = threadIdx.x; e < nbox; e += NT) {
                const int iy = (int)(((unsigned long long)e * mdiv) >> 20), iz = e - iy * bez;
                o[e] = LineFFT<Z1, Z2>::output(Q + iz, QS, wrap(iy - rey, n2), tw2);
            }
            __syncthreads();
        }
    }
}

// Pass A for y and z lengths N <= 32, one wavefront per workgroup and no
// workgroup barriers.  Workgroup = (k, c, block of x-planes); it loops over
// the valence bands and takes G x-planes of one pair per round:
//   y: lane (plane p, z) reads the y-line of u_v and u_c at that z (at fixed y
//      the lanes of one plane read N consecutive elements: coalesced),
//      forms conj(u_v) u_c, does the whole N-point DFT in registers and
//      stores the bey outputs of the dielectric box to Q[p][iy][z] in LDS;
//   z: lane (plane p, iy) reads row Q[p][iy][.], does the N-point DFT in
//      registers and writes the bez box outputs to T[t][x][iz][iy] (iy
//      fastest, so the stores of a wave are contiguous runs).
// The Q row stride N + 1 is odd in 16-byte units, so both the column writes
// and the row reads are free of LDS bank conflicts.
template <int N, int G, int MINW>
__global__ __launch_bounds__(64, MINW) void k_pair_yzr(const double2 *__restrict__ gv, const double2 *__restrict__ gc,
                                                 int nv, int nc, int c0, int ncb, int n1, int rey, int rez, int xblk,
                                                 double2 *__restrict__ T) {
    constexpr int QS = N + 1;
    extern __shared__ double2 Q[];  // [G][bey][QS]
    const int lane = threadIdx.x;
    const int bey = 2 * rey + 1, bez = 2 * rez + 1, nbox = bey * bez;
    const int nxb = (n1 + xblk - 1) / xblk;
    const int cl = blockIdx.x % ncb;
    const int rest = blockIdx.x / ncb;
    const int xb = rest % nxb;
    const int k = rest / nxb;
    const int x0 = xb * xblk, x1 = min(n1, x0 + xblk);
    const size_t plane = (size_t)N * N;
    const size_t NB = (size_t)n1 * plane;
    const double2 *uc = gc + (size_t)(k * nc + c0 + cl) * NB;
    const double2 *uvk = gv + (size_t)k * nv * NB;
    const int py = lane / N, zl = lane - py * N;   // y-stage role
    const int pz = lane / bey, iy = lane - pz * bey;  // z-stage role
#pragma unroll 1
    for (int v = 0; v < nv; ++v) {
        const long long tl = ((long long)k * nv + v) * ncb + cl;
#pragma unroll 1
        for (int xg = x0; xg < x1; xg += G) {
            {
                const int x = xg + py;
                const bool act = py < G && x < x1;
                double2 d[N];
                if (act) {
                    // the u_c line first, then u_v in blocks of 8 with one block in
                    // flight ahead of the products (bounded register footprint)
                    const double2 *a = uvk + v * NB + x * plane + zl;
                    const double2 *b = uc + x * plane + zl;
#pragma unroll
                    for (int y = 0; y < N; ++y) d[y] = b[y * N];
                    double2 ra[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) ra[i] = a[i * N];
#pragma unroll
                    for (int y0 = 0; y0 < N; y0 += 8) {
                        double2 na[8];
                        if (y0 + 8 < N) {
#pragma unroll
                            for (int i = 0; i < 8; ++i) na[i] = a[(y0 + 8 + i) * N];
                        }
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int i = 0; i < 8; ++i) d[y0 + i] = cconjmul(ra[i], d[y0 + i]);
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int i = 0; i < 8; ++i) ra[i] = na[i];
                    }
                } else {
#pragma unroll
                    for (int y = 0; y < N; ++y) d[y] = make_double2(0.0, 0.0);
                }
                LineDFT<N>::run(d);
                if (act) {
                    double2 *q = Q + py * bey * QS + zl;
#pragma unroll
                    for (int ky = 0; ky < N; ++ky) {
                        const int m = ky <= N / 2 ? ky : ky - N;
                        if (m >= -rey && m <= rey) q[(m + rey) * QS] = d[ky];
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            {
                const int x = xg + pz;
                const bool act = pz < G && x < x1;
                double2 e[N];
                if (act) {
                    const double2 *q = Q + (pz * bey + iy) * QS;
#pragma unroll
                    for (int z = 0; z < N; ++z) e[z] = q[z];
                } else {
#pragma unroll
                    for (int z = 0; z < N; ++z) e[z] = make_double2(0.0, 0.0);
                }
                LineDFT<N>::run(e);
                if (act) {
                    double2 *o = T + ((size_t)tl * n1 + x) * nbox + iy;
#pragma unroll
                    for (int kz = 0; kz < N; ++kz) {
                        const int m = kz <= N / 2 ? kz : kz - N;
                        if (m >= -rez && m <= rez) o[(m + rez) * bey] = e[kz];
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
}

// Pass B.  T: [npairs][n1][nbox], box point (iy, iz) at iy * ys + iz * zs;
// sphere points in (mx, my, mz) order (ge_code2),
// written back in the original order (ge_out).  XS planes staged per round.
template <int ACC, int NT, int XS>
__global__ __launch_bounds__(NT) void k_pair_x(const double2 *__restrict__ T, int n1, int nbox, int bez,
                                               const double2 *__restrict__ tw1g, const int *__restrict__ ge_code,
                                               const int *__restrict__ ge_out, int ng, double inv_n,
                                               double2 *__restrict__ M, int nv, int nc, int c0, int ncb,
                                               long long m_row0, int ys, int zs) {
    extern __shared__ double2 lds[];
    double2 *tw1 = lds, *Ts = tw1 + n1;  // [XS][nbox]
    for (int i = threadIdx.x; i < n1; i += NT) tw1[i] = tw1g[i];
    const long long t = blockIdx.x;
    const double2 *Tt = T + (size_t)t * n1 * nbox;
    int slot[ACC], ph[ACC], mxs[ACC];
    double2 acc[ACC];
#pragma unroll
    for (int i = 0; i < ACC; ++i) {
        const int g = threadIdx.x + i * NT;
        const int cd = g < ng ? ge_code[g] : -1;
        slot[i] = cd >= 0 ? ((cd >> 8) & 0xff) * ys + (cd >> 16) * zs : -1;
        mxs[i] = cd >= 0 ? (cd & 0xff) : 0;
        ph[i] = 0;
        acc[i] = make_double2(0.0, 0.0);
    }
    for (int xs = 0; xs < n1; xs += XS) {
        const int nx = min(XS, n1 - xs);
        __syncthreads();
        {
            // eight loads per thread in flight before their LDS stores
            const int cnt = nx * nbox;
            const double2 *src = Tt + (size_t)xs * nbox;
            for (int e0 = 0; e0 < cnt; e0 += 8 * NT) {
                double2 v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + u * NT + threadIdx.x;
                    v[u] = e < cnt ? src[e] : make_double2(0.0, 0.0);
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int e = e0 + u * NT + threadIdx.x;
                    if (e < cnt) Ts[e] = v[u];
                }
            }
        }
        __syncthreads();
        for (int xx = 0; xx < nx; ++xx) {
#pragma unroll
            for (int i = 0; i < ACC; ++i) {
                if (slot[i] >= 0) {
                    acc[i] = cadd(acc[i], cmul(tw1[ph[i]], Ts[xx * nbox + slot[i]]));
                    ph[i] += mxs[i];
                    if (ph[i] >= n1) ph[i] -= n1;
                }
            }
        }
    }
    const long long cl = t % ncb, kv = t / ncb;  // kv = k * nv + v within the k-batch
    double2 *out = M + (size_t)(m_row0 + kv * nc + c0 + cl) * ng;
#pragma unroll
    for (int i = 0; i < ACC; ++i) {
        const int g = threadIdx.x + i * NT;
        if (g < ng) out[ge_out[g]] = cscale(acc[i], inv_n);
    }
}

// ------------------------------------------------------------------ band kernel

// One workgroup per band.  Box sizes: bwy x bwz around 0 (Rwy, Rwz).  The z
// expansion thread owns z = tid % n3 and rows y = tid / n3 + j * (NT / n3).
template <int BW, int NT>
__global__ __launch_bounds__(NT) void k_band_to_real2(const double2 *__restrict__ C, int ngw, int n1, int n2, int n3,
                                                      const double2 *__restrict__ tw1g,
                                                      const double2 *__restrict__ tw2g,
                                                      const double2 *__restrict__ tw3g, SphereMaps sm, int rwy,
                                                      double2 *__restrict__ grids) {
    const int bwy = 2 * rwy + 1, bwz = sm.bwz, rwz = sm.rwz;
    extern __shared__ double2 lds[];
    double2 *tw1 = lds, *tw2 = tw1 + n1;
    double2 *Qb = tw2 + n2;       // [bwy][bwz]   x-stick sums
    double2 *S = Qb + bwy * bwz;  // [n2][bwz]    after the y expansion
    for (int i = threadIdx.x; i < n1; i += NT) tw1[i] = tw1g[i];
    for (int i = threadIdx.x; i < n2; i += NT) tw2[i] = tw2g[i];

    // per-thread z twiddles exp(+2 pi i mz z / n3), mz = iz - rwz
    const int zt = threadIdx.x % n3;
    const int rows_step = NT / n3;
    const int y_start = threadIdx.x / n3;
    const bool active = y_start < rows_step;
    double2 tz[BW];
#pragma unroll
    for (int iz = 0; iz < BW; ++iz) {
        tz[iz] = make_double2(0.0, 0.0);
        if (iz < bwz) {
            const int mz = iz - rwz;
            int idx = (mz * zt) % n3;
            if (idx < 0) idx += n3;
            tz[iz] = tw3g[idx];
        }
    }
    const size_t N = (size_t)n1 * n2 * n3;
    const double2 *cb = C + (size_t)blockIdx.x * ngw;
    double2 *out = grids + (size_t)blockIdx.x * N;
    __syncthreads();

    for (int x = 0; x < n1; ++x) {
        // x stage: stick sums into the (my, mz) box; untouched box cells are zero
        for (int e = threadIdx.x; e < bwy * bwz; e += NT) Qb[e] = make_double2(0.0, 0.0);
        __syncthreads();
        for (int s = threadIdx.x; s < sm.nstick; s += NT) {
            double2 a = make_double2(0.0, 0.0);
            for (int i = sm.stick_start[s]; i < sm.stick_start[s + 1]; ++i) {
                int idx = sm.stick_mx[i] * x;
                idx -= (idx / n1) * n1;
                a = cadd(a, cmul(tw1[idx], cb[sm.stick_g[i]]));
            }
            const int yz = sm.stick_yz2[s];
            Qb[(yz & 0xffff) * bwz + (yz >> 16)] = a;
        }
        __syncthreads();
        // y stage: S[y][iz] = sum_iy w^{my y} Qb[iy][iz]
        for (int e = threadIdx.x; e < n2 * bwz; e += NT) {
            const int y = e / bwz, iz = e - y * bwz;
            int idx = (-rwy * y) % n2;
            if (idx < 0) idx += n2;
            double2 a = make_double2(0.0, 0.0);
            for (int iy = 0; iy < bwy; ++iy) {
                a = cadd(a, cmul(tw2[idx], Qb[iy * bwz + iz]));
                idx += y;
                if (idx >= n2) idx -= n2;
            }
            S[e] = a;
        }
        __syncthreads();
        // z stage: u[y][z] = sum_iz w^{mz z} S[y][iz]
        if (active) {
            double2 *o = out + (size_t)x * n2 * n3;
            for (int y = y_start; y < n2; y += rows_step) {
                double2 a = make_double2(0.0, 0.0);
#pragma unroll
                for (int iz = 0; iz < BW; ++iz)
                    if (iz < bwz) a = cadd(a, cmul(tz[iz], S[y * bwz + iz]));
                o[y * n3 + zt] = a;
            }
        }
        __syncthreads();
    }
}


// Band kernel for fast z lengths: x stage summed per stick (stick metadata in
// registers, coefficients gathered once per band into LDS in stick order when
// they fit), y stage as a direct sum over the box rows, z stage as the
// register radix-R1 FFT of the zero-padded lines (all n3 outputs kept),
// written with coalesced stores.
template <int Z1, int Z2, int NT, int SPT>
__global__ __launch_bounds__(NT) void k_band_to_real3(const double2 *__restrict__ C, int ngw, int n1, int n2,
                                                      const double2 *__restrict__ tw1g,
                                                      const double2 *__restrict__ tw2g,
                                                      const double2 *__restrict__ tw3g, SphereMaps sm, int rwy, int lc,
                                                      int cache_c, double2 *__restrict__ grids) {
    constexpr int n3 = Z1 * Z2;
    constexpr int PS = plane_stride<Z1, Z2>();
    const int bwy = 2 * rwy + 1, bwz = sm.bwz, rwz = sm.rwz;
    extern __shared__ double2 lds[];
    double2 *tw1 = lds, *tw2 = tw1 + n1, *tw3 = tw2 + n2;
    double2 *Qb = tw3 + n3;       // [bwy][bwz]  x-stick sums
    double2 *S = Qb + bwy * bwz;  // [n2][bwz]   after the y expansion
    double2 *Z = S + n2 * bwz;    // [lc][PS]    z lines
    double2 *Cs = Z + lc * PS;    // [ngw]       coefficients in stick order (if cached)
    int *mxl = reinterpret_cast<int *>(Cs + (cache_c ? ngw : 0));  // [ngw] mx mod n1 in stick order
    for (int i = threadIdx.x; i < n1; i += NT) tw1[i] = tw1g[i];
    for (int i = threadIdx.x; i < n2; i += NT) tw2[i] = tw2g[i];
    for (int i = threadIdx.x; i < n3; i += NT) tw3[i] = tw3g[i];
    const double2 *cg = C + (size_t)blockIdx.x * ngw;
    for (int i = threadIdx.x; i < ngw; i += NT) {
        if (cache_c) Cs[i] = cg[sm.stick_g[i]];
        mxl[i] = sm.stick_mx[i];
    }
    int s0[SPT], s1[SPT], syz[SPT];
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
        const int s = threadIdx.x + j * NT;
        s0[j] = s1[j] = 0;
        syz[j] = -1;
        if (s < sm.nstick) {
            s0[j] = sm.stick_start[s];
            s1[j] = sm.stick_start[s + 1];
            syz[j] = sm.stick_yz2[s];
        }
    }
    // (m * x) mod n1 as m*x - n1 * ((m*x*md) >> 20), exact for m*x < n1^2 <= 2^14
    const unsigned md = (1u << 20) / (unsigned)n1 + 1u;
    const size_t N = (size_t)n1 * n2 * n3;
    double2 *out = grids + (size_t)blockIdx.x * N;
    __syncthreads();

    for (int x = 0; x < n1; ++x) {
        for (int e = threadIdx.x; e < bwy * bwz; e += NT) Qb[e] = make_double2(0.0, 0.0);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < SPT; ++j) {
            if (syz[j] < 0) continue;
            double2 a = make_double2(0.0, 0.0);
            for (int i = s0[j]; i < s1[j]; ++i) {
                const unsigned prod = (unsigned)(mxl[i] * x);
                const int idx = (int)(prod - (unsigned)n1 * (unsigned)(((unsigned long long)prod * md) >> 20));
                const double2 cv = cache_c ? Cs[i] : cg[sm.stick_g[i]];
                a = cadd(a, cmul(tw1[idx], cv));
            }
            Qb[(syz[j] & 0xffff) * bwz + (syz[j] >> 16)] = a;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < n2 * bwz; e += NT) {
            const int y = e / bwz, iz = e - y * bwz;
            int idx = (-rwy * y) % n2;
            if (idx < 0) idx += n2;
            double2 a = make_double2(0.0, 0.0);
            for (int iy = 0; iy < bwy; ++iy) {
                a = cadd(a, cmul(tw2[idx], Qb[iy * bwz + iz]));
                idx += y;
                if (idx >= n2) idx -= n2;
            }
            S[e] = a;
        }
        __syncthreads();
        for (int y0 = 0; y0 < n2; y0 += lc) {
            const int L = min(lc, n2 - y0);
            for (int e = threadIdx.x; e < L * n3; e += NT) {
                const int yy = e / n3, z = e - yy * n3;
                const int mz = z <= rwz ? z : z - n3;
                Z[yy * PS + z] = (mz >= -rwz && mz <= rwz) ? S[(y0 + yy) * bwz + mz + rwz] : make_double2(0.0, 0.0);
            }
            __syncthreads();
            LineFFT<Z1, Z2>::stage1(Z, L, PS, 1, tw3);
            __syncthreads();
            double2 *o = out + ((size_t)x * n2 + y0) * n3;
            for (int e = threadIdx.x; e < L * n3; e += NT) {
                const int yy = e / n3, z = e - yy * n3;
                o[e] = LineFFT<Z1, Z2>::output(Z + yy * PS, 1, z, tw3);
            }
            __syncthreads();
        }
    }
}

// Two-pass band transform for cubic boxes of side N = 16, 24 or 32 (the
// inverse direction of the pair passes).
// Pass X (k_band_x): lane = (band, box cell (iy, iz)).  The cell's x-stick
// holds consecutive mx; each is placed at register mx mod N (zero elsewhere)
// and the whole N-point DFT along x runs in registers.  The N results go to
// W[band][x][iz][iy] (iy fastest; cells without a stick get zeros).
template <int N>
__global__ __launch_bounds__(256) void k_band_x(const double2 *__restrict__ C, int ngw, SphereMaps sm,
                                                double2 *__restrict__ W) {
    const int cell = blockIdx.x * 256 + threadIdx.x;
    const int band = blockIdx.y;
    if (cell >= sm.ncell) return;
    const int s = sm.cell_stick[cell];
    int base = 0, cnt = 0, lo = 0;
    if (s >= 0) {
        base = sm.stick_start[s];
        cnt = sm.stick_start[s + 1] - base;
        lo = sm.st_lo[s];
    }
    const double2 *cb = C + (size_t)band * ngw;
    // all sphere indices of the stick first, then all coefficients, so each
    // round of loads is in flight together
    int gi[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int j = (k <= N / 2 ? k : k - N) - lo;
        gi[k] = (j >= 0 && j < cnt) ? sm.st_gs[base + j] : -1;
    }
    double2 d[N];
#pragma unroll
    for (int k = 0; k < N; ++k) d[k] = gi[k] >= 0 ? cb[gi[k]] : make_double2(0.0, 0.0);
    LineDFT<N>::run(d);
    double2 *o = W + (size_t)band * N * sm.ncell + cell;
#pragma unroll
    for (int x = 0; x < N; ++x) o[(size_t)x * sm.ncell] = d[x];
}

// Pass YZ (k_band_yz): one wavefront per workgroup = (band, block of
// x-planes), G planes per round.
//   z: lane (plane p, iy) reads the bwz values W[band][x][.][iy] (coalesced
//      over iy), places them at registers mz mod N, does the N-point DFT and
//      stores the row to Q[p][iy][.] in LDS;
//   y: lane (plane p, z) reads the bwy values Q[p][.][z], places them at my
//      mod N, does the N-point DFT and stores u[band][x][y][z] for all y
//      (coalesced over z).
template <int N, int G>
__global__ __launch_bounds__(64) void k_band_yz(const double2 *__restrict__ W, int ncell, int rwy, int rwz, int xblk,
                                                double2 *__restrict__ grids) {
    constexpr int QS = N + 1;
    extern __shared__ double2 Q[];  // [G][bwy][QS]
    const int lane = threadIdx.x;
    const int bwy = 2 * rwy + 1;
    const int nxb = (N + xblk - 1) / xblk;
    const int band = blockIdx.x / nxb;
    const int xb = blockIdx.x - band * nxb;
    const int x0 = xb * xblk, x1 = min(N, x0 + xblk);
    const double2 *wb = W + (size_t)band * N * ncell;
    double2 *ob = grids + (size_t)band * N * N * N;
    const int pz = lane / bwy, iy = lane - pz * bwy;  // z-stage role
    const int py = lane / N, zl = lane - py * N;      // y-stage role
#pragma unroll 1
    for (int xg = x0; xg < x1; xg += G) {
        {
            const int x = xg + pz;
            const bool act = pz < G && x < x1;
            const double2 *w = wb + (size_t)x * ncell + iy;
            double2 d[N];
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const int m = k <= N / 2 ? k : k - N;
                d[k] = (act && m >= -rwz && m <= rwz) ? w[(m + rwz) * bwy] : make_double2(0.0, 0.0);
            }
            LineDFT<N>::run(d);
            if (act) {
                double2 *q = Q + (pz * bwy + iy) * QS;
#pragma unroll
                for (int z = 0; z < N; ++z) q[z] = d[z];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        {
            const int x = xg + py;
            const bool act = py < G && x < x1;
            const double2 *q = Q + py * bwy * QS + zl;
            double2 e[N];
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const int m = k <= N / 2 ? k : k - N;
                e[k] = (act && m >= -rwy && m <= rwy) ? q[(m + rwy) * QS] : make_double2(0.0, 0.0);
            }
            LineDFT<N>::run(e);
            if (act) {
                double2 *o = ob + (size_t)x * N * N + zl;
#pragma unroll
                for (int y = 0; y < N; ++y) o[y * N] = e[y];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// ------------------------------------------------------------------ host side

namespace {
template <int Z1, int Z2, int LC>
int launch_pair_yz_t(const double2 *gv, const double2 *gc, int nkb, int nv, int nc, int c0, int ncb,
                     const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz, int rey, int rez, double2 *T,
                     hipStream_t st) {
    constexpr int n = Z1 * Z2;
    constexpr int PS = plane_stride<Z1, Z2>();
    const int bez = 2 * rez + 1;
    const size_t lds = sizeof(double2) * ((size_t)n + n + (size_t)LC * PS + (size_t)n * bez);
    if (lds > 150 * 1024) return BGW_ERR_UNSUPPORTED;
    auto kern = k_pair_yz<Z1, Z2, 256, LC>;
    BGW_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int n1 = px.n;
    const int xblk = std::max(1, std::min(n1, 8));
    const int nxb = (n1 + xblk - 1) / xblk;
    const long long grid = (long long)nkb * nxb * ncb;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), lds, st, gv, gc, nkb, nv, nc, c0, ncb, n1, py.tw, pz.tw,
                       rey, rez, xblk, T);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

template <int ACC>
int launch_pair_x_t(const double2 *T, long long npairs, const AxisPlan &px, int nbox, int bez, const int *ge_code2,
                    const int *ge_out, int ng, double inv_n, double2 *M, int nv, int nc, int c0, int ncb,
                    long long row0, int ys, int zs, hipStream_t st) {
    constexpr int XS = 8;
    const size_t lds = sizeof(double2) * ((size_t)px.n + (size_t)XS * nbox);
    if (lds > 150 * 1024) return BGW_ERR_UNSUPPORTED;
    auto kern = k_pair_x<ACC, 256, XS>;
    BGW_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kern, dim3((unsigned)npairs), dim3(256), lds, st, T, px.n, nbox, bez, px.tw, ge_code2, ge_out,
                       ng, inv_n, M, nv, nc, c0, ncb, row0, ys, zs);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

template <int N, int G, int MINW>
int launch_pair_yzr_t(const double2 *gv, const double2 *gc, int nkb, int nv, int nc, int c0, int ncb, int n1,
                      int rey, int rez, double2 *T, hipStream_t st) {
    const int bey = 2 * rey + 1;
    if (bey > N || 2 * rez + 1 > N || G * bey > 64) return BGW_ERR_UNSUPPORTED;
    const size_t lds = sizeof(double2) * (size_t)G * bey * (N + 1);
    auto kern = k_pair_yzr<N, G, MINW>;
    BGW_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int xblk = std::max(G, std::min(n1, 4 * G));
    const int nxb = (n1 + xblk - 1) / xblk;
    const long long grid = (long long)nkb * nxb * ncb;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64), lds, st, gv, gc, nv, nc, c0, ncb, n1, rey, rez, xblk, T);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

template <int Z1, int Z2, int LCF>
int launch_pair_yz_sel(const double2 *gv, const double2 *gc, int nkb, int nv, int nc, int c0, int ncb,
                       const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz, int rey, int rez, double2 *T,
                       hipStream_t st) {
    return launch_pair_yz_t<Z1, Z2, LCF>(gv, gc, nkb, nv, nc, c0, ncb, px, py, pz, rey, rez, T, st);
}
}  // namespace

size_t pair_yz_bytes_per_pair(int n1, int rey, int rez) {
    return sizeof(double2) * (size_t)n1 * (size_t)(2 * rey + 1) * (2 * rez + 1);
}

bool pair_two_pass_supported(const AxisPlan &py, const AxisPlan &pz) {
    if (py.n != pz.n) return false;
    switch (pz.n) {
        case 16: case 24: case 32: case 48: case 64: case 96: case 128: return true;
        default: return false;
    }
}

// Pass A for fast sizes (y and z lengths equal, 16 r or 24).
int launch_pair_yz(const double2 *gv, const double2 *gc, int nkb, int nv, int nc, int c0, int ncb,
                   const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz, int rey, int rez, double2 *T,
                   hipStream_t st) {
    if (py.n != pz.n) return BGW_ERR_UNSUPPORTED;
    switch (pz.n) {
        case 16: return launch_pair_yz_sel<16, 1, 16>(gv, gc, nkb, nv, nc, c0, ncb, px, py, pz, rey, rez, T, st);
        case 24: return launch_pair_yz_sel<8, 3, 24>(gv, gc, nkb, nv, nc, c0, ncb, px, py, pz, rey, rez, T, st);
        case 32: return launch_pair_yz_sel<16, 2, 32>(gv, gc, nkb, nv, nc, c0, ncb, px, py, pz, rey, rez, T, st);
        case 48: return launch_pair_yz_sel<16, 3, 48>(gv, gc, nkb, nv, nc, c0, ncb, px, py, pz, rey, rez, T, st);
        case 64: return launch_pair_yz_sel<16, 4, 32>(gv, gc, nkb, nv, nc, c0, ncb, px, py, pz, rey, rez, T, st);
        case 96: return launch_pair_yz_sel<16, 6, 16>(gv, gc, nkb, nv, nc, c0, ncb, px, py, pz, rey, rez, T, st);
        case 128: return launch_pair_yz_sel<16, 8, 16>(gv, gc, nkb, nv, nc, c0, ncb, px, py, pz, rey, rez, T, st);
        default: return BGW_ERR_UNSUPPORTED;
    }
}

// Pass A with one lane per line (y and z lengths 16, 24 or 32).  T then holds
// each x-plane's box with iy fastest.  BGW_ERR_UNSUPPORTED when it does not apply.
int launch_pair_yzr(const double2 *gv, const double2 *gc, int nkb, int nv, int nc, int c0, int ncb,
                    const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz, int rey, int rez, double2 *T,
                    hipStream_t st) {
    if (py.n != pz.n) return BGW_ERR_UNSUPPORTED;
    switch (pz.n) {
        case 16: return launch_pair_yzr_t<16, 4, 1>(gv, gc, nkb, nv, nc, c0, ncb, px.n, rey, rez, T, st);
        case 24: return launch_pair_yzr_t<24, 2, 1>(gv, gc, nkb, nv, nc, c0, ncb, px.n, rey, rez, T, st);
        case 32: return launch_pair_yzr_t<32, 2, 1>(gv, gc, nkb, nv, nc, c0, ncb, px.n, rey, rez, T, st);
        default: return BGW_ERR_UNSUPPORTED;
    }
}

// yfast: T box points stored iy fastest (lane-per-line pass A), else iz fastest.
int launch_pair_x(const double2 *T, long long npairs, const AxisPlan &px, int rey, int rez, const int *ge_code2,
                  const int *ge_out, int ng, double2 *M, int nv, int nc, int c0, int ncb, long long row0, size_t N,
                  bool yfast, hipStream_t st) {
    const int bez = 2 * rez + 1, bey = 2 * rey + 1, nbox = bey * bez;
    const int ys = yfast ? 1 : bez, zs = yfast ? bey : 1;
    const double inv_n = 1.0 / (double)N;
    const int per = (ng + 255) / 256;
#define BGW_PX(A)                                                                                               \
    if (per <= A)                                                                                               \
        return launch_pair_x_t<A>(T, npairs, px, nbox, bez, ge_code2, ge_out, ng, inv_n, M, nv, nc, c0, ncb, row0, \
                                  ys, zs, st);
    BGW_PX(1)
    BGW_PX(2)
    BGW_PX(4)
    BGW_PX(6)
    BGW_PX(8)
    BGW_PX(12)
    BGW_PX(16)
    BGW_PX(24)
    BGW_PX(32)
#undef BGW_PX
    return BGW_ERR_UNSUPPORTED;
}

namespace {
template <int Z1, int Z2>
int launch_band3_t(const double2 *C, int nbands, int ngw, const AxisPlan &px, const AxisPlan &py,
                   const AxisPlan &pz, const SphereMaps &sm, int rwy, double2 *grids, hipStream_t st) {
    constexpr int PS = plane_stride<Z1, Z2>();
    if (sm.nstick > 4 * 256 || px.n > 128) return BGW_ERR_UNSUPPORTED;
    const int bwy = 2 * rwy + 1;
    const size_t fixed = sizeof(double2) * ((size_t)px.n + py.n + pz.n + (size_t)bwy * sm.bwz + (size_t)py.n * sm.bwz) +
                         sizeof(int) * (size_t)ngw;
    // aim at two workgroups per CU (<= 78 KB) with the coefficients cached
    int cache_c = 1;
    int lc = py.n;
    auto bytes = [&](int l, int cc) { return fixed + sizeof(double2) * ((size_t)l * PS + (cc ? (size_t)ngw : 0)); };
    while (lc > 8 && bytes(lc, 1) > 78 * 1024) lc = (lc + 1) / 2;
    if (bytes(lc, 1) > 78 * 1024) {
        cache_c = 0;
        lc = py.n;
        while (lc > 4 && bytes(lc, 0) > 78 * 1024) lc = (lc + 1) / 2;
    }
    const size_t lds = bytes(lc, cache_c);
    if (lds > 150 * 1024) return BGW_ERR_UNSUPPORTED;
#define BGW_B3(SPT)                                                                                              \
    {                                                                                                            \
        auto kern = k_band_to_real3<Z1, Z2, 256, SPT>;                                                           \
        BGW_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));  \
        hipLaunchKernelGGL(kern, dim3(nbands), dim3(256), lds, st, C, ngw, px.n, py.n, px.tw, py.tw, pz.tw, sm, \
                           rwy, lc, cache_c, grids);                                                              \
    }
    if (sm.nstick <= 256)
        BGW_B3(1)
    else if (sm.nstick <= 512)
        BGW_B3(2)
    else
        BGW_B3(4)
#undef BGW_B3
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}
}  // namespace

int launch_band_to_real2(const double2 *C, int nbands, int ngw, const AxisPlan &px, const AxisPlan &py,
                         const AxisPlan &pz, const SphereMaps &sm, int rwy, double2 *grids, hipStream_t st) {
    if (nbands <= 0) return BGW_OK;
    switch (pz.n) {
        case 16: return launch_band3_t<16, 1>(C, nbands, ngw, px, py, pz, sm, rwy, grids, st);
        case 24: return launch_band3_t<8, 3>(C, nbands, ngw, px, py, pz, sm, rwy, grids, st);
        case 32: return launch_band3_t<16, 2>(C, nbands, ngw, px, py, pz, sm, rwy, grids, st);
        case 48: return launch_band3_t<16, 3>(C, nbands, ngw, px, py, pz, sm, rwy, grids, st);
        case 64: return launch_band3_t<16, 4>(C, nbands, ngw, px, py, pz, sm, rwy, grids, st);
        case 96: return launch_band3_t<16, 6>(C, nbands, ngw, px, py, pz, sm, rwy, grids, st);
        case 128: return launch_band3_t<16, 8>(C, nbands, ngw, px, py, pz, sm, rwy, grids, st);
        default: break;
    }
    const int bwy = 2 * rwy + 1;
    if (sm.bwz > 32 || pz.n > 256) return BGW_ERR_UNSUPPORTED;
    const size_t lds = sizeof(double2) * ((size_t)px.n + py.n + (size_t)bwy * sm.bwz + (size_t)py.n * sm.bwz);
    if (lds > 150 * 1024) return BGW_ERR_UNSUPPORTED;
    if (sm.bwz <= 16) {
        auto kern = k_band_to_real2<16, 256>;
        BGW_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kern, dim3(nbands), dim3(256), lds, st, C, ngw, px.n, py.n, pz.n, px.tw, py.tw, pz.tw, sm,
                           rwy, grids);
    } else {
        auto kern = k_band_to_real2<32, 256>;
        BGW_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kern, dim3(nbands), dim3(256), lds, st, C, ngw, px.n, py.n, pz.n, px.tw, py.tw, pz.tw, sm,
                           rwy, grids);
    }
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

// Band transform by the two lane-per-line passes when the box is a cube of
// side 16, 24 or 32 and every x-stick is contiguous in mx; W must hold
// sizeof(double2) * nbands * N * ncell bytes.  BGW_ERR_UNSUPPORTED (nothing
// launched) otherwise.
size_t band_lines_bytes(const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz, const SphereMaps &sm,
                        int nbands) {
    return sizeof(double2) * (size_t)nbands * px.n * sm.ncell;
}

bool band_lines_supported(const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz, const SphereMaps &sm) {
    if (px.n != py.n || py.n != pz.n || !sm.sticks_contiguous) return false;
    const int n = pz.n, G = n == 16 ? 4 : 2;
    return (n == 16 || n == 24 || n == 32) && G * (2 * sm.rwy + 1) <= 64;
}

namespace {
template <int N, int G>
int launch_band_lines_t(const double2 *C, int nbands, int ngw, const SphereMaps &sm, double2 *W, double2 *grids,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_band_x<N>, dim3((unsigned)((sm.ncell + 255) / 256), (unsigned)nbands), dim3(256), 0, st, C,
                       ngw, sm, W);
    BGW_HIP(hipGetLastError());
    const int bwy = 2 * sm.rwy + 1;
    const size_t lds = sizeof(double2) * (size_t)G * bwy * (N + 1);
    auto kern = k_band_yz<N, G>;
    BGW_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int xblk = 4 * G;
    const int nxb = (N + xblk - 1) / xblk;
    hipLaunchKernelGGL(kern, dim3((unsigned)((long long)nbands * nxb)), dim3(64), lds, st, W, sm.ncell, sm.rwy,
                       sm.rwz, xblk, grids);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}
}  // namespace

int launch_band_lines(const double2 *C, int nbands, int ngw, const AxisPlan &px, const AxisPlan &py,
                      const AxisPlan &pz, const SphereMaps &sm, double2 *W, double2 *grids, hipStream_t st) {
    if (nbands <= 0) return BGW_OK;
    if (!band_lines_supported(px, py, pz, sm)) return BGW_ERR_UNSUPPORTED;
    switch (pz.n) {
        case 16: return launch_band_lines_t<16, 4>(C, nbands, ngw, sm, W, grids, st);
        case 24: return launch_band_lines_t<24, 2>(C, nbands, ngw, sm, W, grids, st);
        case 32: return launch_band_lines_t<32, 2>(C, nbands, ngw, sm, W, grids, st);
        default: return BGW_ERR_UNSUPPORTED;
    }
}

}  // namespace bgw
