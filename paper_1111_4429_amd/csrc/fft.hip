// Pair densities M_vc(G) by FFT (epsilon section: the matrix element is a
// G-space convolution, rewritten as the Fourier transform of the real-space
// product conj(phi_v(r)) phi_c(r)).
//
//   k_band_to_real : C_n(G) on the wavefunction sphere -> u_n(r) on the n1 x n2 x n3
//                    grid, u_n(r_j) = sum_G C_n(G) exp(+2 pi i m_G.j/n).  Pruned:
//                    the x stage is a direct sum over each x-stick of the sphere,
//                    the y and z stages are LDS-staged FFTs of zero-padded lines.
//   k_pair_fft     : per pair, per x-plane: product conj(u_v) u_c (fused into the
//                    load), z FFT, prune to the dielectric box, y FFT, prune, then
//                    the x stage is accumulated directly on the sphere outputs
//                    (one phase multiply per sphere point and plane), in registers.
//
// Both transforms use the +2 pi i sign; M carries the 1/N of the inverse DFT.
// FFTs are Stockham autosort passes of radix 4, 2 and 3 with ping-pong LDS
// buffers; twiddles come from host tables exp(+2 pi i j/n) computed in long
// double and staged into LDS.
#include "common.h"

namespace bgw {

namespace {

constexpr int kThreads = 256;
constexpr double kSin60 = 0.86602540378443864676;  // sin(2 pi / 3)

__device__ inline void dft2(double2 &a, double2 &b) {
    double2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

// y_r = sum_s x_s exp(+2 pi i r s / 3)
__device__ inline void dft3(double2 &a, double2 &b, double2 &c) {
    double2 t1 = cadd(b, c), t2 = csub(b, c);
    double2 y0 = cadd(a, t1);
    double2 m = make_double2(a.x - 0.5 * t1.x, a.y - 0.5 * t1.y);
    double2 is = make_double2(-kSin60 * t2.y, kSin60 * t2.x);  // i sin60 (b - c)
    a = y0;
    b = cadd(m, is);
    c = csub(m, is);
}

// y_r = sum_s x_s exp(+2 pi i r s / 4)
__device__ inline void dft4(double2 &a, double2 &b, double2 &c, double2 &d) {
    double2 t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), t3 = csub(b, d);
    double2 it3 = make_double2(-t3.y, t3.x);
    a = cadd(t0, t2);
    c = csub(t0, t2);
    b = cadd(t1, it3);
    d = csub(t1, it3);
}

// One Stockham pass of radix R over `nlines` lines of length n; element e of
// line l sits at buf[l * ls + e * es].  Ns = product of the radices already
// applied.  tw: LDS table exp(+2 pi i j / n).
template <int R>
__device__ void stockham_pass(const double2 *src, double2 *dst, int nlines, int n, int ls, int es, int Ns,
                              const double2 *tw) {
    const int m = n / R;
    const int total = nlines * m;
    const int twstep = n / (Ns * R);
    for (int item = threadIdx.x; item < total; item += blockDim.x) {
        const int l = item / m;
        const int j = item - l * m;
        const double2 *s = src + l * ls;
        double2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = s[(j + r * m) * es];
        const int k = j % Ns;
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[r * k * twstep]);
        if (R == 2) dft2(v[0], v[1]);
        if (R == 3) dft3(v[0], v[1], v[2]);
        if (R == 4) dft4(v[0], v[1], v[2], v[3]);
        const int idx = (j / Ns) * Ns * R + k;
        double2 *d = dst + l * ls;
#pragma unroll
        for (int r = 0; r < R; ++r) d[(idx + r * Ns) * es] = v[r];
    }
}

// Full transform of `nlines` lines; returns the buffer holding the result
// (a or b).  Ends with a __syncthreads().
__device__ double2 *lds_fft(double2 *a, double2 *b, int nlines, int ls, int es, const AxisPlan &p,
                            const double2 *tw) {
    double2 *src = a, *dst = b;
    int Ns = 1;
    for (int i = 0; i < p.nrad; ++i) {
        const int R = p.rad[i];
        if (R == 4)
            stockham_pass<4>(src, dst, nlines, p.n, ls, es, Ns, tw);
        else if (R == 2)
            stockham_pass<2>(src, dst, nlines, p.n, ls, es, Ns, tw);
        else
            stockham_pass<3>(src, dst, nlines, p.n, ls, es, Ns, tw);
        __syncthreads();
        double2 *t = src;
        src = dst;
        dst = t;
        Ns *= R;
    }
    return src;
}

__device__ inline void load_twiddles(double2 *tw1, double2 *tw2, double2 *tw3, const AxisPlan &px,
                                     const AxisPlan &py, const AxisPlan &pz) {
    for (int i = threadIdx.x; i < px.n; i += blockDim.x) tw1[i] = px.tw[i];
    for (int i = threadIdx.x; i < py.n; i += blockDim.x) tw2[i] = py.tw[i];
    for (int i = threadIdx.x; i < pz.n; i += blockDim.x) tw3[i] = pz.tw[i];
}

}  // namespace

// One workgroup per band.  C: [nb][ngw]; grids: [nb][n1][n2][n3].
__global__ __launch_bounds__(kThreads) void k_band_to_real(const double2 *__restrict__ C, int ngw, AxisPlan px,
                                                           AxisPlan py, AxisPlan pz, SphereMaps sm, int lc,
                                                           double2 *__restrict__ grids) {
    extern __shared__ double2 lds[];
    const int n1 = px.n, n2 = py.n, n3 = pz.n;
    const int bwz = sm.bwz;
    double2 *tw1 = lds, *tw2 = tw1 + n1, *tw3 = tw2 + n2;
    double2 *Q = tw3 + n3, *Q2 = Q + n2 * bwz;
    double2 *bufA = Q2 + n2 * bwz, *bufB = bufA + lc * n3;
    int *zmap = reinterpret_cast<int *>(bufB + lc * n3);

    load_twiddles(tw1, tw2, tw3, px, py, pz);
    for (int z = threadIdx.x; z < n3; z += blockDim.x) {
        int iz = z - n3;  // z as a negative frequency
        int m = (z <= sm.rwz) ? z : (iz >= -sm.rwz ? iz : 1 << 20);
        zmap[z] = (m == (1 << 20)) ? -1 : m + sm.rwz;
    }
    const size_t N = (size_t)n1 * n2 * n3;
    const double2 *cb = C + (size_t)blockIdx.x * ngw;
    double2 *out = grids + (size_t)blockIdx.x * N;
    __syncthreads();

    for (int x = 0; x < n1; ++x) {
        for (int e = threadIdx.x; e < n2 * bwz; e += blockDim.x) Q[e] = make_double2(0.0, 0.0);
        __syncthreads();
        // x stage: each stick (fixed my, mz) sums its coefficients times exp(+2 pi i mx x / n1)
        for (int s = threadIdx.x; s < sm.nstick; s += blockDim.x) {
            double2 acc = make_double2(0.0, 0.0);
            for (int i = sm.stick_start[s]; i < sm.stick_start[s + 1]; ++i) {
                const double2 c = cb[sm.stick_g[i]];
                const double2 ph = tw1[(sm.stick_mx[i] * x) % n1];
                acc = cadd(acc, cmul(ph, c));
            }
            const int yz = sm.stick_yz[s];
            Q[(yz & 0xffff) * bwz + (yz >> 16)] = acc;
        }
        __syncthreads();
        // y stage: bwz zero-padded columns of length n2
        const double2 *r = lds_fft(Q, Q2, bwz, 1, bwz, py, tw2);
        // z stage in chunks of lc lines
        for (int y0 = 0; y0 < n2; y0 += lc) {
            const int L = min(lc, n2 - y0);
            for (int e = threadIdx.x; e < L * n3; e += blockDim.x) {
                const int yy = e / n3, z = e - yy * n3;
                const int iz = zmap[z];
                bufA[e] = iz >= 0 ? r[(y0 + yy) * bwz + iz] : make_double2(0.0, 0.0);
            }
            __syncthreads();
            const double2 *r3 = lds_fft(bufA, bufB, L, n3, 1, pz, tw3);
            double2 *o = out + ((size_t)x * n2 + y0) * n3;
            for (int e = threadIdx.x; e < L * n3; e += blockDim.x) o[e] = r3[e];
            __syncthreads();
        }
    }
}

// One workgroup per pair of the k-batch.  Pair t = (k*nv + v)*nc + c within the
// batch; gv: [nkb][nv][N] valence grids, gc: [nkb][nc][N] conduction grids.
// M row (m_row0 + t), ng columns.  ACC = sphere points per thread (ng <= 256*ACC).
template <int ACC>
__global__ __launch_bounds__(kThreads) void k_pair_fft(const double2 *__restrict__ gv,
                                                       const double2 *__restrict__ gc, int nv, int nc,
                                                       AxisPlan px, AxisPlan py, AxisPlan pz, SphereMaps sm,
                                                       int lc, double2 *__restrict__ M, long long m_row0) {
    extern __shared__ double2 lds[];
    const int n1 = px.n, n2 = py.n, n3 = pz.n;
    const int bez = sm.bez;
    double2 *tw1 = lds, *tw2 = tw1 + n1, *tw3 = tw2 + n2;
    double2 *Q = tw3 + n3, *Q2 = Q + n2 * bez;
    double2 *bufA = Q2 + n2 * bez, *bufB = bufA + lc * n3;

    load_twiddles(tw1, tw2, tw3, px, py, pz);

    const int t = blockIdx.x;
    const int c = t % nc;
    const int kv = t / nc;
    const int v = kv % nv;
    const int k = kv / nv;
    const size_t N = (size_t)n1 * n2 * n3;
    const double2 *uv = gv + (size_t)(k * nv + v) * N;
    const double2 *uc = gc + (size_t)(k * nc + c) * N;

    int code[ACC];
    double2 acc[ACC];
#pragma unroll
    for (int i = 0; i < ACC; ++i) {
        const int g = threadIdx.x + i * kThreads;
        code[i] = g < sm.ng ? sm.ge_code[g] : -1;
        acc[i] = make_double2(0.0, 0.0);
    }
    __syncthreads();

    for (int x = 0; x < n1; ++x) {
        for (int y0 = 0; y0 < n2; y0 += lc) {
            const int L = min(lc, n2 - y0);
            const double2 *pv = uv + ((size_t)x * n2 + y0) * n3;
            const double2 *pc = uc + ((size_t)x * n2 + y0) * n3;
            for (int e = threadIdx.x; e < L * n3; e += blockDim.x) bufA[e] = cconjmul(pv[e], pc[e]);
            __syncthreads();
            const double2 *r = lds_fft(bufA, bufB, L, n3, 1, pz, tw3);
            for (int e = threadIdx.x; e < L * bez; e += blockDim.x) {
                const int yy = e / bez, iz = e - yy * bez;
                const int mz = iz - sm.rez;
                Q[(y0 + yy) * bez + iz] = r[yy * n3 + (mz < 0 ? mz + n3 : mz)];
            }
            __syncthreads();
        }
        const double2 *r2 = lds_fft(Q, Q2, bez, 1, bez, py, tw2);
#pragma unroll
        for (int i = 0; i < ACC; ++i) {
            const int cd = code[i];
            if (cd >= 0) {
                const int mx = cd & 0xff, yrow = (cd >> 8) & 0xff, iz = cd >> 16;
                const double2 ph = tw1[(mx * x) % n1];
                acc[i] = cadd(acc[i], cmul(ph, r2[yrow * bez + iz]));
            }
        }
        __syncthreads();
    }
    const double inv = 1.0 / (double)N;
    double2 *out = M + (size_t)(m_row0 + t) * sm.ng;
#pragma unroll
    for (int i = 0; i < ACC; ++i) {
        const int g = threadIdx.x + i * kThreads;
        if (g < sm.ng) out[g] = cscale(acc[i], inv);
    }
}

// ---------------------------------------------------------------- host launchers

size_t band_lds_bytes(const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz, int bwz, int lc) {
    return sizeof(double2) * ((size_t)px.n + py.n + pz.n + 2 * (size_t)py.n * bwz + 2 * (size_t)lc * pz.n) +
           sizeof(int) * pz.n;
}

size_t pair_lds_bytes(const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz, int bez, int lc) {
    return sizeof(double2) * ((size_t)px.n + py.n + pz.n + 2 * (size_t)py.n * bez + 2 * (size_t)lc * pz.n);
}

int launch_band_to_real(const double2 *C, int nbands, int ngw, const AxisPlan &px, const AxisPlan &py,
                        const AxisPlan &pz, const SphereMaps &sm, int lc, double2 *grids, hipStream_t st) {
    if (nbands <= 0) return BGW_OK;
    const size_t lds = band_lds_bytes(px, py, pz, sm.bwz, lc);
    BGW_HIP(hipFuncSetAttribute((const void *)k_band_to_real, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    hipLaunchKernelGGL(k_band_to_real, dim3(nbands), dim3(kThreads), lds, st, C, ngw, px, py, pz, sm, lc,
                       grids);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

template <int ACC>
static int launch_pair_t(const double2 *gv, const double2 *gc, int nkb, int nv, int nc, const AxisPlan &px,
                         const AxisPlan &py, const AxisPlan &pz, const SphereMaps &sm, int lc, double2 *M,
                         long long row0, hipStream_t st) {
    const size_t lds = pair_lds_bytes(px, py, pz, sm.bez, lc);
    BGW_HIP(hipFuncSetAttribute((const void *)k_pair_fft<ACC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds));
    const long long npairs = (long long)nkb * nv * nc;
    hipLaunchKernelGGL(k_pair_fft<ACC>, dim3((unsigned)npairs), dim3(kThreads), lds, st, gv, gc, nv, nc, px, py,
                       pz, sm, lc, M, row0);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

int launch_pair_fft(const double2 *gv, const double2 *gc, int nkb, int nv, int nc, const AxisPlan &px,
                    const AxisPlan &py, const AxisPlan &pz, const SphereMaps &sm, int lc, double2 *M,
                    long long row0, hipStream_t st) {
    const int per = (sm.ng + kThreads - 1) / kThreads;
    if (per <= 1) return launch_pair_t<1>(gv, gc, nkb, nv, nc, px, py, pz, sm, lc, M, row0, st);
    if (per <= 2) return launch_pair_t<2>(gv, gc, nkb, nv, nc, px, py, pz, sm, lc, M, row0, st);
    if (per <= 4) return launch_pair_t<4>(gv, gc, nkb, nv, nc, px, py, pz, sm, lc, M, row0, st);
    if (per <= 8) return launch_pair_t<8>(gv, gc, nkb, nv, nc, px, py, pz, sm, lc, M, row0, st);
    if (per <= 16) return launch_pair_t<16>(gv, gc, nkb, nv, nc, px, py, pz, sm, lc, M, row0, st);
    if (per <= 32) return launch_pair_t<32>(gv, gc, nkb, nv, nc, px, py, pz, sm, lc, M, row0, st);
    set_error("dielectric sphere larger than 8192 G-vectors on the generic transform path (a box outside the "
              "register-resident lengths) is not supported");
    return BGW_ERR_UNSUPPORTED;
}

}  // namespace bgw
