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

template <int Z1, int Z2, int Y1, int Y2, int ACC, int NT>
__global__ __launch_bounds__(NT) void k_pair_fft2(const double2 *__restrict__ gv, const double2 *__restrict__ gc,
                                                  int nkb, int nv, int nc, int n1, const double2 *__restrict__ tw1g,
                                                  const double2 *__restrict__ tw2g, const double2 *__restrict__ tw3g,
                                                  const int *__restrict__ ge_code, int ng, int rey, int rez, int lc,
                                                  int vb, int cb, double2 *__restrict__ M, long long m_row0) {
    constexpr int n3 = Z1 * Z2, n2 = Y1 * Y2;
    constexpr int PS = plane_stride<Z1, Z2>();
    const int bez = 2 * rez + 1, bey = 2 * rey + 1;
    const int QS = bez;
    extern __shared__ double2 lds[];
    double2 *tw1 = lds, *tw2 = tw1 + n1, *tw3 = tw2 + n2;
    double2 *P = tw3 + n3;            // [lc][PS]
    double2 *Q = P + lc * PS;         // [n2][QS]
    double2 *R = Q + n2 * QS;         // [bey][bez]

    for (int i = threadIdx.x; i < n1; i += NT) tw1[i] = tw1g[i];
    for (int i = threadIdx.x; i < n2; i += NT) tw2[i] = tw2g[i];
    for (int i = threadIdx.x; i < n3; i += NT) tw3[i] = tw3g[i];

    // ---- work order: XCD-contiguous chunks, then (k, c-tile, v-tile, c, v) with v fastest
    const long long total = (long long)nkb * nv * nc;
    long long L = blockIdx.x;
    {
        const long long per = total / 8;
        if (L < per * 8) L = (L % 8) * per + L / 8;
    }
    const int vtiles = (nv + vb - 1) / vb;
    const int ctiles = (nc + cb - 1) / cb;
    long long rem = L;
    // tiles may be ragged at the edges: walk (k, ct, vt) then the inner (c, v)
    int k = (int)(rem / ((long long)nv * nc));
    rem -= (long long)k * nv * nc;
    int v = 0, c = 0;
    {
        // rem in [0, nv*nc): locate the (ct, vt) tile containing it
        const int cw_full = cb;
        int done = 0;
        for (int ct = 0; ct < ctiles; ++ct) {
            const int cw = min(cw_full, nc - ct * cb);
            const int rowblock = cw * nv;  // pairs in this c-tile
            if (rem < done + rowblock) {
                int r2 = (int)(rem - done);
                for (int vt = 0; vt < vtiles; ++vt) {
                    const int vw = min(vb, nv - vt * vb);
                    const int blk = vw * cw;
                    if (r2 < blk) {
                        v = vt * vb + r2 % vw;
                        c = ct * cb + r2 / vw;
                        break;
                    }
                    r2 -= blk;
                }
                break;
            }
            done += rowblock;
        }
    }
    const long long t = ((long long)k * nv + v) * nc + c;
    const size_t N = (size_t)n1 * n2 * n3;
    const double2 *uv = gv + (size_t)(k * nv + v) * N;
    const double2 *uc = gc + (size_t)(k * nc + c) * N;

    int code[ACC], ph[ACC], mxs[ACC];
    double2 acc[ACC];
#pragma unroll
    for (int i = 0; i < ACC; ++i) {
        const int g = threadIdx.x + i * NT;
        code[i] = g < ng ? ge_code[g] : -1;
        mxs[i] = code[i] >= 0 ? (code[i] & 0xff) : 0;
        ph[i] = 0;
        acc[i] = make_double2(0.0, 0.0);
    }
    __syncthreads();

    for (int x = 0; x < n1; ++x) {
        for (int y0 = 0; y0 < n2; y0 += lc) {
            const int Lc = min(lc, n2 - y0);
            const double2 *pv = uv + ((size_t)x * n2 + y0) * n3;
            const double2 *pc = uc + ((size_t)x * n2 + y0) * n3;
            for (int e = threadIdx.x; e < Lc * n3; e += NT) {
                const int yy = e / n3, z = e - yy * n3;
                P[yy * PS + z] = cconjmul(pv[e], pc[e]);
            }
            __syncthreads();
            LineFFT<Z1, Z2>::stage1(P, Lc, PS, 1, tw3);
            __syncthreads();
            for (int e = threadIdx.x; e < Lc * bez; e += NT) {
                const int yy = e / bez, iz = e - yy * bez;
                Q[(y0 + yy) * QS + iz] = LineFFT<Z1, Z2>::output(P + yy * PS, 1, wrap(iz - rez, n3), tw3);
            }
            __syncthreads();
        }
        LineFFT<Y1, Y2>::stage1(Q, bez, 1, QS, tw2);
        __syncthreads();
        for (int e = threadIdx.x; e < bey * bez; e += NT) {
            const int iy = e / bez, iz = e - iy * bez;
            R[e] = LineFFT<Y1, Y2>::output(Q + iz, QS, wrap(iy - rey, n2), tw2);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ACC; ++i) {
            if (code[i] >= 0) {
                const int iy = (code[i] >> 8) & 0xff, iz = code[i] >> 16;
                acc[i] = cadd(acc[i], cmul(tw1[ph[i]], R[iy * bez + iz]));
                ph[i] += mxs[i];
                if (ph[i] >= n1) ph[i] -= n1;
            }
        }
    }
    const double inv = 1.0 / (double)N;
    double2 *out = M + (size_t)(m_row0 + t) * ng;
#pragma unroll
    for (int i = 0; i < ACC; ++i) {
        const int g = threadIdx.x + i * NT;
        if (g < ng) out[g] = cscale(acc[i], inv);
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

// ------------------------------------------------------------------ host side

namespace {

template <int Z1, int Z2, int ACC, int NT>
int launch_pair2_t(const double2 *gv, const double2 *gc, int nkb, int nv, int nc, const AxisPlan &px,
                   const AxisPlan &py, const AxisPlan &pz, const int *ge_code, int ng, int rey, int rez, double2 *M,
                   long long row0, hipStream_t st) {
    constexpr int n = Z1 * Z2;
    constexpr int PS = plane_stride<Z1, Z2>();
    const int bez = 2 * rez + 1, bey = 2 * rey + 1;
    // lines per z chunk: keep the workgroup's LDS at or below ~80 KB (two per CU)
    const size_t fixed = sizeof(double2) * ((size_t)px.n + n + n + (size_t)n * bez + (size_t)bey * bez);
    const size_t budget = 78 * 1024;
    int lc = n;
    while (lc > 4 && fixed + sizeof(double2) * (size_t)lc * PS > budget) lc = (lc + 1) / 2;
    const size_t lds = fixed + sizeof(double2) * (size_t)lc * PS;
    auto kern = k_pair_fft2<Z1, Z2, Z1, Z2, ACC, NT>;
    BGW_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const long long npairs = (long long)nkb * nv * nc;
    const int vb = std::min(nv, 8);
    const int cb = std::max(1, 256 / vb);
    hipLaunchKernelGGL(kern, dim3((unsigned)npairs), dim3(NT), lds, st, gv, gc, nkb, nv, nc, px.n, px.tw, py.tw,
                       pz.tw, ge_code, ng, rey, rez, lc, vb, cb, M, row0);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}

template <int Z1, int Z2, int NT>
int launch_pair2_n(int per, const double2 *gv, const double2 *gc, int nkb, int nv, int nc, const AxisPlan &px,
                   const AxisPlan &py, const AxisPlan &pz, const int *ge_code, int ng, int rey, int rez, double2 *M,
                   long long row0, hipStream_t st) {
#define BGW_P2(A)                                                                                                \
    if (per <= A)                                                                                                \
        return launch_pair2_t<Z1, Z2, A, NT>(gv, gc, nkb, nv, nc, px, py, pz, ge_code, ng, rey, rez, M, row0, st);
    BGW_P2(1)
    BGW_P2(2)
    BGW_P2(4)
    BGW_P2(8)
    BGW_P2(16)
    BGW_P2(32)
#undef BGW_P2
    return BGW_ERR_UNSUPPORTED;
}

}  // namespace

// Returns BGW_ERR_UNSUPPORTED (without launching) when no fast path applies.
int launch_pair_fft2(const double2 *gv, const double2 *gc, int nkb, int nv, int nc, const AxisPlan &px,
                     const AxisPlan &py, const AxisPlan &pz, const int *ge_code2, int ng, int rey, int rez,
                     double2 *M, long long row0, hipStream_t st) {
    if (py.n != pz.n) return BGW_ERR_UNSUPPORTED;
    const int n = pz.n;
    const int per = (ng + 255) / 256;
    switch (n) {
        case 16: return launch_pair2_n<16, 1, 256>(per, gv, gc, nkb, nv, nc, px, py, pz, ge_code2, ng, rey, rez, M, row0, st);
        case 24: return launch_pair2_n<8, 3, 256>(per, gv, gc, nkb, nv, nc, px, py, pz, ge_code2, ng, rey, rez, M, row0, st);
        case 32: return launch_pair2_n<16, 2, 256>(per, gv, gc, nkb, nv, nc, px, py, pz, ge_code2, ng, rey, rez, M, row0, st);
        case 48: return launch_pair2_n<16, 3, 256>(per, gv, gc, nkb, nv, nc, px, py, pz, ge_code2, ng, rey, rez, M, row0, st);
        case 64: return launch_pair2_n<16, 4, 256>(per, gv, gc, nkb, nv, nc, px, py, pz, ge_code2, ng, rey, rez, M, row0, st);
        case 96: return launch_pair2_n<16, 6, 256>(per, gv, gc, nkb, nv, nc, px, py, pz, ge_code2, ng, rey, rez, M, row0, st);
        case 128: return launch_pair2_n<16, 8, 256>(per, gv, gc, nkb, nv, nc, px, py, pz, ge_code2, ng, rey, rez, M, row0, st);
        default: return BGW_ERR_UNSUPPORTED;
    }
}

int launch_band_to_real2(const double2 *C, int nbands, int ngw, const AxisPlan &px, const AxisPlan &py,
                         const AxisPlan &pz, const SphereMaps &sm, int rwy, double2 *grids, hipStream_t st) {
    if (nbands <= 0) return BGW_OK;
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

}  // namespace bgw
