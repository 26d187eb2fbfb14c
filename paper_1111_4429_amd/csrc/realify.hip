// Real coefficients from complex ones (the paper's real and complex
// flavors).  With inversion and time-reversal symmetry every state can be
// chosen with real plane-wave coefficients; a plane-wave code usually
// returns them complex: a non-degenerate state as real times a global phase,
// a group of d degenerate states as any orthonormal basis of a subspace that
// the real and imaginary parts of the d states span in d real dimensions.
// Per group, Gram-Schmidt over the 2d vectors Re c_b, Im c_b (b in the group,
// in that order), the remaining vector of largest norm first (lowest index on
// ties), gives the group's d real orthonormal states.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "handle.h"

namespace bgw {

namespace {
constexpr int kRealifyThreads = 256;
constexpr int kRealifyMaxGroup = 32;  // states in one degenerate group

struct RealifyGroup {
    int k, b0, d, pad;
};

__device__ __forceinline__ double block_sum(double x, double *sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kRealifyThreads / 64; ++w) t += sh[w];
    __syncthreads();  // sh is reused by the next sum
    return t;
}
}  // namespace

// One workgroup per degenerate group.  v: the group's 2d candidate vectors
// (row 2i = Re c_{b0+i}, row 2i+1 = Im c_{b0+i}), workspace; every thread
// reads and writes only its own coefficient indices g = tid + 256 j, so the
// block sums are the only exchange between threads.
__global__ __launch_bounds__(kRealifyThreads) void k_realify(const RealifyGroup *__restrict__ groups,
                                                             const double2 *__restrict__ c, int nb, int ngw,
                                                             double *__restrict__ vws, double *__restrict__ r,
                                                             int *__restrict__ nbad) {
    __shared__ double sh[kRealifyThreads / 64];
    __shared__ unsigned long long used;  // bit j: candidate j taken
    const RealifyGroup G = groups[blockIdx.x];
    const int d = G.d, m = 2 * d, tid = threadIdx.x;
    const size_t row0 = (size_t)G.k * nb + G.b0;  // first band of the group
    double *v = vws + 2 * row0 * ngw;
    for (int i = 0; i < d; ++i) {
        const double2 *cb = c + (row0 + i) * ngw;
        for (int g = tid; g < ngw; g += kRealifyThreads) {
            const double2 z = cb[g];
            v[(size_t)(2 * i) * ngw + g] = z.x;
            v[(size_t)(2 * i + 1) * ngw + g] = z.y;
        }
    }
    if (tid == 0) used = 0ull;
    __syncthreads();
    bool deficient = false;
    for (int s = 0; s < d; ++s) {
        int p = -1;
        double best = -1.0;
        for (int j = 0; j < m; ++j) {
            if ((used >> j) & 1ull) continue;  // uniform
            double nn = 0.0;
            const double *vj = v + (size_t)j * ngw;
            for (int g = tid; g < ngw; g += kRealifyThreads) nn += vj[g] * vj[g];
            nn = block_sum(nn, sh);
            if (nn > best) {
                best = nn;
                p = j;
            }
        }
        __syncthreads();  // every thread has read `used`
        double *q = r + (row0 + s) * ngw;
        if (p < 0 || !(best > 0.0)) {  // uniform: fewer than d real dimensions (or NaN norms)
            deficient = true;
            for (int g = tid; g < ngw; g += kRealifyThreads) q[g] = 0.0;
            __syncthreads();
            continue;
        }
        if (tid == 0) used |= 1ull << p;
        const double *vp = v + (size_t)p * ngw;
        const double inv = 1.0 / sqrt(best);
        for (int g = tid; g < ngw; g += kRealifyThreads) q[g] = vp[g] * inv;
        __syncthreads();  // `used` updated
        for (int j = 0; j < m; ++j) {
            if ((used >> j) & 1ull) continue;
            double *vj = v + (size_t)j * ngw;
            double dot = 0.0;
            for (int g = tid; g < ngw; g += kRealifyThreads) dot += q[g] * vj[g];
            dot = block_sum(dot, sh);
            for (int g = tid; g < ngw; g += kRealifyThreads) vj[g] -= dot * q[g];
        }
    }
    // what is left must be (numerically) zero: the group was real up to a unitary
    double rest = 0.0;
    for (int j = 0; j < m; ++j) {
        if ((used >> j) & 1ull) continue;
        double nn = 0.0;
        const double *vj = v + (size_t)j * ngw;
        for (int g = tid; g < ngw; g += kRealifyThreads) nn += vj[g] * vj[g];
        rest = fmax(rest, block_sum(nn, sh));
    }
    if (tid == 0 && (deficient || sqrt(rest) > 1e-6)) atomicAdd(nbad, 1);
}

__global__ void k_realify_zero(int *nbad) { *nbad = 0; }

namespace {
// Degenerate groups of every k: consecutive bands whose energies differ by at
// most tol from their neighbour.  Returns the largest group size.
int realify_groups(int nk, int nb, const double *e, double tol, std::vector<RealifyGroup> &out) {
    int dmax = 0;
    for (int k = 0; k < nk; ++k) {
        const double *ek = e + (size_t)k * nb;
        int b0 = 0;
        while (b0 < nb) {
            int b1 = b0 + 1;
            while (b1 < nb && ek[b1] - ek[b1 - 1] <= tol) ++b1;
            out.push_back(RealifyGroup{k, b0, b1 - b0, 0});
            dmax = std::max(dmax, b1 - b0);
            b0 = b1;
        }
    }
    return dmax;
}

int realify_check(int nk, int nb, int ngw, const double *e, double tol) {
    if (nk < 1 || nb < 1 || ngw < 1 || !e || !(tol >= 0.0)) return fail(BGW_ERR_ARG, "bad arguments to bgw_realify");
    for (int k = 0; k < nk; ++k)
        for (int b = 1; b < nb; ++b)
            if (!(e[(size_t)k * nb + b] >= e[(size_t)k * nb + b - 1]))
                return fail(BGW_ERR_ARG, "bgw_realify: energies must ascend within each k");
    return BGW_OK;
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

size_t realify_ws_bytes(int nk, int nb, int ngw, size_t ngroups) {
    return al256(sizeof(double) * 2 * (size_t)nk * nb * ngw) + al256(sizeof(RealifyGroup) * ngroups);
}
}  // namespace

}  // namespace bgw

using namespace bgw;

extern "C" int bgw_realify_workspace(bgw_handle_t h, int nk, int nb, int ngw, const double *e, double tol,
                                     size_t *bytes) {
    clear_error();
    BGW_TRY(realify_check(nk, nb, ngw, e, tol));
    if (!h || !bytes) return fail(BGW_ERR_ARG, "null handle or output");
    std::vector<RealifyGroup> groups;
    realify_groups(nk, nb, e, tol, groups);
    *bytes = realify_ws_bytes(nk, nb, ngw, groups.size());
    return BGW_OK;
}

extern "C" int bgw_realify(bgw_handle_t h, int nk, int nb, int ngw, const double *c, const double *e, double tol,
                           double *r, int *nbad, void *stream) {
    clear_error();
    BGW_TRY(realify_check(nk, nb, ngw, e, tol));
    std::vector<RealifyGroup> groups;
    if (realify_groups(nk, nb, e, tol, groups) > kRealifyMaxGroup)
        return fail(BGW_ERR_UNSUPPORTED, "bgw_realify: a degenerate group of more than 32 states");
    if (!h || !c || !r || !nbad) return fail(BGW_ERR_ARG, "null handle or array");
    BGW_TRY(set_device(h));
    hipStream_t st = (hipStream_t)stream;
    const size_t need = realify_ws_bytes(nk, nb, ngw, groups.size());
    BGW_TRY(ensure_ws(h, need, st));
    char *ws = (char *)h->ws.p;
    double *vws = (double *)ws;
    RealifyGroup *dg = (RealifyGroup *)(ws + al256(sizeof(double) * 2 * (size_t)nk * nb * ngw));
    // the group table goes up with the stream's work; the host copy lives until it has
    BGW_HIP(hipMemcpyAsync(dg, groups.data(), sizeof(RealifyGroup) * groups.size(), hipMemcpyHostToDevice, st));
    BGW_HIP(hipStreamSynchronize(st));
    hipLaunchKernelGGL(k_realify_zero, dim3(1), dim3(1), 0, st, nbad);
    hipLaunchKernelGGL(k_realify, dim3((unsigned)groups.size()), dim3(kRealifyThreads), 0, st,
                       (const RealifyGroup *)dg, (const double2 *)c, nb, ngw, vws, r, nbad);
    BGW_HIP(hipGetLastError());
    return BGW_OK;
}
