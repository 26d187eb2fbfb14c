// Internal definitions shared by the HIP translation units of libbgw.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "bgw.h"

namespace bgw {

// thread-local error message (bgw_last_error)
void set_error(const std::string &msg);
void clear_error();

#define BGW_HIP(call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            ::bgw::set_error(std::string("HIP error in ") + #call + ": " + hipGetErrorString(e_)); \
            return BGW_ERR_HIP;                                                                    \
        }                                                                                          \
    } while (0)

#define BGW_TRY(expr)              \
    do {                           \
        int rc_ = (expr);          \
        if (rc_ != BGW_OK) return rc_; \
    } while (0)

constexpr double kHartreeEv = 27.211386245988;  // CODATA 2018
constexpr int kMaxFFT = 128;

// ---------------------------------------------------------------- complex helpers
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cconjmul(double2 a, double2 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }

// ---------------------------------------------------------------- FFT plans
// One axis of a 3D transform: length n = product of radices (each 2, 3 or 4),
// twiddle table tw[j] = exp(+2 pi i j / n), j in [0, n), in device memory.
struct AxisPlan {
    int n;
    int nrad;
    int rad[8];
    const double2 *tw;
};

// Sphere description used by the kernels (device pointers).
struct SphereMaps {
    // wavefunction sphere grouped in sticks along x: stick s covers
    // stick_g[stick_start[s] .. stick_start[s+1]) (indices into the coefficient
    // list), with yz position stick_yz[s] = (my mod n2) | (iz << 16), iz = mz + Rwz,
    // and stick_mx[g] = mx mod n1 for each entry.
    int nstick;
    const int *stick_start;
    const int *stick_g;
    const int *stick_mx;
    const int *stick_yz;
    const int *stick_yz2;  // (my + Rwy) | (iz << 16): box row instead of FFT row
    int bwz, rwz;          // wavefunction box extent along z (2 Rwz + 1), Rwz
    int rwy;               // wavefunction box half-extent along y
    // dielectric sphere outputs: ge_code[g] = (mx mod n1) | ((my mod n2) << 8) | (iz << 16),
    // iz = mz + Rez
    int ng;
    const int *ge_code;
    const int *ge_code2;   // (mx mod n1) | ((my + Rey) << 8) | ((mz + Rez) << 16), in (mx, my, mz) order
    const int *ge_out;     // original index of the p-th point of that order
    int bez, rez;          // dielectric box extent along z, Rez
    int rey;               // dielectric box half-extent along y
    // lane-per-line band path (x-sticks contiguous in mx): cell c = iz * bwy + iy
    // of the (my, mz) box holds stick cell_stick[c] (-1: none); stick s has
    // entries st_gs[stick_start[s] .. stick_start[s+1]) in ascending mx from st_lo[s]
    int ncell;
    const int *cell_stick;
    const int *st_lo;
    const int *st_gs;
    bool sticks_contiguous;
};

// One q of a split-precision chi-sum launch (split.hip), a device table
// entry.  The launch covers the pair chunks [chunk0, chunk0 + nch) of every
// entry (96 pairs per chunk) and, per entry, all of its weight vectors.
struct SplitQ {
    const double2 *M;          // [K][ng]
    const double *w;           // weight vector v at w + v * wstride, [K] each
    const unsigned short *SB;  // BF16 digit slices of M for the launch's chunks: [4][nch][6][gpad][32]
    const int *EB;             // chunk-column exponents of those slices: [nch][gpad]
    double2 *out;              // raw upper-tile sums of (vector v, K split s): out + v * vstride + s * ng * ng
    const unsigned *tiles;     // upper tiles (64-row x 128-column) in walk order: I | J << 16
    long long K, wstride, vstride;
    long long item0, nitems;   // work items of this entry (nitems a multiple of 8)
    int ng, gpad, nvec, ntiles;
    int chunk0, nch;           // chunk range of the launch
    int ns;                    // K splits of the chunk range: split s takes chunks [s nch / ns, (s + 1) nch / ns)
    int add;                   // 1: add to the raw sums already in out (later chunk ranges)
    int pad[2];
    const signed char *EA;     // [nvec][nch][gpad] chunk-column exponents of the weighted side
};

// Upper-triangle tile number u -> (ti, tj) in grouped order: bands of four
// tile rows, each band walked column by column.  Consecutive tiles then
// share a few A row blocks and B column blocks, which is what the blocks
// co-resident on one XCD read at the same time.
__device__ inline void grouped_tile(int u, int nt, int &ti, int &tj) {
    constexpr int R = 4;
    int r0 = 0;
    for (;; r0 += R) {
        const int r1 = min(r0 + R - 1, nt - 1);
        int cnt = 0;
        for (int c = r0; c < nt; ++c) cnt += min(c, r1) - r0 + 1;
        if (u < cnt || r1 == nt - 1) break;
        u -= cnt;
    }
    const int r1 = min(r0 + R - 1, nt - 1);
    for (int c = r0;; ++c) {
        const int rows = min(c, r1) - r0 + 1;
        if (u < rows || c == nt - 1) {
            ti = r0 + u;
            tj = c;
            return;
        }
        u -= rows;
    }
}

// ---------------------------------------------------------------- batched chi sum
// One (q, omega) problem of a batched chi0 call.  Plain data: the tables are
// copied to device memory and read by the persistent kernels.
struct HerkProb {
    const double2 *M;  // [K][ng]
    const double *w;   // [K] weights of this omega
    double2 *out;      // [ns][ng][ng] raw upper-tile sums (or chi itself, ns == 1, in place)
    long long K;
    long long kper;    // pairs per work item (K split into ns ranges)
    long long item0;   // first work item of this problem in the batch
    long long nitems;  // work items of this problem: tiles * ns rounded up to a multiple of 8
    int ng;
    int tile;          // output tile edge: 64 or 32
    int nt;            // tiles per side
    int ns;            // K splits
};

// One product C = P^H Q (k_gemm_phq): P [K][ldp] (first m columns used), Q
// [K][ldq] (first n used); raw sums of the ns contraction ranges to
// out[ns][m][n].
struct GemmProb {
    const double2 *P;
    const double2 *Q;
    double2 *out;
    long long K, kper, ldp, ldq;
    int m, n, ntr, ntc, ns, pad;
};

// Real flavor: one real rank-K update problem (one weight vector) and its
// output matrix, as HerkProb / FinProb for real M and chi.  Output tiles are
// kSyrkTile square; the contraction advances kSyrkK pairs per LDS stage.
constexpr int kSyrkTile = 128;
constexpr int kSyrkK = 16;
struct SyrkProb {
    const double *M;   // [K][ng] real
    const double *w;   // [K]
    double *out;       // [ns][ng][ng] raw upper-tile sums (or chi itself, ns == 1, in place)
    long long K, kper, item0, nitems;
    int ng, nt, ns, pad;
};

struct SyrkFin {
    const double *part;  // [ns][ng][ng]
    double *chi;         // [ng][ng] output
    double pf;
    int ns, ng, accumulate, inplace;
};

// One output matrix of a chi0 call: chi = pf * (A + i B) where A (and, on
// the real frequency axis, B) are the Hermitian chi sums of one weight
// vector each, held as raw upper-triangle sums.
struct FinProb {
    const double2 *part;     // [ns][ng][ng] raw sums of A (unused in place)
    const double2 *part_im;  // [ns][ng][ng] raw sums of B, or null (imaginary axis: chi = pf A)
    double2 *chi;            // [ng][ng]
    double pf;
    int ns, ng;
    int accumulate;
    int skip;      // row/column left untouched (FP64 head row written separately), -1 for none
    int inplace;   // raw upper-triangle sums already sit in chi (ns == 1, no accumulation, no B)
    int pad;
};

// Kinds of weight vectors (k_weights), Delta = E_v,k+q - E_c,k < 0, all in hartree:
//   imaginary axis   w = Delta / (Delta^2 + omega^2)   (omega = 0: static 1 / Delta)
//   real axis        w = (1/2) [1/(Delta - E -+ i delta) + 1/(Delta + E +- i delta)]
//                    (upper signs retarded, lower advanced), as its real part and
//                    its imaginary part, each a real weight vector;
//   given            w = a weight array passed in (the Coulomb factor of the
//                    Bethe-Salpeter exchange kernel).
enum WeightKind { kWeightImag = 0, kWeightRealRe = 1, kWeightRetIm = 2, kWeightAdvIm = 3, kWeightGiven = 4 };

struct WProb {
    const double *ev;  // [nk][nv] eV (kWeightGiven: the weights themselves, [K])
    const double *ec;  // [nk][nc] eV
    double *w;         // [K]
    double omega_ha;   // |omega| (imaginary axis) or E (real axis), hartree
    double delta_ha;   // broadening (real axis), hartree
    int nk, nv, nc, kind;
};

}  // namespace bgw
