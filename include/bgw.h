/*
 * bgw.h -- C-ABI of the MI355X hot path of the RPA polarizability step of
 * the GW method (Deslippe et al., "BerkeleyGW: A massively parallel computer
 * package ...", section "RPA Dielectric Matrix: epsilon").
 *
 * The paper splits the epsilon step into three computationally intensive
 * parts (epsilon section, paragraph that opens "The computation of
 * epsilon^-1 ... involves three computationally intensive steps"):
 *   1. the plane-wave matrix elements M_nn'(k,q,G)   -> bgw_pair_density
 *   2. the chi summation                             -> bgw_chi0
 *   3. the dielectric matrix and its inversion       -> bgw_eps_inv
 *
 * Conventions shared by every call:
 *   - complex numbers are interleaved (re, im) doubles, row-major arrays,
 *     i.e. the memory layout of numpy/torch complex128;
 *   - "DEVICE" pointers are HIP device memory on the handle's GPU, "HOST"
 *     pointers are ordinary host memory; the caller owns every input and
 *     output buffer, the library owns only its workspace (held by the
 *     handle, grown on demand, released by bgw_destroy);
 *   - `stream` is a hipStream_t (NULL = default stream); all GPU work is
 *     enqueued asynchronously on it and the call returns without waiting;
 *     calls on one handle must not overlap (they share the workspace);
 *   - every function returns BGW_OK or a negative BGW_ERR_* code and sets a
 *     thread-local message readable with bgw_last_error(); no C++ exception
 *     crosses this interface.
 *
 * Environment switches, read at each call.  The first two are limits a
 * deployment may set; the others force one of the library's own code paths
 * (for tests and comparisons) and change no result beyond rounding order:
 *   BGW_WORKSPACE_LIMIT=<bytes>    cap on the handle's device workspace;
 *   BGW_TUNE_CACHE=<file>          JSON-lines cache of bgw_autotune choices;
 *   BGW_FFT_BOX=full               transform on the caller's grid, not the
 *                                  smallest alias-free box;
 *   BGW_GENERIC_FFT=1              generic 2^a 3^b transform kernels only;
 *   BGW_HERK_TILE=32|64            FP64 chi-sum output tile;
 *   BGW_SPLIT_SLICE_BYTES=<bytes>  split chi-sum slice budget per launch
 *                                  (a smaller one cuts K into more launches);
 *   BGW_GJE_PATH=coop              cooperative panels in bgw_eps_inv also
 *                                  for ng <= 1536.
 *
 * Units: energies and frequencies in eV (converted with 1 Ha =
 * 27.211386245988 eV), lengths in bohr, Miller indices in reciprocal-
 * lattice units with components in [-n/2, n/2) (paper, Appendix on file
 * formats).
 */
#ifndef BGW_H
#define BGW_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BGW_OK 0
#define BGW_ERR_ARG (-1)         /* null/negative/inconsistent argument, omega < 0 */
#define BGW_ERR_ALIAS (-2)       /* FFT grid too small: some axis has n_i <= 2 max|gw_i| + max|ge_i| */
#define BGW_ERR_SHAPE (-3)       /* duplicate G, component outside [-n/2, n/2), |q+G| = 0 */
#define BGW_ERR_HIP (-4)         /* a HIP runtime call failed */
#define BGW_ERR_NOMEM (-5)       /* workspace could not be allocated (or exceeds BGW_WORKSPACE_LIMIT) */
#define BGW_ERR_UNSUPPORTED (-6) /* e.g. an FFT grid length that is not 2^a 3^b in [4, 1024] */

#define BGW_AXIS_IMAG 0          /* chi0 at imaginary frequencies i|omega| (omega = 0: static) */
#define BGW_AXIS_RETARDED 1      /* chi0^r at real frequencies E >= 0 with broadening delta */
#define BGW_AXIS_ADVANCED 2      /* chi0^a at real frequencies E >= 0 with broadening delta */

#define BGW_FP64 0               /* chi-sum on FP64 MFMA */
#define BGW_SPLIT_BF16 1         /* chi-sum as split BF16 slices, FP32 accumulation, FP64 recombination */

typedef struct bgw_handle_s *bgw_handle_t;

/* Library version, as 10000*major + 100*minor + patch. */
int bgw_version(void);

/* Create a handle bound to HIP device `hip_device`.  Allocates nothing on
 * the GPU until the first compute call. */
int bgw_create(bgw_handle_t *h, int hip_device);

/* Release the handle and its workspace.  Waits for the handle's device to
 * finish outstanding work first.  NULL is accepted. */
int bgw_destroy(bgw_handle_t h);

/* Message for the last non-zero return on the calling thread ("" if none). */
const char *bgw_last_error(void);

/* Bytes of device workspace the handle currently holds (it grows to the
 * largest requirement of the calls made so far).  What a given call needs
 * is returned, before the call, by bgw_pair_density_workspace,
 * bgw_chi0_workspace and bgw_eps_inv_workspace; a call allocates exactly
 * that much when the handle holds less, and fails with BGW_ERR_NOMEM when
 * it exceeds the environment variable BGW_WORKSPACE_LIMIT (bytes). */
size_t bgw_workspace_bytes(bgw_handle_t h);

/* ------------------------------------------------------------------------
 * Pair densities (plane-wave matrix elements)
 *
 * M_t(G) = <v,k+q| e^{i(q+G).r} |c,k>  (epsilon section, matrix-element
 * equation) for every pair t = (k*nv + v)*nc + c, computed the paper's way
 * (the FFT rewrite of the same section): the bands are taken to real space,
 * the product conj(u_v(r)) u_c(r) is formed on the n1 x n2 x n3 grid and
 * Fourier transformed back, and the dielectric-sphere entries are kept:
 *     u_n(r_j) = sum_{G in wfn sphere} C_n(G) exp(+2 pi i m_G . j / n)
 *     M_t(G)   = (1/N) sum_j conj(u_v(r_j)) u_c(r_j) exp(+2 pi i m_G . j / n)
 * This equals the matrix element exactly when no axis aliases, i.e.
 * n_i > 2 max|gw_i| + max|ge_i| for i = 1..3 (else BGW_ERR_ALIAS).
 * Because the result does not depend on the grid once it is alias-free, the
 * transforms run on a small alias-free box b (each b_i >= 2 max|gw_i| +
 * max|ge_i| + 1, b_i <= n_i): the least lengths of {16, 24, 32, 48, 64, 96,
 * 128} (equal along y and z) when they fit in n, which have register-resident
 * kernels, else the least 2^a 3^b length per axis.  Setting the environment
 * variable BGW_FFT_BOX=full makes the library use n itself;
 * bgw_pair_transform_box reports the box.  The box must be at most 128 on
 * every axis (BGW_ERR_UNSUPPORTED otherwise); the caller's grid itself may
 * be up to 1024 per axis.
 * ---------------------------------------------------------------------- */
typedef struct {
    int n[3];          /* FFT grid; each n_i = 2^a 3^b with 4 <= n_i <= 1024 */
    int ngw;           /* wavefunction sphere size */
    const int *gw;     /* HOST int32 [ngw][3] Miller indices of the coefficients */
    int ng;            /* dielectric sphere size (columns of M) */
    const int *ge;     /* HOST int32 [ng][3] Miller indices of the outputs */
    int nk, nv, nc;    /* k-points, valence bands (at k+q), conduction bands (at k) */
    const double *cv;  /* DEVICE complex128 [nk][nv][ngw]: valence at k+q */
    const double *cc;  /* DEVICE complex128 [nk][nc][ngw]: conduction at k */
} bgw_pair_desc;

/* Host-only validation of a descriptor (sizes, null pointers, G-vector
 * ranges and duplicates, alias-free grid).  Touches no GPU and no
 * coefficient memory.  Returns BGW_OK or the code bgw_pair_density would. */
int bgw_pair_desc_check(const bgw_pair_desc *d);

/* Host-only: the transform box b[3] bgw_pair_density will use for d. */
int bgw_pair_transform_box(const bgw_pair_desc *d, int box[3]);

/* M: DEVICE complex128 [nk*nv*nc][ng] (pair-major), written in full.
 * Must not overlap cv/cc.  Deterministic: identical inputs give bitwise
 * identical M. */
int bgw_pair_density(bgw_handle_t h, const bgw_pair_desc *d, double *M, void *stream);

/* Device workspace bgw_pair_density(h, d, ...) needs, in bytes, written to
 * *bytes (HOST).  The k-batch adapts to the free device memory and to
 * BGW_WORKSPACE_LIMIT, so the answer holds for a call made next, with no
 * allocation in between.  Builds (and caches in h) the transform plan, a
 * few small device tables; allocates no workspace. */
int bgw_pair_density_workspace(bgw_handle_t h, const bgw_pair_desc *d, size_t *bytes);

/* ------------------------------------------------------------------------
 * Polarizability chi0_GG'(q, omega)
 *
 * Static chi equation of the epsilon section, with its compact form
 * chi = M^H diag(w) M over the composite pair index (n, n', k), and the
 * implicit 1/(N_k V_uc) of every k sum (GW-BSE overview) passed in as
 * `prefactor`:
 *     chi_GG'(omega) = prefactor * sum_t conj(M_t(G)) w_t(omega) M_t(G')
 *     Delta_t        = E_{v,k+q} - E_{c,k}  (hartree; < 0 for insulators)
 * Imaginary axis (axis = BGW_AXIS_IMAG): w_t = Delta_t / (Delta_t^2 + omega^2);
 * omega = 0 is the static case 1/Delta, omega > 0 the paper's
 * retarded/advanced bracket evaluated at E = i omega with vanishing
 * broadening.  chi is Hermitian; the full matrix is returned (lower triangle
 * = conjugate mirror of the upper one).
 * Real axis (full-frequency section of the epsilon step, retarded/advanced
 * dielectric equation): omega[] holds real frequencies E >= 0 and
 *     w_t = (1/2) [1/(Delta_t - E -+ i delta) + 1/(Delta_t + E +- i delta)]
 * with the upper signs for the retarded function (BGW_AXIS_RETARDED) and the
 * lower ones for the advanced function (BGW_AXIS_ADVANCED), delta the
 * broadening.  The weight is complex, so chi = pf (A + i B) with A and B the
 * Hermitian sums of Re w and Im w: chi is a general complex matrix, and
 * chi^a(E) = chi^r(E)^H.  Both sums run on the kernels of the Hermitian case.
 * Row and column `head` (the index of G = 0, or -1) are always computed in
 * FP64 from M, also in split precision, because v(q0+0) ~ 1/q0^2 amplifies
 * them.
 * ---------------------------------------------------------------------- */
typedef struct {
    int ng;              /* rows/cols of chi for this q, 1 .. 12288 (uneven across q allowed) */
    int nk, nv, nc;      /* pair count K = nk*nv*nc, t = (k*nv + v)*nc + c */
    const double *M;     /* DEVICE complex128 [K][ng], e.g. from bgw_pair_density */
    const double *ev;    /* DEVICE f64 [nk][nv], valence energies at k+q (eV) */
    const double *ec;    /* DEVICE f64 [nk][nc], conduction energies at k (eV) */
    int head;            /* index of G = 0 in this q's list, -1 if absent */
    double prefactor;    /* usually 1/(N_k V_uc) in bohr^-3 */
    double *chi;         /* DEVICE complex128 [nw][ng][ng], output */
} bgw_chi_q;

typedef struct {
    int nq;              /* number of q entries, >= 1 */
    const bgw_chi_q *q;  /* HOST array [nq] */
    int nw;              /* number of frequencies, >= 1 */
    const double *omega; /* HOST f64 [nw], imaginary-axis |omega| in eV, >= 0 */
    int precision;       /* BGW_FP64 or BGW_SPLIT_BF16 */
    int accumulate;      /* 0: chi = result; 1: chi += result (K-chunked sums) */
    int use_graph;       /* 1: capture the call's launch sequence into a HIP graph the first
                            time this exact descriptor (same pointers, sizes, frequencies) is
                            seen, and replay the graph on later calls; 0: launch directly */
    int axis;            /* BGW_AXIS_IMAG (0), BGW_AXIS_RETARDED or BGW_AXIS_ADVANCED */
    double broadening;   /* delta in eV, > 0 on the real axis (ignored on the imaginary axis) */
} bgw_chi_desc;

/* All q entries and all frequencies form one batch: one weight vector per
 * (q, frequency) on the imaginary axis, two (Re w, Im w) on the real axis.
 * FP64: one launch for the weights, one persistent rank-K-update launch per
 * output-tile size over every (vector, output tile, K range) work item, one
 * finalize launch.  Split: weights in one launch; the frequency-independent
 * digit slices of every q (k_split_slice); one persistent BF16 launch over
 * every (q, vector, tile, K range) item whose slices fit in the workspace
 * together (usually the whole batch), which slices the weighted side in
 * registers; the FP64 head rows of all vectors of a q in one pass over M;
 * one finalize launch.  Output tiles and K-split counts per size class
 * (ng rounded up to 512, ceil(log2 K)) come from bgw_autotune when it has
 * run, from fixed rules otherwise.  Work is ordered on `stream`; calls on one
 * handle must not run concurrently (they share its workspace). */
int bgw_chi0(bgw_handle_t h, const bgw_chi_desc *d, void *stream);

/* Device workspace bgw_chi0(h, d, ...) needs, in bytes (HOST *bytes):
 * weights, partial sums and, in split precision, the digit slices.
 * Allocates nothing. */
int bgw_chi0_workspace(bgw_handle_t h, const bgw_chi_desc *d, size_t *bytes);

/* Autotuner.  For every size class present in d (precision taken from d),
 * times the candidate configurations (FP64: output tile 32 or 64 and the
 * K-split density; split: the GEMM's K-split count) on the class's first q
 * and first frequency, with K cut to at most 2^17 pairs, and keeps the
 * fastest in the handle.  Synchronises `stream`.  Overwrites chi[0] of the q
 * entries it times (an output buffer).  When the environment variable
 * BGW_TUNE_CACHE names a file, the choices are appended to it as JSON lines
 * and read back by later handles of the same device type. */
int bgw_autotune(bgw_handle_t h, const bgw_chi_desc *d, void *stream);

/* Configuration bgw_chi0 uses for one size class: cfg[0] FP64 output tile,
 * cfg[1] FP64 target work items per compute unit, cfg[2] split GEMM K-split
 * count (0 = rule), cfg[3] 1 if it comes from the autotuner. */
int bgw_tuned_config(bgw_handle_t h, int precision, int ng, long long K, int *cfg);

/* ------------------------------------------------------------------------
 * Real flavor (section on real and complex flavors)
 *
 * With inversion and time-reversal symmetry the plane-wave coefficients can
 * be chosen real; the pair densities M_vc(G) are then real and the chi sum
 * is a real symmetric rank-K update (four times fewer flops than the complex
 * one, half the memory for M and chi).
 * ---------------------------------------------------------------------- */
/* bgw_pair_density for real coefficients: d->cv and d->cc point to DEVICE
 * f64 [nk][nv][ngw] and [nk][nc][ngw]; M is DEVICE f64 [K][ng].  The
 * transforms run in the complex pipeline (its workspace as for
 * bgw_pair_density) with the conduction bands two to a complex band
 * (c_2j + i c_2j+1): M is linear in the conduction state and real, so the
 * complex result for (v, j) is M_v,2j + i M_v,2j+1, half the transforms of
 * one band at a time.  The complex copies and that complex M are held in a
 * second handle buffer of 16 (nk (nv + ceil(nc/2)) ngw + nk nv ceil(nc/2) ng)
 * bytes.  Errors as bgw_pair_density. */
int bgw_pair_density_real(bgw_handle_t h, const bgw_pair_desc *d, double *M, void *stream);

/* bgw_chi0 for real M: q[i].M is DEVICE f64 [K][ng], q[i].chi DEVICE f64
 * [nw][ng][ng] (real symmetric, written in full); FP64 on the imaginary axis
 * only (BGW_ERR_UNSUPPORTED otherwise), no graph capture, `head` ignored.
 * One weights launch, one persistent real rank-K-update launch over every
 * (q, frequency, K range, 128 x 128 upper tile) item, one finalize. */
int bgw_chi0_real(bgw_handle_t h, const bgw_chi_desc *d, void *stream);

/* Device workspace bgw_chi0_real(h, d, ...) needs, in bytes (HOST *bytes).
 * Allocates nothing. */
int bgw_chi0_real_workspace(bgw_handle_t h, const bgw_chi_desc *d, size_t *bytes);

/* Real coefficients from complex ones (the same section): a plane-wave code
 * returns a non-degenerate state as real times a global phase, and a group
 * of d degenerate states as any orthonormal basis of its subspace; the real
 * and imaginary parts of the group's states then span d real dimensions.
 * Bands of one k whose energies differ by at most tol from their neighbour
 * form a group; Gram-Schmidt over the group's 2d vectors Re c_b, Im c_b (in
 * that order), the remaining vector of largest norm first (lowest index on
 * ties), gives its d real orthonormal states (for one state: the phase
 * divided out, up to sign).
 * c: DEVICE complex128 [nk][nb][ngw]; e: HOST f64 [nk][nb], ascending within
 * each k; r: DEVICE f64 [nk][nb][ngw], output (not aliasing c); nbad:
 * DEVICE int32 [1], set to the number of groups that were not real up to a
 * unitary (more than d real dimensions left a norm above 1e-6, or fewer than
 * d were found).  BGW_ERR_ARG for bad arguments or unsorted energies,
 * BGW_ERR_UNSUPPORTED for a group of more than 32 states (both checked
 * before the handle).  Workspace: 16 nk nb ngw bytes plus the group table,
 * which is uploaded on `stream`; the call waits for that upload, so the
 * stream's earlier work finishes before it returns. */
int bgw_realify(bgw_handle_t h, int nk, int nb, int ngw, const double *c, const double *e, double tol, double *r,
                int *nbad, void *stream);

/* Device workspace bgw_realify(h, nk, nb, ngw, e, tol, ...) needs, in bytes
 * (HOST *bytes).  Allocates nothing. */
int bgw_realify_workspace(bgw_handle_t h, int nk, int nb, int ngw, const double *e, double tol, size_t *bytes);

/* ------------------------------------------------------------------------
 * Exchange kernel of the Bethe-Salpeter equation
 *
 *   Kx[t][t'] = prefactor * sum over G != G0 of conj(M_t(G)) v(q+G) M_t'(G)
 *
 * (optical-properties section, exchange-term equation) for the pairs
 * t = (k, v, c) of the matrix elements M_vc(k, q, G) of bgw_pair_density.
 * It is the chi sum with the roles of pairs and G exchanged: M is
 * transposed into the workspace (G becomes the contraction index, the G0
 * row zeroed) and the chi-sum kernels run with the weights v, FP64 or split
 * BF16 as in bgw_chi0.  Kx is Hermitian positive semidefinite for v > 0.
 * The split form scales its digits per run of 96 consecutive G vectors, so a
 * term orders of magnitude above its neighbours (v(q0+0) ~ 1/q0^2 at small q
 * with head = -1) costs digits of the whole run: leave G = 0 out through
 * `head`, or use FP64, when v has such a term.
 * ---------------------------------------------------------------------- */
typedef struct {
    const double *M;     /* DEVICE complex128 [K][ng], e.g. from bgw_pair_density */
    long long K;         /* pairs, 1 .. 65536 */
    int ng;              /* G vectors, >= 1 */
    int head;            /* index of G = 0 in the G list (its term is left out), -1: keep all */
    const double *v;     /* DEVICE f64 [ng]: v(q+G), e.g. from bgw_vcoul_bulk */
    double prefactor;    /* scale of the sum */
    int precision;       /* BGW_FP64 or BGW_SPLIT_BF16 */
    int pad;             /* unused, 0 */
    double *kx;          /* DEVICE complex128 [K][K], output, written in full */
} bgw_kx_desc;

/* Work is ordered on `stream`; the handle's workspace holds the transposed M
 * (16 K ng bytes) and what the chi sum needs.  Errors as bgw_chi0. */
int bgw_bse_kx(bgw_handle_t h, const bgw_kx_desc *d, void *stream);

/* Device workspace bgw_bse_kx(h, d, ...) needs, in bytes (HOST *bytes).
 * Allocates nothing. */
int bgw_bse_kx_workspace(bgw_handle_t h, const bgw_kx_desc *d, size_t *bytes);

/* ------------------------------------------------------------------------
 * Static self-energy matrix elements of one q (self-energy section)
 *
 * With M[i][n][G] = M_{n''n}(G) for inner states i = n'' and outer states n
 * (bgw_pair_density with nk = 1, the inner states as its "valence" set at
 * k - q and the outer states as its "conduction" set at k, on the G list
 * that carries the sign convention of the equations):
 *   BGW_SIGMA_X   bare exchange (hf-x equation)
 *       S[n][n'] = -pf sum_i sum_{G != head} conj(M[i][n][G]) v(G) M[i][n'][G]
 *   BGW_SIGMA_SX  screened exchange (cohsex-sx equation)
 *       S[n][n'] = -pf sum_i sum_{G,G'} conj(M[i][n][G]) einv[G][G'] v(G') M[i][n'][G']
 *   BGW_SIGMA_CH  Coulomb hole, sum over states (cohsex-ch-sum equation)
 *       S[n][n'] = pf/2 sum_i sum_{G,G'} conj(M[i][n][G]) (einv[G][G'] - delta) v(G') M[i][n'][G']
 * The caller passes the occupied inner states for X and SX, all inner states
 * for CH, and sums the q terms (accumulate).  X runs on the chi-sum kernels
 * (contraction over (i, G), FP64 or split BF16); SX and CH form W M with an
 * FP64 MFMA product, regroup it by inner state and contract over (i, G).
 * ---------------------------------------------------------------------- */
#define BGW_SIGMA_X 0
#define BGW_SIGMA_SX 1
#define BGW_SIGMA_CH 2

typedef struct {
    const double *M;      /* DEVICE complex128 [ninner][nouter][ng] */
    int ninner, nouter;   /* inner states (>= 1), outer states (1 .. 65536) */
    int ng;               /* G vectors, 1 .. 12288 */
    int kind;             /* BGW_SIGMA_X, BGW_SIGMA_SX or BGW_SIGMA_CH */
    int head;             /* BGW_SIGMA_X: index of G = 0 left out, -1 none; ignored otherwise */
    int precision;        /* BGW_SIGMA_X: BGW_FP64 or BGW_SPLIT_BF16; SX and CH: BGW_FP64 */
    const double *v;      /* DEVICE f64 [ng]: v(q+G) */
    const double *epsinv; /* DEVICE complex128 [ng][ng]: eps^-1(q; 0) for SX and CH, NULL for X */
    double prefactor;     /* pf */
    int accumulate;       /* 0: sigma = term; 1: sigma += term */
    int pad;              /* unused, 0 */
    double *sigma;        /* DEVICE complex128 [nouter][nouter], output */
} bgw_sigma_desc;

/* Work is ordered on `stream`; the handle's workspace holds the operands.
 * Errors as bgw_chi0 (BGW_ERR_ARG for a bad kind, size or null pointer,
 * BGW_ERR_UNSUPPORTED for split precision with SX or CH). */
int bgw_sigma(bgw_handle_t h, const bgw_sigma_desc *d, void *stream);

/* Device workspace bgw_sigma(h, d, ...) needs, in bytes (HOST *bytes).
 * Allocates nothing. */
int bgw_sigma_workspace(bgw_handle_t h, const bgw_sigma_desc *d, size_t *bytes);

/* ------------------------------------------------------------------------
 * Dielectric matrix and its inverse
 *
 * epsilon_GG'(omega) = delta_GG' - v(q+G) chi_GG'(omega)   (epsilon section,
 * dielectric-matrix equation, asymmetric Coulomb form), then epsilon^-1 by
 * elimination with partial pivoting (the paper inverts with ZGESV).  The
 * pivot sequence is that of LU with partial pivoting (largest |Re|+|Im|,
 * first index on ties).  info[w] = 0 on success, i > 0 if the i-th pivot
 * (1-based) is exactly zero; epsinv[w] is then unspecified; info[w] = -1000
 * if an internal wait between workgroups gave up (the call still returns).
 * ng is 1 .. 12288.  For ng <= 1536 each panel is eliminated by one
 * workgroup per matrix; the environment variable BGW_GJE_PATH=coop selects
 * the cooperative multi-workgroup panels used above that size (same results
 * to rounding).
 * ---------------------------------------------------------------------- */
/* vcoul: DEVICE f64 [ng]; chi: DEVICE complex128 [nw][ng][ng];
 * epsinv: DEVICE complex128 [nw][ng][ng], may be the same pointer as chi
 * (in-place); info: DEVICE int32 [nw]. */
int bgw_eps_inv(bgw_handle_t h, int ng, int nw, const double *vcoul, const double *chi,
                double *epsinv, int *info, void *stream);

/* bgw_eps_inv for chi Hermitian and negative semidefinite, as chi0 is at
 * zero and at imaginary frequency (every weight of the chi sum is negative),
 * with v > 0.  Then epsilon = S (1 - S chi S) S^-1 with S = diag(v^1/2), the
 * middle factor Hermitian with eigenvalues >= 1, so every elimination pivot
 * is real and >= 1 and the elimination needs no row interchanges: only the
 * 64 x 64 diagonal block of each panel is eliminated column by column, the
 * rest is parallel.  Same arguments and results (to rounding) as
 * bgw_eps_inv.  The precondition is checked: info[w] = -2 when chi[w] is
 * not Hermitian to 1e-8 relative on the scale sqrt(v_G v_G') (or some v <= 0,
 * or a value is not finite), -3 when a pivot has real part below 1/2 or is
 * not real to half of that (chi not negative semidefinite); epsinv[w] is
 * then unspecified and the caller inverts the original chi with
 * bgw_eps_inv.  That fallback needs chi intact: an in-place call (epsinv ==
 * chi) has overwritten it with epsilon, so a caller that may need the
 * fallback passes a separate epsinv. */
int bgw_eps_inv_nsd(bgw_handle_t h, int ng, int nw, const double *vcoul, const double *chi, double *epsinv,
                    int *info, void *stream);

/* Device workspace bgw_eps_inv(h, ng, nw, ...) or bgw_eps_inv_nsd(h, ng, nw,
 * ...) needs, in bytes (HOST *bytes).  Allocates nothing. */
int bgw_eps_inv_workspace(bgw_handle_t h, int ng, int nw, size_t *bytes);

/* bgw_eps_inv for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, kernels and results as bgw_eps_inv; it calls no hipMalloc,
 * hipFree or allocating library routine and records no timings.  Its scratch
 * is a fixed 32 MiB device array inside the library, one per device, held
 * until the process ends (its address is taken by bgw_create); the matrices
 * are inverted in launches of as many as that scratch holds.  Fails with
 * BGW_ERR_UNSUPPORTED if one matrix needs more (not the case for ng <= 12288:
 * about 1 KiB per unit of ng below 3000, 2 KiB from there).  Every call on one device shares that
 * device's scratch: calls that overlap on one device (other streams, other
 * threads, other handles) race and must be serialised by the caller. */
int bgw_eps_inv_noalloc(bgw_handle_t h, int ng, int nw, const double *vcoul, const double *chi,
                        double *epsinv, int *info, void *stream);

/* ------------------------------------------------------------------------
 * Per-kernel timing.  When enabled, every kernel launch (or launch group)
 * of the compute calls is bracketed by HIP events recorded on the call's
 * stream.  bgw_get_timing waits for the recorded events, adds their elapsed
 * times to the kernel's totals and returns the totals since the last reset.
 * ---------------------------------------------------------------------- */
#define BGW_KERNEL_BAND 0        /* band G -> r transforms */
#define BGW_KERNEL_PAIR 1        /* pair product + z/y FFTs (+ x and gather when single-pass) */
#define BGW_KERNEL_WEIGHTS 2     /* energy weights */
#define BGW_KERNEL_HERK 3        /* FP64 chi-sum (rank-K update) */
#define BGW_KERNEL_FINALIZE 4    /* split reduction, prefactor, Hermitian mirror */
#define BGW_KERNEL_SPLIT_SLICE 5 /* BF16 slicing of M (split precision) */
#define BGW_KERNEL_SPLIT_HERK 6  /* BF16 chi-sum with FP64 recombination */
#define BGW_KERNEL_HEADWING 7    /* FP64 head/wing row of chi (split precision) */
#define BGW_KERNEL_EPS_BUILD 8   /* epsilon = 1 - v chi */
#define BGW_KERNEL_INVERT 9      /* whole epsilon inversion (all panels) */
#define BGW_KERNEL_PAIR_X 10     /* x pass + sphere gather of the two-pass pair transform */
#define BGW_KERNEL_COUNT 11

int bgw_set_timing(bgw_handle_t h, int enable);
/* total_ms and launches may be NULL.  Unknown kernel id: BGW_ERR_ARG. */
int bgw_get_timing(bgw_handle_t h, int kernel, double *total_ms, long long *launches);
int bgw_reset_timing(bgw_handle_t h);

/* Host helper: the real-frequency grid of a full-frequency calculation
 * (epsilon section, frequency-grid figure): E = 0, spacing, 2 spacing, ...
 * up to low_cutoff, then each step longer than the previous one by
 * `increment`, up to high_cutoff (all in eV).  Writes min(maxn, count)
 * points to E (HOST, may be NULL when maxn = 0) and the count to *n.
 * BGW_ERR_ARG for spacing <= 0, negative cutoffs or increment, or
 * high_cutoff < low_cutoff. */
int bgw_ff_grid(double spacing, double low_cutoff, double high_cutoff, double increment, int maxn, double *E, int *n);

/* Host helper: bulk bare Coulomb v(q+G) = 4 pi / |q+G|^2 (epsilon section,
 * untruncated bare-Coulomb equation).  bvec: HOST f64 [3][3], rows are the
 * reciprocal lattice vectors in bohr^-1; q: HOST f64 [3] in crystal units;
 * ge: HOST int32 [ng][3]; v: HOST f64 [ng].  BGW_ERR_SHAPE if |q+G| = 0. */
int bgw_vcoul_bulk(const double *bvec, const double *q, int ng, const int *ge, double *v);

#ifdef __cplusplus
}
#endif
#endif /* BGW_H */
