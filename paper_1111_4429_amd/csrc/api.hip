// C-ABI entry points (include/bgw.h): argument validation, the handle with its
// workspace and plan cache, and the sequencing of the kernels on the caller's
// stream.  No arithmetic of the method happens on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "handle.h"

namespace bgw {

// ---- kernels' launchers (fft.hip, chi.hip, eps.hip)
size_t band_lds_bytes(const AxisPlan &, const AxisPlan &, const AxisPlan &, int bwz, int lc);
size_t pair_lds_bytes(const AxisPlan &, const AxisPlan &, const AxisPlan &, int bez, int lc);
int launch_band_to_real(const double2 *C, int nbands, int ngw, const AxisPlan &, const AxisPlan &,
                        const AxisPlan &, const SphereMaps &, int lc, double2 *grids, hipStream_t);
int launch_pair_fft(const double2 *gv, const double2 *gc, int nkb, int nv, int nc, const AxisPlan &,
                    const AxisPlan &, const AxisPlan &, const SphereMaps &, int lc, double2 *M, long long row0,
                    hipStream_t);
size_t pair_yz_bytes_per_pair(int n1, int rey, int rez);
size_t band_lines_bytes(const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz, const SphereMaps &sm,
                        int nbands);
bool band_lines_supported(const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz, const SphereMaps &sm);
int launch_band_lines(const double2 *C, int nbands, int ngw, const AxisPlan &px, const AxisPlan &py,
                      const AxisPlan &pz, const SphereMaps &sm, double2 *W, double2 *grids, hipStream_t st);
bool pair_two_pass_supported(const AxisPlan &py, const AxisPlan &pz);
int launch_pair_yz(const double2 *gv, const double2 *gc, int nkb, int nv, int nc, int c0, int ncb,
                   const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz, int rey, int rez, double2 *T,
                   hipStream_t st);
int launch_pair_yzr(const double2 *gv, const double2 *gc, int nkb, int nv, int nc, int c0, int ncb,
                    const AxisPlan &px, const AxisPlan &py, const AxisPlan &pz, int rey, int rez, double2 *T,
                    hipStream_t st);
int launch_pair_x(const double2 *T, long long npairs, const AxisPlan &px, int rey, int rez, const int *ge_code2,
                  const int *ge_out, int ng, double2 *M, int nv, int nc, int c0, int ncb, long long row0, size_t N,
                  bool yfast, hipStream_t st);
int launch_band_to_real2(const double2 *C, int nbands, int ngw, const AxisPlan &, const AxisPlan &,
                         const AxisPlan &, const SphereMaps &, int rwy, double2 *grids, hipStream_t);
int launch_eps_build(const double2 *chi, const double *v, int ng, int nw, double2 *eps, hipStream_t);
size_t gje_workspace_bytes(int n, int nmat, int R);
int gje_rows_per_wg(int n);
int gje_max_group(int n);
int launch_gje_invert(double2 *A, int n, int nmat, int *info, void *ws, int *ipiv_ws, hipStream_t);
size_t nsd_workspace_bytes(int n, int nmat, int nall);
int launch_nsd_check(const double2 *chi, const double *v, int n, int nall, int nmat, void *ws, hipStream_t);
int launch_nsd_invert(double2 *A, int n, int nmat, int m0, int nall, int *info, void *ws, hipStream_t);

namespace {
thread_local std::string g_err;
constexpr size_t kLdsBudget = 150 * 1024;

// Fixed device scratch of the allocation-free inversion (bgw_eps_inv_noalloc).
// Each device that loads the library holds its own copy until the process
// ends.  In host code `scratch` is only the symbol's host stand-in: its
// device address is looked up once per device (scratch_setup, called from
// bgw_create with the device current) and only that address is passed on.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
}  // namespace

void set_error(const std::string &msg) { g_err = msg; }
void clear_error() { g_err.clear(); }

int fail(int code, const std::string &msg) {
    set_error(msg);
    return code;
}

// ---------------------------------------------------------------- validation (host only)

bool is_2a3b(int n) {
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

static int check_glist(const int *g, int count, const int n[3], const char *what, int maxabs[3]) {
    maxabs[0] = maxabs[1] = maxabs[2] = 0;
    std::vector<long long> keys((size_t)count);
    for (int i = 0; i < count; ++i) {
        long long key = 0;
        for (int d = 0; d < 3; ++d) {
            const int m = g[3 * i + d];
            if (m < -n[d] / 2 || m >= n[d] - n[d] / 2)
                return fail(BGW_ERR_SHAPE, std::string(what) + ": Miller index outside [-n/2, n/2)");
            maxabs[d] = std::max(maxabs[d], std::abs(m));
            key = key * 512 + (m + 256);
        }
        keys[(size_t)i] = key;
    }
    std::sort(keys.begin(), keys.end());
    if (std::adjacent_find(keys.begin(), keys.end()) != keys.end())
        return fail(BGW_ERR_SHAPE, std::string(what) + ": duplicate G-vector");
    return BGW_OK;
}

}  // namespace bgw

using namespace bgw;

namespace bgw {
static void transform_box(const bgw_pair_desc *d, int box[3]);
// Largest caller grid per axis; the transform itself runs on the smallest
// alias-free box, which must fit the transform kernels (kMaxFFT per axis).
constexpr int kMaxGrid = 1024;
}  // namespace bgw

extern "C" int bgw_pair_desc_check(const bgw_pair_desc *d) {
    clear_error();
    if (!d) return fail(BGW_ERR_ARG, "null descriptor");
    for (int i = 0; i < 3; ++i) {
        if (d->n[i] < 1) return fail(BGW_ERR_ARG, "FFT grid dimensions must be positive");
        if (!is_2a3b(d->n[i]) || d->n[i] < 4 || d->n[i] > kMaxGrid)
            return fail(BGW_ERR_UNSUPPORTED, "FFT grid dimensions must be 2^a 3^b in [4, 1024]");
    }
    if (d->ngw < 1 || d->ng < 1 || d->nk < 1 || d->nv < 1 || d->nc < 1)
        return fail(BGW_ERR_ARG, "ngw, ng, nk, nv, nc must be >= 1");
    if (!d->gw || !d->ge || !d->cv || !d->cc) return fail(BGW_ERR_ARG, "null pointer in descriptor");
    if (d->ng > kMaxNg) return fail(BGW_ERR_UNSUPPORTED, "dielectric sphere larger than 12288 G-vectors");
    int mw[3], me[3];
    BGW_TRY(check_glist(d->gw, d->ngw, d->n, "wavefunction sphere", mw));
    BGW_TRY(check_glist(d->ge, d->ng, d->n, "dielectric sphere", me));
    for (int i = 0; i < 3; ++i)
        if (d->n[i] <= 2 * mw[i] + me[i])
            return fail(BGW_ERR_ALIAS, "FFT grid too small: need n_i > 2 max|gw_i| + max|ge_i| on every axis");
    int box[3];
    transform_box(d, box);
    for (int i = 0; i < 3; ++i)
        if (box[i] > kMaxFFT)
            return fail(BGW_ERR_UNSUPPORTED, "the alias-free transform box needs more than 128 points on an axis");
    return BGW_OK;
}

extern "C" int bgw_vcoul_bulk(const double *bvec, const double *q, int ng, const int *ge, double *v) {
    clear_error();
    if (!bvec || !q || !ge || !v || ng < 1) return fail(BGW_ERR_ARG, "bad arguments to bgw_vcoul_bulk");
    for (int g = 0; g < ng; ++g) {
        double x[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < 3; ++i) {
            const double m = q[i] + ge[3 * g + i];
            for (int c = 0; c < 3; ++c) x[c] += m * bvec[3 * i + c];
        }
        const double q2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
        if (!(q2 > 0.0)) return fail(BGW_ERR_SHAPE, "|q+G| = 0 in bgw_vcoul_bulk");
        v[g] = 4.0 * M_PI / q2;
    }
    return BGW_OK;
}

extern "C" int bgw_ff_grid(double spacing, double low_cutoff, double high_cutoff, double increment, int maxn,
                           double *E, int *n) {
    clear_error();
    if (!(spacing > 0.0) || !(low_cutoff >= 0.0) || !(high_cutoff >= low_cutoff) || !(increment >= 0.0) || !n ||
        maxn < 0 || (maxn > 0 && !E))
        return fail(BGW_ERR_ARG, "bad frequency-grid parameters");
    const double tol = 1e-12;
    // uniform part: i * spacing up to the low cutoff
    const long long nu = (long long)std::floor(low_cutoff / spacing * (1.0 + tol)) + 1;
    std::vector<double> g;
    for (long long i = 0; i < nu; ++i) g.push_back((double)i * spacing);
    // then every step longer than the previous one by `increment`
    double step = spacing, last = g.back();
    if (increment > 0.0 || last + step <= high_cutoff * (1.0 + tol)) {
        for (;;) {
            step += increment;
            const double nx = last + step;
            if (nx > high_cutoff * (1.0 + tol)) break;
            g.push_back(nx);
            last = nx;
            if (g.size() > 100000000) return fail(BGW_ERR_ARG, "frequency grid larger than 1e8 points");
        }
    }
    *n = (int)g.size();
    for (int i = 0; i < std::min<int>(maxn, (int)g.size()); ++i) E[i] = g[(size_t)i];
    return BGW_OK;
}

extern "C" int bgw_version(void) { return 200; }

extern "C" const char *bgw_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------- handle, plans, workspace

namespace bgw {

static int upload(FFTPlan &pl, const void *host, size_t bytes, const void **dev) {
    auto b = std::make_unique<DevBuf>();
    BGW_HIP(hipMalloc(&b->p, std::max<size_t>(bytes, 16)));
    b->bytes = bytes;
    if (bytes) BGW_HIP(hipMemcpy(b->p, host, bytes, hipMemcpyHostToDevice));
    *dev = b->p;
    pl.bufs.push_back(std::move(b));
    return BGW_OK;
}

static void radices(int n, int *nrad, int *rad) {
    int k = 0;
    while (n % 4 == 0) { rad[k++] = 4; n /= 4; }
    while (n % 2 == 0) { rad[k++] = 2; n /= 2; }
    while (n % 3 == 0) { rad[k++] = 3; n /= 3; }
    *nrad = k;
}

static size_t env_limit() {
    const char *s = std::getenv("BGW_WORKSPACE_LIMIT");
    if (!s || !*s) return (size_t)-1;
    return (size_t)std::strtoull(s, nullptr, 10);
}

int ensure_ws(bgw_handle_t h, size_t bytes, hipStream_t st) {
    if (h->ws.bytes >= bytes) return BGW_OK;
    if (bytes > env_limit()) return fail(BGW_ERR_NOMEM, "workspace request exceeds BGW_WORKSPACE_LIMIT");
    BGW_HIP(hipStreamSynchronize(st));
    if (h->ws.p) {
        BGW_HIP(hipFree(h->ws.p));
        h->ws.p = nullptr;
        h->ws.bytes = 0;
    }
    if (hipMalloc(&h->ws.p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        h->ws.p = nullptr;
        return fail(BGW_ERR_NOMEM, "device workspace allocation failed (" + std::to_string(bytes) + " bytes)");
    }
    h->ws.bytes = bytes;
    return BGW_OK;
}

// Transform box: the matrix element is the integral of the matrix-element
// equation, and the discrete transform reproduces it exactly on any box whose
// every axis satisfies b_i > 2 max|gw_i| + max|ge_i| (no aliasing of the
// product's Fourier components onto the dielectric sphere).  The smallest such
// length among those with register-resident kernels (16 .. 128, y and z
// equal) is used when one fits in the caller's grid, else the smallest
// 2^a 3^b length per axis (at most the caller's n_i); BGW_FFT_BOX=full forces
// the caller's grid.
static void transform_box(const bgw_pair_desc *d, int box[3]) {
    const char *env = std::getenv("BGW_FFT_BOX");
    const bool full = env && std::strcmp(env, "full") == 0;
    int mw[3] = {0, 0, 0}, me[3] = {0, 0, 0};
    for (int g = 0; g < d->ngw; ++g)
        for (int a = 0; a < 3; ++a) mw[a] = std::max(mw[a], std::abs(d->gw[3 * g + a]));
    for (int g = 0; g < d->ng; ++g)
        for (int a = 0; a < 3; ++a) me[a] = std::max(me[a], std::abs(d->ge[3 * g + a]));
    if (full) {
        for (int a = 0; a < 3; ++a) box[a] = d->n[a];
        return;
    }
    int need[3];
    for (int a = 0; a < 3; ++a) need[a] = std::max(4, 2 * mw[a] + me[a] + 1);
    // lengths with register-resident transform kernels (equal y and z for the two-pass pair transform)
    static const int kFast[] = {16, 24, 32, 48, 64, 96, 128};
    auto fast_at_least = [](int lo, int hi) {
        for (int f : kFast)
            if (f >= lo && f <= hi) return f;
        return 0;
    };
    const int fx = fast_at_least(need[0], d->n[0]);
    const int fyz = fast_at_least(std::max(need[1], need[2]), std::min(d->n[1], d->n[2]));
    if (fx && fyz) {
        box[0] = fx;
        box[1] = box[2] = fyz;
        return;
    }
    for (int a = 0; a < 3; ++a) {
        int b = need[a];
        while (!is_2a3b(b)) ++b;
        box[a] = std::min(b, d->n[a]);
    }
}

static std::string plan_key(const bgw_pair_desc *d) {
    // grid + exact G lists (FNV-1a over the index bytes)
    unsigned long long hw = 1469598103934665603ull, he = hw;
    const unsigned char *pw = reinterpret_cast<const unsigned char *>(d->gw);
    for (size_t i = 0; i < sizeof(int) * 3 * (size_t)d->ngw; ++i) hw = (hw ^ pw[i]) * 1099511628211ull;
    const unsigned char *pe = reinterpret_cast<const unsigned char *>(d->ge);
    for (size_t i = 0; i < sizeof(int) * 3 * (size_t)d->ng; ++i) he = (he ^ pe[i]) * 1099511628211ull;
    int box[3];
    transform_box(d, box);
    return std::to_string(box[0]) + "x" + std::to_string(box[1]) + "x" + std::to_string(box[2]) + ":" +
           std::to_string(d->ngw) + ":" + std::to_string(hw) + ":" + std::to_string(d->ng) + ":" + std::to_string(he);
}

static int get_plan(bgw_handle_t h, const bgw_pair_desc *d, FFTPlan **out) {
    const std::string key = plan_key(d);
    auto it = h->plans.find(key);
    if (it != h->plans.end()) {
        *out = it->second.get();
        return BGW_OK;
    }
    auto pl = std::make_unique<FFTPlan>();
    transform_box(d, pl->box);
    // twiddles exp(+2 pi i j / n), evaluated in long double and rounded once
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int a = 0; a < 3; ++a) {
        const int n = pl->box[a];
        std::vector<double2> tw((size_t)n);
        for (int j = 0; j < n; ++j) {
            const long double ang = 2.0L * pi * (long double)j / (long double)n;
            tw[(size_t)j] = make_double2((double)cosl(ang), (double)sinl(ang));
        }
        pl->ax[a].n = n;
        radices(n, &pl->ax[a].nrad, pl->ax[a].rad);
        const void *dp = nullptr;
        BGW_TRY(upload(*pl, tw.data(), sizeof(double2) * n, &dp));
        pl->ax[a].tw = (const double2 *)dp;
    }
    const int n1 = pl->box[0], n2 = pl->box[1];
    auto mod = [](int m, int n) { return ((m % n) + n) % n; };
    // wavefunction sticks along x, keyed by (my, mz), entries in ascending G order
    int rwz = 0, rwy = 0;
    for (int g = 0; g < d->ngw; ++g) {
        rwz = std::max(rwz, std::abs(d->gw[3 * g + 2]));
        rwy = std::max(rwy, std::abs(d->gw[3 * g + 1]));
    }
    std::map<std::pair<int, int>, std::vector<int>> sticks;
    for (int g = 0; g < d->ngw; ++g) sticks[{d->gw[3 * g + 1], d->gw[3 * g + 2]}].push_back(g);
    std::vector<int> start, sg, smx, syz, syz2;
    start.push_back(0);
    for (auto &kv : sticks) {
        for (int g : kv.second) {
            sg.push_back(g);
            smx.push_back(mod(d->gw[3 * g], n1));
        }
        start.push_back((int)sg.size());
        syz.push_back(mod(kv.first.first, n2) | ((kv.first.second + rwz) << 16));
        syz2.push_back((kv.first.first + rwy) | ((kv.first.second + rwz) << 16));
    }
    // the same sticks with entries in ascending mx, and the (my, mz) box cells
    const int bwy_ = 2 * rwy + 1, bwz_ = 2 * rwz + 1;
    std::vector<int> cell((size_t)bwy_ * bwz_, -1), slo, sgs;
    bool contiguous = true;
    int rwx = 0;
    {
        int s = 0;
        for (auto &kv : sticks) {
            std::vector<std::pair<int, int>> e;
            for (int g : kv.second) {
                e.push_back({d->gw[3 * g], g});
                rwx = std::max(rwx, std::abs(d->gw[3 * g]));
            }
            std::sort(e.begin(), e.end());
            for (size_t i = 0; i < e.size(); ++i) {
                if (i && e[i].first != e[i - 1].first + 1) contiguous = false;
                sgs.push_back(e[i].second);
            }
            slo.push_back(e.front().first);
            cell[(size_t)(kv.first.second + rwz) * bwy_ + (kv.first.first + rwy)] = s;
            ++s;
        }
    }
    if (2 * rwx + 1 > n1 || bwy_ > n2 || bwz_ > pl->box[2]) contiguous = false;
    SphereMaps &sm = pl->sm;
    sm.nstick = (int)syz.size();
    sm.rwz = rwz;
    sm.bwz = 2 * rwz + 1;
    const void *dp = nullptr;
    BGW_TRY(upload(*pl, start.data(), sizeof(int) * start.size(), &dp));
    sm.stick_start = (const int *)dp;
    BGW_TRY(upload(*pl, sg.data(), sizeof(int) * sg.size(), &dp));
    sm.stick_g = (const int *)dp;
    BGW_TRY(upload(*pl, smx.data(), sizeof(int) * smx.size(), &dp));
    sm.stick_mx = (const int *)dp;
    BGW_TRY(upload(*pl, syz.data(), sizeof(int) * syz.size(), &dp));
    sm.stick_yz = (const int *)dp;
    BGW_TRY(upload(*pl, syz2.data(), sizeof(int) * syz2.size(), &dp));
    sm.stick_yz2 = (const int *)dp;
    sm.rwy = rwy;
    sm.ncell = bwy_ * bwz_;
    sm.sticks_contiguous = contiguous;
    BGW_TRY(upload(*pl, cell.data(), sizeof(int) * cell.size(), &dp));
    sm.cell_stick = (const int *)dp;
    BGW_TRY(upload(*pl, slo.data(), sizeof(int) * slo.size(), &dp));
    sm.st_lo = (const int *)dp;
    BGW_TRY(upload(*pl, sgs.data(), sizeof(int) * sgs.size(), &dp));
    sm.st_gs = (const int *)dp;
    int rez = 0, rey = 0;
    for (int g = 0; g < d->ng; ++g) {
        rez = std::max(rez, std::abs(d->ge[3 * g + 2]));
        rey = std::max(rey, std::abs(d->ge[3 * g + 1]));
    }
    std::vector<int> code((size_t)d->ng), code2((size_t)d->ng), order((size_t)d->ng);
    for (int g = 0; g < d->ng; ++g) {
        code[(size_t)g] = mod(d->ge[3 * g], n1) | (mod(d->ge[3 * g + 1], n2) << 8) | ((d->ge[3 * g + 2] + rez) << 16);
        order[(size_t)g] = g;
    }
    // accumulation order of the fast pair kernel: by (mx, my, mz)
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        for (int c = 0; c < 3; ++c)
            if (d->ge[3 * a + c] != d->ge[3 * b + c]) return d->ge[3 * a + c] < d->ge[3 * b + c];
        return false;
    });
    for (int p = 0; p < d->ng; ++p) {
        const int g = order[(size_t)p];
        code2[(size_t)p] = mod(d->ge[3 * g], n1) | ((d->ge[3 * g + 1] + rey) << 8) | ((d->ge[3 * g + 2] + rez) << 16);
    }
    BGW_TRY(upload(*pl, code.data(), sizeof(int) * code.size(), &dp));
    sm.ge_code = (const int *)dp;
    BGW_TRY(upload(*pl, code2.data(), sizeof(int) * code2.size(), &dp));
    sm.ge_code2 = (const int *)dp;
    BGW_TRY(upload(*pl, order.data(), sizeof(int) * order.size(), &dp));
    sm.ge_out = (const int *)dp;
    sm.rey = rey;
    sm.ng = d->ng;
    sm.rez = rez;
    sm.bez = 2 * rez + 1;
    *out = pl.get();
    h->plans[key] = std::move(pl);
    return BGW_OK;
}

static int pick_lc(int n2, int n3, size_t fixed_bytes) {
    // lines per z chunk: all n2 if the LDS budget allows
    if (fixed_bytes >= kLdsBudget) return 0;
    const size_t per_line = 2 * sizeof(double2) * (size_t)n3;
    const int lc = (int)std::min<size_t>(n2, (kLdsBudget - fixed_bytes) / per_line);
    return lc;
}

// BGW_GENERIC_FFT=1 forces the generic (any 2^a 3^b length) transform kernels.
static bool generic_fft() {
    const char *s = std::getenv("BGW_GENERIC_FFT");
    return s && *s == '1';
}

int set_device(bgw_handle_t h) {
    BGW_HIP(hipSetDevice(h->device));
    return BGW_OK;
}

}  // namespace bgw

namespace {
// Device address of `scratch` on device dev, looked up once with dev current.
int scratch_setup(int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return BGW_OK;
    int prev = 0;
    BGW_HIP(hipGetDevice(&prev));
    BGW_HIP(hipSetDevice(dev));
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    (void)hipSetDevice(prev);
    if (e != hipSuccess || !ptr)
        return fail(BGW_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
    return BGW_OK;
}
}  // namespace

extern "C" int bgw_create(bgw_handle_t *h, int hip_device) {
    clear_error();
    if (!h) return fail(BGW_ERR_ARG, "null handle pointer");
    *h = nullptr;
    int count = 0;
    BGW_HIP(hipGetDeviceCount(&count));
    if (hip_device < 0 || hip_device >= count) return fail(BGW_ERR_ARG, "no such HIP device");
    if (hip_device >= kMaxDevices) return fail(BGW_ERR_UNSUPPORTED, "device index beyond 63");
    BGW_TRY(scratch_setup(hip_device));
    auto *hh = new (std::nothrow) bgw_handle_s();
    if (!hh) return fail(BGW_ERR_NOMEM, "out of host memory");
    hh->device = hip_device;
    *h = hh;
    return BGW_OK;
}

extern "C" int bgw_destroy(bgw_handle_t h) {
    clear_error();
    if (!h) return BGW_OK;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    delete h;
    return BGW_OK;
}

extern "C" size_t bgw_workspace_bytes(bgw_handle_t h) { return h ? h->ws.bytes : 0; }

namespace bgw {

// Everything bgw_pair_density decides on the host before it launches: the
// transform plan, the k- and c-batches and the workspace carve-up.
struct PairRun {
    FFTPlan *pl = nullptr;
    int lcb = 0, lcp = 0, ncb = 0, kb = 0;
    bool two_pass = false, band_lines = false;
    size_t N = 0, t_off = 0, w_off = 0, ws_need = 0;
};

static int plan_pair(bgw_handle_t h, const bgw_pair_desc *d, PairRun &R) {
    FFTPlan *pl = nullptr;
    BGW_TRY(get_plan(h, d, &pl));
    R.pl = pl;
    const AxisPlan &px = pl->ax[0], &py = pl->ax[1], &pz = pl->ax[2];
    const int n2 = pl->box[1], n3 = pl->box[2];
    const size_t fixed_b = band_lds_bytes(px, py, pz, pl->sm.bwz, 0) + sizeof(int) * n3;
    const size_t fixed_p = pair_lds_bytes(px, py, pz, pl->sm.bez, 0);
    R.lcb = pick_lc(n2, n3, fixed_b);
    R.lcp = pick_lc(n2, n3, fixed_p);
    if (R.lcb < 1 || R.lcp < 1) return fail(BGW_ERR_UNSUPPORTED, "FFT grid/sphere too large for the LDS budget");

    const size_t N = (size_t)pl->box[0] * n2 * n3;
    R.N = N;
    const size_t per_k = sizeof(double2) * N * (size_t)(d->nv + d->nc);
    // two-pass transform (y,z pass -> T in workspace -> x pass) on the fast sizes
    const bool two_pass = !generic_fft() && pair_two_pass_supported(py, pz);
    R.two_pass = two_pass;
    const size_t t_per_pair = pair_yz_bytes_per_pair(pl->box[0], pl->sm.rey, pl->sm.rez);
    size_t free_b = 0, total_b = 0;
    BGW_HIP(hipMemGetInfo(&free_b, &total_b));
    const size_t budget = std::min(env_limit(), h->ws.bytes + (size_t)(0.85 * (double)free_b));
    // T for one k-point's pairs of a c-batch is capped at 8 GiB (or a quarter of the budget)
    const size_t t_cap = std::min<size_t>((size_t)8 << 30, budget / 4);
    int ncb = d->nc;
    if (two_pass) {
        ncb = (int)std::max<size_t>(1, std::min<size_t>((size_t)d->nc, t_cap / (t_per_pair * d->nv)));
    }
    R.ncb = ncb;
    const size_t t_bytes_for = two_pass ? t_per_pair * (size_t)d->nv * ncb : 0;  // per k in the batch
    // x-stick results of the lane-per-line band path, reused by the valence and conduction launches
    const bool band_lines = !generic_fft() && band_lines_supported(px, py, pz, pl->sm);
    R.band_lines = band_lines;
    const size_t w_per_k = band_lines ? band_lines_bytes(px, py, pz, pl->sm, std::max(d->nv, d->nc)) : 0;
    int kb = (int)std::min<size_t>((size_t)d->nk, budget / (per_k + t_bytes_for + w_per_k + 1));
    if (kb < 1) return fail(BGW_ERR_NOMEM, "workspace for one k-point of band grids does not fit");
    if (two_pass) kb = (int)std::min<size_t>((size_t)kb, std::max<size_t>(1, t_cap / (t_per_pair * d->nv * ncb)));
    R.kb = kb;
    const size_t grid_bytes = per_k * kb;
    R.t_off = ((grid_bytes + 255) / 256) * 256;
    R.w_off = R.t_off + ((two_pass ? t_bytes_for * kb : 0) + 255) / 256 * 256;
    R.ws_need = R.w_off + w_per_k * kb;
    return BGW_OK;
}

}  // namespace bgw

extern "C" int bgw_pair_density_workspace(bgw_handle_t h, const bgw_pair_desc *d, size_t *bytes) {
    BGW_TRY(bgw_pair_desc_check(d));
    if (!h || !bytes) return fail(BGW_ERR_ARG, "null handle or output");
    BGW_TRY(set_device(h));
    PairRun R;
    BGW_TRY(plan_pair(h, d, R));
    *bytes = R.ws_need;
    return BGW_OK;
}

extern "C" int bgw_pair_density(bgw_handle_t h, const bgw_pair_desc *d, double *M, void *stream) {
    BGW_TRY(bgw_pair_desc_check(d));
    if (!h || !M) return fail(BGW_ERR_ARG, "null handle or output");
    BGW_TRY(set_device(h));
    hipStream_t st = (hipStream_t)stream;
    PairRun R;
    BGW_TRY(plan_pair(h, d, R));
    FFTPlan *pl = R.pl;
    const AxisPlan &px = pl->ax[0], &py = pl->ax[1], &pz = pl->ax[2];
    const int lcb = R.lcb, lcp = R.lcp, ncb = R.ncb, kb = R.kb;
    const bool two_pass = R.two_pass, band_lines = R.band_lines;
    const size_t N = R.N, t_off = R.t_off, w_off = R.w_off;
    BGW_TRY(ensure_ws(h, R.ws_need, st));
    double2 *gv = (double2 *)h->ws.p;
    double2 *T = (double2 *)((char *)h->ws.p + t_off);
    double2 *Wb = (double2 *)((char *)h->ws.p + w_off);
    const double2 *cv = (const double2 *)d->cv, *cc = (const double2 *)d->cc;
    for (int k0 = 0; k0 < d->nk; k0 += kb) {
        const int kn = std::min(kb, d->nk - k0);
        double2 *gc = gv + (size_t)kn * d->nv * N;
        {
            Timed tm(h, BGW_KERNEL_BAND, st);
            const double2 *cvk = cv + (size_t)k0 * d->nv * d->ngw, *cck = cc + (size_t)k0 * d->nc * d->ngw;
            if (band_lines) {
                BGW_TRY(launch_band_lines(cvk, kn * d->nv, d->ngw, px, py, pz, pl->sm, Wb, gv, st));
                BGW_TRY(launch_band_lines(cck, kn * d->nc, d->ngw, px, py, pz, pl->sm, Wb, gc, st));
            } else {
                int rc = generic_fft() ? BGW_ERR_UNSUPPORTED
                                       : launch_band_to_real2(cvk, kn * d->nv, d->ngw, px, py, pz, pl->sm, pl->sm.rwy,
                                                              gv, st);
                if (rc == BGW_ERR_UNSUPPORTED) {
                    BGW_TRY(launch_band_to_real(cvk, kn * d->nv, d->ngw, px, py, pz, pl->sm, lcb, gv, st));
                    BGW_TRY(launch_band_to_real(cck, kn * d->nc, d->ngw, px, py, pz, pl->sm, lcb, gc, st));
                } else {
                    BGW_TRY(rc);
                    BGW_TRY(launch_band_to_real2(cck, kn * d->nc, d->ngw, px, py, pz, pl->sm, pl->sm.rwy, gc, st));
                }
            }
        }
        const long long row0 = (long long)k0 * d->nv * d->nc;
        if (two_pass) {
            for (int c0 = 0; c0 < d->nc; c0 += ncb) {
                const int cn = std::min(ncb, d->nc - c0);
                bool yfast = true;
                {
                    Timed tm(h, BGW_KERNEL_PAIR, st);
                    int rc = launch_pair_yzr(gv, gc, kn, d->nv, d->nc, c0, cn, px, py, pz, pl->sm.rey, pl->sm.rez, T, st);
                    if (rc == BGW_ERR_UNSUPPORTED) {
                        yfast = false;
                        rc = launch_pair_yz(gv, gc, kn, d->nv, d->nc, c0, cn, px, py, pz, pl->sm.rey, pl->sm.rez, T, st);
                    }
                    BGW_TRY(rc);
                }
                Timed tm(h, BGW_KERNEL_PAIR_X, st);
                BGW_TRY(launch_pair_x(T, (long long)kn * d->nv * cn, px, pl->sm.rey, pl->sm.rez, pl->sm.ge_code2,
                                      pl->sm.ge_out, d->ng, (double2 *)M, d->nv, d->nc, c0, cn, row0, N, yfast, st));
            }
        } else {
            Timed tm(h, BGW_KERNEL_PAIR, st);
            BGW_TRY(launch_pair_fft(gv, gc, kn, d->nv, d->nc, px, py, pz, pl->sm, lcp, (double2 *)M, row0, st));
        }
    }
    return BGW_OK;
}

extern "C" int bgw_pair_density_real(bgw_handle_t h, const bgw_pair_desc *d, double *M, void *stream) {
    BGW_TRY(bgw_pair_desc_check(d));
    if (!h || !M) return fail(BGW_ERR_ARG, "null handle or output");
    BGW_TRY(set_device(h));
    hipStream_t st = (hipStream_t)stream;
    // complex copies of the real valence coefficients, the conduction bands two to a
    // complex band, and the complex M of (valence, band pair)
    const int ncp = (d->nc + 1) / 2;
    const long long nvw = (long long)d->nk * d->nv * d->ngw, ncw = (long long)d->nk * ncp * d->ngw;
    const long long nm = (long long)d->nk * d->nv * ncp * d->ng;
    auto al256 = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t off_cc = al256(sizeof(double2) * nvw), off_m = off_cc + al256(sizeof(double2) * ncw);
    const size_t need = off_m + al256(sizeof(double2) * nm);
    if (h->aux.bytes < need) {
        if (need > env_limit()) return fail(BGW_ERR_NOMEM, "real-flavor staging exceeds BGW_WORKSPACE_LIMIT");
        BGW_HIP(hipStreamSynchronize(st));
        if (h->aux.p) BGW_HIP(hipFree(h->aux.p));
        h->aux.p = nullptr;
        h->aux.bytes = 0;
        if (hipMalloc(&h->aux.p, need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(BGW_ERR_NOMEM, "real-flavor staging allocation failed (" + std::to_string(need) + " bytes)");
        }
        h->aux.bytes = need;
    }
    char *a = (char *)h->aux.p;
    BGW_TRY(launch_real_to_complex(d->cv, nvw, (double2 *)a, st));
    BGW_TRY(launch_pack_band_pairs(d->cc, d->nk, d->nc, d->ngw, (double2 *)(a + off_cc), st));
    bgw_pair_desc dc = *d;
    dc.cv = (const double *)a;
    dc.cc = (const double *)(a + off_cc);
    dc.nc = ncp;
    BGW_TRY(bgw_pair_density(h, &dc, (double *)(a + off_m), stream));
    return launch_unpack_pair_halves((const double2 *)(a + off_m), d->nk * d->nv, d->nc, d->ng, M, st);
}


namespace bgw {
// Matrices inverted per cooperative launch and the workspace the inversion needs.
static void eps_plan(int ng, int nw, int *group, size_t *gws, size_t *need) {
    *group = std::max(1, std::min(nw, gje_max_group(ng)));
    const int rows = gje_rows_per_wg(ng);
    const int R = (ng + rows - 1) / rows;
    *gws = gje_workspace_bytes(ng, *group, R);
    *need = *gws + sizeof(int) * 2 * (size_t)*group * ng + 512;
}

// The interchange-free path: up to 64 matrices per group, all nw checked at once.
static int nsd_group(int nw) { return std::max(1, std::min(nw, 64)); }

// Both inversion paths take the larger of their two needs, so that the
// workspace query answers for either call.
static size_t eps_need(int ng, int nw) {
    int group = 0;
    size_t gws = 0, need = 0;
    eps_plan(ng, nw, &group, &gws, &need);
    return std::max(need, nsd_workspace_bytes(ng, nsd_group(nw), nw));
}
}  // namespace bgw

extern "C" int bgw_eps_inv_workspace(bgw_handle_t h, int ng, int nw, size_t *bytes) {
    clear_error();
    if (!h || ng < 1 || nw < 1 || !bytes) return fail(BGW_ERR_ARG, "bad arguments to bgw_eps_inv_workspace");
    if (ng > kMaxNg) return fail(BGW_ERR_UNSUPPORTED, "ng > 12288");
    BGW_TRY(set_device(h));
    *bytes = eps_need(ng, nw);
    return BGW_OK;
}

extern "C" int bgw_eps_inv(bgw_handle_t h, int ng, int nw, const double *vcoul, const double *chi, double *epsinv,
                           int *info, void *stream) {
    clear_error();
    if (!h || ng < 1 || nw < 1 || !vcoul || !chi || !epsinv || !info)
        return fail(BGW_ERR_ARG, "bad arguments to bgw_eps_inv");
    if (ng > kMaxNg) return fail(BGW_ERR_UNSUPPORTED, "ng > 12288");
    BGW_TRY(set_device(h));
    hipStream_t st = (hipStream_t)stream;
    int group = 0;
    size_t gws = 0, need = 0;
    eps_plan(ng, nw, &group, &gws, &need);
    BGW_TRY(ensure_ws(h, eps_need(ng, nw), st));
    int *ipiv = (int *)((char *)h->ws.p + ((gws + 255) / 256) * 256);
    {
        Timed tm(h, BGW_KERNEL_EPS_BUILD, st);
        BGW_TRY(launch_eps_build((const double2 *)chi, vcoul, ng, nw, (double2 *)epsinv, st));
    }
    Timed tm(h, BGW_KERNEL_INVERT, st);
    for (int w0 = 0; w0 < nw; w0 += group) {
        const int gn = std::min(group, nw - w0);
        BGW_TRY(launch_gje_invert((double2 *)epsinv + (size_t)w0 * ng * ng, ng, gn, info + w0, h->ws.p, ipiv, st));
    }
    return BGW_OK;
}

extern "C" int bgw_eps_inv_nsd(bgw_handle_t h, int ng, int nw, const double *vcoul, const double *chi,
                               double *epsinv, int *info, void *stream) {
    clear_error();
    if (!h || ng < 1 || nw < 1 || !vcoul || !chi || !epsinv || !info)
        return fail(BGW_ERR_ARG, "bad arguments to bgw_eps_inv_nsd");
    if (ng > kMaxNg) return fail(BGW_ERR_UNSUPPORTED, "ng > 12288");
    BGW_TRY(set_device(h));
    hipStream_t st = (hipStream_t)stream;
    BGW_TRY(ensure_ws(h, eps_need(ng, nw), st));
    const int group = nsd_group(nw);
    {
        Timed tm(h, BGW_KERNEL_EPS_BUILD, st);
        // chi is read before epsilon overwrites it (the call may be in place)
        BGW_TRY(launch_nsd_check((const double2 *)chi, vcoul, ng, nw, group, h->ws.p, st));
        BGW_TRY(launch_eps_build((const double2 *)chi, vcoul, ng, nw, (double2 *)epsinv, st));
    }
    Timed tm(h, BGW_KERNEL_INVERT, st);
    for (int w0 = 0; w0 < nw; w0 += group) {
        const int gn = std::min(group, nw - w0);
        BGW_TRY(launch_nsd_invert((double2 *)epsinv + (size_t)w0 * ng * ng, ng, gn, w0, nw, info + w0, h->ws.p, st));
    }
    return BGW_OK;
}

extern "C" int bgw_eps_inv_noalloc(bgw_handle_t h, int ng, int nw, const double *vcoul, const double *chi,
                                   double *epsinv, int *info, void *stream) {
    clear_error();
    if (!h || ng < 1 || nw < 1 || !vcoul || !chi || !epsinv || !info)
        return fail(BGW_ERR_ARG, "bad arguments to bgw_eps_inv_noalloc");
    if (ng > kMaxNg) return fail(BGW_ERR_UNSUPPORTED, "ng > 12288");
    BGW_TRY(set_device(h));
    void *ws = g_scratch_ptr[h->device];
    if (!ws) return fail(BGW_ERR_HIP, "no scratch address for this device");
    hipStream_t st = (hipStream_t)stream;
    // as many matrices per launch as bgw_eps_inv takes, cut to what the scratch holds
    int group = 0;
    size_t gws = 0, need = 0;
    eps_plan(ng, nw, &group, &gws, &need);
    while (group > 1 && need > kNoAllocScratchBytes) {
        const int fewer = group - 1;
        eps_plan(ng, fewer, &group, &gws, &need);
    }
    if (need > kNoAllocScratchBytes)
        return fail(BGW_ERR_UNSUPPORTED, "bgw_eps_inv_noalloc: one matrix of ng = " + std::to_string(ng) + " needs " +
                                             std::to_string(need) + " bytes of scratch, more than the fixed " +
                                             std::to_string(kNoAllocScratchBytes));
    int *ipiv = (int *)((char *)ws + ((gws + 255) / 256) * 256);
    BGW_TRY(launch_eps_build((const double2 *)chi, vcoul, ng, nw, (double2 *)epsinv, st));
    for (int w0 = 0; w0 < nw; w0 += group) {
        const int gn = std::min(group, nw - w0);
        BGW_TRY(launch_gje_invert((double2 *)epsinv + (size_t)w0 * ng * ng, ng, gn, info + w0, ws, ipiv, st));
    }
    return BGW_OK;
}

extern "C" int bgw_pair_transform_box(const bgw_pair_desc *d, int box[3]) {
    BGW_TRY(bgw_pair_desc_check(d));
    if (!box) return fail(BGW_ERR_ARG, "null box");
    transform_box(d, box);
    return BGW_OK;
}

extern "C" int bgw_set_timing(bgw_handle_t h, int enable) {
    clear_error();
    if (!h) return fail(BGW_ERR_ARG, "null handle");
    h->timing = enable != 0;
    return BGW_OK;
}

static int drain_timing(bgw_handle_t h) {
    for (auto &p : h->pending) {
        BGW_HIP(hipEventSynchronize(p.second.second));
        float ms = 0.f;
        BGW_HIP(hipEventElapsedTime(&ms, p.second.first, p.second.second));
        h->total_ms[p.first] += ms;
        h->launches[p.first] += 1;
        h->pool.push_back(p.second.first);
        h->pool.push_back(p.second.second);
    }
    h->pending.clear();
    return BGW_OK;
}

extern "C" int bgw_get_timing(bgw_handle_t h, int kernel, double *total_ms, long long *launches) {
    clear_error();
    if (!h || kernel < 0 || kernel >= BGW_KERNEL_COUNT) return fail(BGW_ERR_ARG, "bad handle or kernel id");
    BGW_TRY(set_device(h));
    BGW_TRY(drain_timing(h));
    if (total_ms) *total_ms = h->total_ms[kernel];
    if (launches) *launches = h->launches[kernel];
    return BGW_OK;
}

extern "C" int bgw_reset_timing(bgw_handle_t h) {
    clear_error();
    if (!h) return fail(BGW_ERR_ARG, "null handle");
    BGW_TRY(set_device(h));
    BGW_TRY(drain_timing(h));
    for (int i = 0; i < BGW_KERNEL_COUNT; ++i) {
        h->total_ms[i] = 0.0;
        h->launches[i] = 0;
    }
    return BGW_OK;
}
