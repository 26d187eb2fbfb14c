// Host-side state of a library handle and the helpers the entry points share
// (error reporting, workspace, per-kernel timing, the kernels' launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "common.h"

namespace bgw {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

struct FFTPlan {
    int box[3];  // transform box actually used (see transform_box)
    AxisPlan ax[3];
    SphereMaps sm;
    std::vector<std::unique_ptr<DevBuf>> bufs;
};

struct ChiState;                 // chi0 batching: tables, tuned configurations, captured graphs
void chi_state_free(ChiState *);

}  // namespace bgw

struct bgw_handle_s {
    int device = 0;
    bgw::DevBuf ws;
    bgw::DevBuf aux;  // real flavor: complex copies of real coefficients and M
    std::map<std::string, std::unique_ptr<bgw::FFTPlan>> plans;
    bgw::ChiState *chi = nullptr;
    bool capturing = false;  // a chi0 call is being captured into a HIP graph
    // timing
    bool timing = false;
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    double total_ms[BGW_KERNEL_COUNT] = {};
    long long launches[BGW_KERNEL_COUNT] = {};
    ~bgw_handle_s() {
        bgw::chi_state_free(chi);
        for (auto &p : pending) {
            pool.push_back(p.second.first);
            pool.push_back(p.second.second);
        }
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    }
};

namespace bgw {

constexpr int kMaxNg = 12288;

int fail(int code, const std::string &msg);
bool is_2a3b(int n);
int ensure_ws(bgw_handle_t h, size_t bytes, hipStream_t st);
int set_device(bgw_handle_t h);

inline hipEvent_t take_event(bgw_handle_t h) {
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records a start event on construction and an end event on destruction
// (nothing while a graph is being captured).
struct Timed {
    bgw_handle_t h;
    int id;
    hipStream_t st;
    hipEvent_t a = nullptr;
    Timed(bgw_handle_t h_, int id_, hipStream_t st_) : h(h_), id(id_), st(st_) {
        if (h->timing && !h->capturing && (a = take_event(h)) != nullptr) (void)hipEventRecord(a, st);
    }
    ~Timed() {
        if (!a) return;
        hipEvent_t b = take_event(h);
        if (!b) return;
        (void)hipEventRecord(b, st);
        h->pending.push_back({id, {a, b}});
    }
};

// ---- chi-sum launchers (chi.hip)
int launch_weights_batch(const WProb *probs, int nprob, long long maxK, hipStream_t);
int herk_blocks_per_cu();
int launch_herk_batch(const HerkProb *probs, int nprob, long long i0, long long i1, int tile, int grid,
                      hipStream_t);
int launch_finalize_batch(const FinProb *probs, int nprob, int maxng, hipStream_t);
int launch_transpose_pairs(const double2 *M, long long K, int ng, int head, double2 *MT, hipStream_t,
                           int batches = 1);
int launch_gemm_phq(const GemmProb &G, int tile, hipStream_t);
// ---- real flavor (real.hip)
int launch_real_to_complex(const double *src, long long n, double2 *dst, hipStream_t);
int launch_pack_band_pairs(const double *src, int nk, int nc, int ngw, double2 *dst, hipStream_t);
int launch_unpack_pair_halves(const double2 *Mp, int nkv, int nc, int ng, double *M, hipStream_t);
int launch_syrk_batch(const SyrkProb *probs, int nprob, long long nitems, int grid, hipStream_t);
int syrk_blocks_per_cu();
int launch_syrk_finalize(const SyrkFin *probs, int nprob, int maxng, hipStream_t);
int launch_sigma_weights(const double *v, int ng, int ninner, double *w, hipStream_t);
int launch_sigma_wt(const double2 *einv, const double *v, int ng, int ch, double2 *WT, hipStream_t);
int launch_sigma_regroup(const double2 *B, int ng, int ninner, int nouter, double2 *B2, hipStream_t);
int launch_gemm_finalize(const double2 *part, int ns, long long mn, double scale, double2 *C, int accumulate,
                         hipStream_t);

// ---- split-precision launchers (split.hip)
int split_gpad(int ng);                         // columns of the digit slices (multiple of 128)
long long split_chunks(long long K);            // chunks (96 pairs each) of K pairs
size_t split_slice_bytes(long long nch, int ng);  // slices + exponents of nch chunks
size_t split_slices_only_bytes(long long nch, int ng);  // the slices alone (the exponents follow them)
void split_tiles(int ng, std::vector<unsigned> &out);  // upper 64 x 128 tiles in walk order
int split_grid();                               // blocks of the persistent split launch
int launch_split_slices(const double2 *M, long long K, int ng, long long c0, int nch, unsigned short *S, int *E,
                        const double *w, long long wstride, int nvec, signed char *EA, hipStream_t);
int launch_chi_split(const SplitQ *qs, int nq, long long nitems, hipStream_t);
int launch_headwing(const double2 *M, long long K, int ng, int head, const double *w, long long wstride, int nvec,
                    int nsplit, double2 *hw, hipStream_t);
int launch_headwing_write(const double2 *hw, int nsplit, int nvec, int ng, int head, double pf, double2 *chi, int nout,
                          int two, int accumulate, hipStream_t);

int device_cus();

}  // namespace bgw
