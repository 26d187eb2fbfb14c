// bgw_chi0 and bgw_autotune: planning of a batched chi0 call (all q of the
// descriptor, all frequencies), its launch sequence, HIP-graph capture and
// replay, and the tile autotuner with its optional JSON-lines cache.
//
// FP64 path: one weights launch, one persistent rank-K-update launch over
// every (q, omega, tile, K-split) work item and one finalize launch, whatever
// the number of q and omega.  Split path: weights for all problems in one
// launch, then per (q, omega) the slicing, the BF16 GEMM, the finalize and
// the FP64 head row (the omega-independent slices are made once per q).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "handle.h"

namespace bgw {

namespace {

// Autotuned choice for one size class.
struct TuneEntry {
    int tile = 64;    // FP64 output tile edge (32 or 64)
    int ipc = 8;      // FP64: target work items per CU when splitting K
    int nsplit = 0;   // split precision: K splits of the BF16 GEMM (0 = heuristic)
    double ms = 0.0;  // measured time of the winner
};

// Size class: precision, ng rounded up to 512, ceil(log2 K).
typedef std::tuple<int, int, int> ClassKey;

ClassKey class_of(int precision, int ng, long long K) {
    int kl = 0;
    while ((1ll << kl) < K) ++kl;
    return ClassKey(precision, (ng + 511) / 512 * 512, kl);
}

struct GraphEntry {
    unsigned long long key = 0;
    hipGraphExec_t exec = nullptr;
    DevBuf tables;
};

}  // namespace

struct ChiState {
    // eager calls: tables staged in pinned host memory, copied on the stream
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    hipEvent_t pinned_done = nullptr;  // the last copy out of `pinned` has completed
    bool pinned_pending = false;
    DevBuf tables;
    // tuning
    std::map<ClassKey, TuneEntry> tune;
    bool cache_loaded = false;
    unsigned generation = 0;
    // graphs
    hipStream_t cap_stream = nullptr;
    std::deque<std::unique_ptr<GraphEntry>> graphs;
    ~ChiState() {
        for (auto &g : graphs)
            if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        if (pinned_done) (void)hipEventDestroy(pinned_done);
        if (pinned) (void)hipHostFree(pinned);
    }
};

void chi_state_free(ChiState *s) { delete s; }

namespace {

constexpr size_t kMaxGraphs = 8;
constexpr int kHerkKC = 16;  // pairs per LDS stage of the FP64 kernel (split ranges are multiples of it)

ChiState *state(bgw_handle_t h) {
    if (!h->chi) h->chi = new ChiState();
    return h->chi;
}

const char *arch_name() {
    static char name[64] = {0};
    if (!name[0]) {
        hipDeviceProp_t p;
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) {
            std::snprintf(name, sizeof(name), "%s", p.gcnArchName);
            for (char *c = name; *c; ++c)
                if (*c == ':') *c = 0;  // drop feature suffixes
        } else {
            std::snprintf(name, sizeof(name), "unknown");
        }
    }
    return name;
}

// ---- JSON-lines cache: one object per line, fixed key order (written by this file).
void load_cache(ChiState *s) {
    if (s->cache_loaded) return;
    s->cache_loaded = true;
    const char *path = std::getenv("BGW_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        char arch[64] = {0};
        int cus = 0, prec = 0, ngc = 0, kl = 0, tile = 0, ipc = 0, nsplit = 0;
        double ms = 0.0;
        const int n = std::sscanf(line,
                                  "{\"arch\": \"%63[^\"]\", \"cus\": %d, \"precision\": %d, \"ng_class\": %d, "
                                  "\"k_log2\": %d, \"tile\": %d, \"ipc\": %d, \"nsplit\": %d, \"ms\": %lf}",
                                  arch, &cus, &prec, &ngc, &kl, &tile, &ipc, &nsplit, &ms);
        if (n != 9 || std::strcmp(arch, arch_name()) != 0 || cus != device_cus()) continue;
        if ((tile != 32 && tile != 64) || ipc < 1 || nsplit < 0) continue;
        TuneEntry e;
        e.tile = tile;
        e.ipc = ipc;
        e.nsplit = nsplit;
        e.ms = ms;
        s->tune[ClassKey(prec, ngc, kl)] = e;  // later lines win
    }
    std::fclose(f);
}

void append_cache(const ClassKey &k, const TuneEntry &e) {
    const char *path = std::getenv("BGW_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f,
                 "{\"arch\": \"%s\", \"cus\": %d, \"precision\": %d, \"ng_class\": %d, \"k_log2\": %d, \"tile\": %d, "
                 "\"ipc\": %d, \"nsplit\": %d, \"ms\": %.6f}\n",
                 arch_name(), device_cus(), std::get<0>(k), std::get<1>(k), std::get<2>(k), e.tile, e.ipc, e.nsplit,
                 e.ms);
    std::fclose(f);
}

TuneEntry lookup(ChiState *s, int precision, int ng, long long K) {
    auto it = s->tune.find(class_of(precision, ng, K));
    if (it != s->tune.end()) return it->second;
    TuneEntry e;  // heuristic defaults
    e.tile = ng <= 1024 ? 32 : 64;
    e.ipc = 8;
    e.nsplit = 0;
    return e;
}

int check_chi_desc(const bgw_chi_desc *d) {
    if (!d || d->nq < 1 || !d->q || d->nw < 1 || !d->omega) return fail(BGW_ERR_ARG, "bad chi descriptor");
    if (d->precision != BGW_FP64 && d->precision != BGW_SPLIT_BF16)
        return fail(BGW_ERR_ARG, "unknown precision");
    if ((long long)d->nq * d->nw > 65535) return fail(BGW_ERR_UNSUPPORTED, "more than 65535 (q, omega) problems");
    for (int i = 0; i < d->nw; ++i)
        if (!(d->omega[i] >= 0.0)) return fail(BGW_ERR_ARG, "frequencies must be >= 0");
    for (int i = 0; i < d->nq; ++i) {
        const bgw_chi_q &q = d->q[i];
        if (q.ng < 1 || q.nk < 1 || q.nv < 1 || q.nc < 1) return fail(BGW_ERR_ARG, "chi q entry: sizes must be >= 1");
        if (q.ng > kMaxNg) return fail(BGW_ERR_UNSUPPORTED, "chi q entry: ng > 8192");
        if (!q.M || !q.ev || !q.ec || !q.chi) return fail(BGW_ERR_ARG, "chi q entry: null pointer");
        if (q.head < -1 || q.head >= q.ng) return fail(BGW_ERR_ARG, "chi q entry: head index out of range");
    }
    return BGW_OK;
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// Everything one chi0 call launches, decided on the host.
struct ChiPlan {
    int precision = 0;
    int nprob = 0;
    std::vector<HerkProb> herk;  // FP64 only, ordered by first work item (tile 64, then tile 32)
    std::vector<int> herk_prob;  // problem index of each herk entry
    long long nitems64 = 0;      // items [0, nitems64) have tile 64
    std::vector<FinProb> fin;
    std::vector<WProb> wts;
    std::vector<int> prob_q, prob_w;
    long long nitems = 0, maxK = 0;
    int maxng = 0, grid = 0;
    // workspace offsets (bytes from the workspace base)
    size_t off_w = 0, off_part = 0, off_split = 0, ws_bytes = 0;
    std::vector<size_t> w_off, part_off;
    std::vector<int> split_ns;  // tuned split override per problem
    size_t table_bytes = 0;
};

// Table layout in device memory: [HerkProb * nprob][FinProb * nprob][WProb * nprob].
size_t table_size(int nprob) {
    return al256(sizeof(HerkProb) * nprob) + al256(sizeof(FinProb) * nprob) + al256(sizeof(WProb) * nprob);
}

int make_plan(bgw_handle_t h, const bgw_chi_desc *d, ChiPlan &P, int force_tile, int force_ipc, int force_nsplit) {
    ChiState *s = state(h);
    load_cache(s);
    P.precision = d->precision;
    P.nprob = d->nq * d->nw;
    P.table_bytes = table_size(P.nprob);
    size_t off = 0;
    P.off_w = off;
    for (int iq = 0; iq < d->nq; ++iq) {
        const bgw_chi_q &q = d->q[iq];
        const long long K = (long long)q.nk * q.nv * q.nc;
        P.maxK = std::max(P.maxK, K);
        P.maxng = std::max(P.maxng, q.ng);
        for (int iw = 0; iw < d->nw; ++iw) {
            P.prob_q.push_back(iq);
            P.prob_w.push_back(iw);
            P.w_off.push_back(off);
            off += al256(sizeof(double) * K);
        }
    }
    P.off_part = off;
    const int cus = device_cus();
    if (d->precision == BGW_FP64) {
        // tiles per problem, then one K-split count for the batch
        long long total_tiles = 0;
        int ipc = 0;
        std::vector<int> tile(P.nprob);
        if (!force_tile) {  // BGW_HERK_TILE=32|64 pins the FP64 output tile
            const char *env = std::getenv("BGW_HERK_TILE");
            if (env && (std::atoi(env) == 32 || std::atoi(env) == 64)) force_tile = std::atoi(env);
        }
        for (int p = 0; p < P.nprob; ++p) {
            const bgw_chi_q &q = d->q[P.prob_q[p]];
            const long long K = (long long)q.nk * q.nv * q.nc;
            const TuneEntry e = lookup(s, BGW_FP64, q.ng, K);
            tile[p] = force_tile ? force_tile : e.tile;
            ipc = std::max(ipc, force_ipc ? force_ipc : e.ipc);
            const long long nt = (q.ng + tile[p] - 1) / tile[p];
            total_tiles += nt * (nt + 1) / 2;
        }
        // K splits: at least ipc work items per CU, then the count whose last
        // round of items fills the resident block slots best (smallest such
        // count within 3% of the best makespan)
        const long long slots = (long long)cus * herk_blocks_per_cu();
        const long long ns_min = std::min<long long>(64, std::max<long long>(1, ((long long)ipc * cus + total_tiles - 1) / total_tiles));
        auto makespan = [&](long long n) { return (double)((total_tiles * n + slots - 1) / slots) / (double)n; };
        double best = makespan(ns_min);
        for (long long n = ns_min; n <= std::max<long long>(ns_min, 32); ++n) best = std::min(best, makespan(n));
        long long ns = ns_min;
        while (makespan(ns) > 1.03 * best) ++ns;
        // keep the partial sums within a quarter of the device memory
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) total_b = (size_t)64 << 30;
        for (;;) {
            size_t part = 0;
            for (int p = 0; p < P.nprob; ++p) {
                const bgw_chi_q &q = d->q[P.prob_q[p]];
                const long long K = (long long)q.nk * q.nv * q.nc;
                const long long nsp = std::min<long long>(ns, std::max<long long>(1, K / (8 * kHerkKC)));
                if (nsp > 1 || d->accumulate) part += al256(sizeof(double2) * (size_t)nsp * q.ng * q.ng);
            }
            if (ns == 1 || part <= total_b / 4) break;
            ns = std::max<long long>(1, ns / 2);
        }
        // per-problem split ranges; items numbered tile-64 problems first so
        // that each tile size is one contiguous item range (one launch each)
        std::vector<HerkProb> hps(P.nprob);
        for (int p = 0; p < P.nprob; ++p) {
            const int iq = P.prob_q[p], iw = P.prob_w[p];
            const bgw_chi_q &q = d->q[iq];
            const long long K = (long long)q.nk * q.nv * q.nc;
            long long nsp = std::min<long long>(ns, std::max<long long>(1, K / (8 * kHerkKC)));
            long long kper = (K + nsp - 1) / nsp;
            kper = (kper + kHerkKC - 1) / kHerkKC * kHerkKC;
            nsp = (K + kper - 1) / kper;
            double2 *chi = (double2 *)q.chi + (size_t)iw * q.ng * q.ng;
            const bool inplace = nsp == 1 && !d->accumulate;
            HerkProb hp;
            hp.M = (const double2 *)q.M;
            hp.w = nullptr;  // set once the workspace base is known
            hp.K = K;
            hp.kper = kper;
            hp.item0 = 0;
            hp.ng = q.ng;
            hp.tile = tile[p];
            hp.nt = (q.ng + tile[p] - 1) / tile[p];
            hp.ns = (int)nsp;
            if (inplace) {
                hp.out = chi;
                P.part_off.push_back((size_t)-1);
            } else {
                hp.out = nullptr;
                P.part_off.push_back(off);
                off += al256(sizeof(double2) * (size_t)nsp * q.ng * q.ng);
            }
            hps[p] = hp;
            FinProb fp;
            fp.part = nullptr;
            fp.chi = chi;
            fp.pf = q.prefactor;
            fp.ns = (int)nsp;
            fp.ng = q.ng;
            fp.accumulate = d->accumulate;
            fp.skip = -1;
            fp.inplace = inplace ? 1 : 0;
            fp.pad = 0;
            P.fin.push_back(fp);
        }
        long long item0 = 0;
        for (int t : {64, 32}) {
            for (int p = 0; p < P.nprob; ++p) {
                if (hps[p].tile != t) continue;
                hps[p].item0 = item0;
                hps[p].nitems = ((long long)hps[p].nt * (hps[p].nt + 1) / 2 * hps[p].ns + 7) / 8 * 8;
                item0 += hps[p].nitems;
                P.herk.push_back(hps[p]);
                P.herk_prob.push_back(p);
            }
            if (t == 64) P.nitems64 = item0;
        }
        P.nitems = item0;
        P.grid = (int)(slots / 8 * 8);  // a multiple of 8: item i stays on XCD i % 8
        P.off_split = off;
    } else {
        P.off_split = off;
        size_t split_need = 0;
        for (int p = 0; p < P.nprob; ++p) {
            const bgw_chi_q &q = d->q[P.prob_q[p]];
            const long long K = (long long)q.nk * q.nv * q.nc;
            const TuneEntry e = lookup(s, BGW_SPLIT_BF16, q.ng, K);
            const int nso = force_nsplit ? force_nsplit : e.nsplit;
            P.split_ns.push_back(nso);
            size_t b = 0;
            BGW_TRY(split_workspace_bytes(K, q.ng, nso, &b));
            split_need = std::max(split_need, b);
            FinProb fp;
            fp.part = nullptr;  // split partial sums, set at launch time
            fp.chi = (double2 *)q.chi + (size_t)P.prob_w[p] * q.ng * q.ng;
            fp.pf = q.prefactor;
            fp.ns = 0;
            fp.ng = q.ng;
            fp.accumulate = d->accumulate;
            fp.skip = q.head;
            fp.inplace = 0;
            fp.pad = 0;
            P.fin.push_back(fp);
        }
        off += al256(split_need + 256);
    }
    for (int p = 0; p < P.nprob; ++p) {
        const bgw_chi_q &q = d->q[P.prob_q[p]];
        WProb wp;
        wp.ev = q.ev;
        wp.ec = q.ec;
        wp.w = nullptr;
        wp.omega_ha = d->omega[P.prob_w[p]] / kHartreeEv;
        wp.nk = q.nk;
        wp.nv = q.nv;
        wp.nc = q.nc;
        wp.pad = 0;
        P.wts.push_back(wp);
    }
    P.ws_bytes = off + 256;
    return BGW_OK;
}

// Fill the workspace-dependent pointers of the tables.
void bind_plan(ChiPlan &P, char *ws) {
    for (int p = 0; p < P.nprob; ++p) {
        double *w = (double *)(ws + P.w_off[p]);
        P.wts[p].w = w;
    }
    for (size_t i = 0; i < P.herk.size(); ++i) {
        const int p = P.herk_prob[i];
        P.herk[i].w = P.wts[p].w;
        if (P.part_off[p] != (size_t)-1) {
            P.herk[i].out = (double2 *)(ws + P.part_off[p]);
            P.fin[p].part = P.herk[i].out;
        }
    }
}

void write_tables(const ChiPlan &P, void *host) {
    char *b = (char *)host;
    std::memset(b, 0, P.table_bytes);
    if (!P.herk.empty()) std::memcpy(b, P.herk.data(), sizeof(HerkProb) * P.nprob);
    b += al256(sizeof(HerkProb) * P.nprob);
    std::memcpy(b, P.fin.data(), sizeof(FinProb) * P.nprob);
    b += al256(sizeof(FinProb) * P.nprob);
    std::memcpy(b, P.wts.data(), sizeof(WProb) * P.nprob);
}

// The launch sequence of one chi0 call.  tab: device copy of the tables (for
// the split path the finalize entries' part pointers are patched on the host
// copy `P` and re-sent per problem through `patch`).
int enqueue(bgw_handle_t h, const bgw_chi_desc *d, ChiPlan &P, char *ws, char *tab, hipStream_t st) {
    const HerkProb *dherk = (const HerkProb *)tab;
    FinProb *dfin = (FinProb *)(tab + al256(sizeof(HerkProb) * P.nprob));
    const WProb *dw = (const WProb *)((char *)dfin + al256(sizeof(FinProb) * P.nprob));
    {
        Timed tm(h, BGW_KERNEL_WEIGHTS, st);
        BGW_TRY(launch_weights_batch(dw, P.nprob, P.maxK, st));
    }
    if (P.precision == BGW_FP64) {
        {
            Timed tm(h, BGW_KERNEL_HERK, st);
            BGW_TRY(launch_herk_batch(dherk, P.nprob, 0, P.nitems64, 64, P.grid, st));
            BGW_TRY(launch_herk_batch(dherk, P.nprob, P.nitems64, P.nitems, 32, P.grid, st));
        }
        Timed tm(h, BGW_KERNEL_FINALIZE, st);
        BGW_TRY(launch_finalize_batch(dfin, P.nprob, P.maxng, st));
        return BGW_OK;
    }
    // split precision, problem by problem (q-major, omega-minor)
    void *sws = ws + P.off_split;
    for (int p = 0; p < P.nprob; ++p) {
        const int iq = P.prob_q[p], iw = P.prob_w[p];
        const bgw_chi_q &q = d->q[iq];
        const long long K = (long long)q.nk * q.nv * q.nc;
        const double *w = P.wts[p].w;
        const SplitLayout L = split_layout(K, q.ng, P.split_ns[p], sws);
        // the slices of the unweighted side do not depend on omega: with a
        // single super-chunk they are made once per q
        const bool resident_b = L.sc_pairs >= K;
        int nslots = 0;
        for (long long t0 = 0; t0 < K; t0 += L.sc_pairs) {
            const long long kn = std::min<long long>(L.sc_pairs, K - t0);
            const int nch = (int)((kn + 127) / 128);
            {
                Timed tm(h, BGW_KERNEL_SPLIT_SLICE, st);
                BGW_TRY(launch_split_slices(L, (const double2 *)q.M, K, q.ng, w, t0, nch, !(resident_b && iw > 0),
                                            st));
            }
            Timed tm(h, BGW_KERNEL_SPLIT_HERK, st);
            int used = 0;
            BGW_TRY(launch_split_gemm(L, q.ng, nch, nslots, &used, st));
            if (!nslots) nslots = used;
        }
        if (P.fin[p].ns != nslots || P.fin[p].part != L.part) return fail(BGW_ERR_HIP, "split plan mismatch");
        {
            Timed tm(h, BGW_KERNEL_FINALIZE, st);
            BGW_TRY(launch_finalize_batch(dfin + p, 1, q.ng, st));
        }
        if (q.head >= 0) {
            Timed tm(h, BGW_KERNEL_HEADWING, st);
            BGW_TRY(launch_split_headwing(L, (const double2 *)q.M, K, q.ng, q.head, w, q.prefactor,
                                          (double2 *)P.fin[p].chi, d->accumulate, st));
        }
    }
    return BGW_OK;
}

// The split layout's partial-sum pointer and slot count are fixed by the
// plan: fill them into the finalize entries before the tables are sent.
void bind_split(const bgw_chi_desc *d, ChiPlan &P, char *ws) {
    if (P.precision != BGW_SPLIT_BF16) return;
    for (int p = 0; p < P.nprob; ++p) {
        const bgw_chi_q &q = d->q[P.prob_q[p]];
        const long long K = (long long)q.nk * q.nv * q.nc;
        const SplitLayout L = split_layout(K, q.ng, P.split_ns[p], ws + P.off_split);
        // slots used by the first super-chunk (the largest): same rule as launch_split_gemm
        const long long nch = std::min<long long>(L.sc_pairs, K) / 128 + ((std::min<long long>(L.sc_pairs, K) % 128) != 0);
        int ns = (int)std::min<long long>(L.nsplit, nch);
        const int cps = (int)((nch + ns - 1) / ns);
        ns = (int)((nch + cps - 1) / cps);
        P.fin[p].part = L.part;
        P.fin[p].ns = ns;
    }
}

unsigned long long fnv(unsigned long long hsh, const void *p, size_t n) {
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) hsh = (hsh ^ c[i]) * 1099511628211ull;
    return hsh;
}

unsigned long long desc_key(bgw_handle_t h, const bgw_chi_desc *d) {
    unsigned long long k = 1469598103934665603ull;
    k = fnv(k, &d->nq, sizeof(int));
    k = fnv(k, d->q, sizeof(bgw_chi_q) * d->nq);
    k = fnv(k, &d->nw, sizeof(int));
    k = fnv(k, d->omega, sizeof(double) * d->nw);
    k = fnv(k, &d->precision, sizeof(int));
    k = fnv(k, &d->accumulate, sizeof(int));
    k = fnv(k, &h->ws.p, sizeof(void *));
    k = fnv(k, &h->ws.bytes, sizeof(size_t));
    k = fnv(k, &h->chi->generation, sizeof(unsigned));
    return k;
}

int run_eager(bgw_handle_t h, const bgw_chi_desc *d, ChiPlan &P, hipStream_t st) {
    ChiState *s = state(h);
    BGW_TRY(ensure_ws(h, P.ws_bytes, st));
    char *ws = (char *)h->ws.p;
    bind_plan(P, ws);
    bind_split(d, P, ws);
    if (s->tables.bytes < P.table_bytes) {
        BGW_HIP(hipStreamSynchronize(st));
        if (s->tables.p) BGW_HIP(hipFree(s->tables.p));
        s->tables.p = nullptr;
        s->tables.bytes = 0;
        BGW_HIP(hipMalloc(&s->tables.p, P.table_bytes));
        s->tables.bytes = P.table_bytes;
    }
    if (s->pinned_pending) {
        BGW_HIP(hipEventSynchronize(s->pinned_done));
        s->pinned_pending = false;
    }
    if (s->pinned_bytes < P.table_bytes) {
        if (s->pinned) BGW_HIP(hipHostFree(s->pinned));
        s->pinned = nullptr;
        s->pinned_bytes = 0;
        BGW_HIP(hipHostMalloc(&s->pinned, P.table_bytes, hipHostMallocDefault));
        s->pinned_bytes = P.table_bytes;
    }
    if (!s->pinned_done) BGW_HIP(hipEventCreateWithFlags(&s->pinned_done, hipEventDisableTiming));
    write_tables(P, s->pinned);
    BGW_HIP(hipMemcpyAsync(s->tables.p, s->pinned, P.table_bytes, hipMemcpyHostToDevice, st));
    BGW_HIP(hipEventRecord(s->pinned_done, st));
    s->pinned_pending = true;
    return enqueue(h, d, P, ws, (char *)s->tables.p, st);
}

int run_graph(bgw_handle_t h, const bgw_chi_desc *d, ChiPlan &P, hipStream_t st) {
    ChiState *s = state(h);
    BGW_TRY(ensure_ws(h, P.ws_bytes, st));  // before the key: the key holds the workspace address
    const unsigned long long key = desc_key(h, d);
    for (auto &g : s->graphs)
        if (g->key == key) {
            BGW_HIP(hipGraphLaunch(g->exec, st));
            return BGW_OK;
        }
    char *ws = (char *)h->ws.p;
    bind_plan(P, ws);
    bind_split(d, P, ws);
    auto g = std::make_unique<GraphEntry>();
    g->key = key;
    BGW_HIP(hipMalloc(&g->tables.p, P.table_bytes));
    g->tables.bytes = P.table_bytes;
    std::vector<char> host(P.table_bytes);
    write_tables(P, host.data());
    BGW_HIP(hipMemcpy(g->tables.p, host.data(), P.table_bytes, hipMemcpyHostToDevice));
    if (!s->cap_stream) BGW_HIP(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    BGW_HIP(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeRelaxed));
    h->capturing = true;
    const int rc = enqueue(h, d, P, ws, (char *)g->tables.p, s->cap_stream);
    h->capturing = false;
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(s->cap_stream, &graph);
    if (rc != BGW_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        BGW_HIP(ec);
    }
    const hipError_t ei = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    BGW_HIP(ei);
    BGW_HIP(hipGraphLaunch(g->exec, st));
    if (s->graphs.size() >= kMaxGraphs) {
        BGW_HIP(hipStreamSynchronize(st));  // the evicted graph may still run
        (void)hipGraphExecDestroy(s->graphs.front()->exec);
        s->graphs.pop_front();
    }
    s->graphs.push_back(std::move(g));
    return BGW_OK;
}

}  // namespace

}  // namespace bgw

using namespace bgw;

extern "C" int bgw_chi0(bgw_handle_t h, const bgw_chi_desc *d, void *stream) {
    clear_error();
    BGW_TRY(check_chi_desc(d));
    if (!h) return fail(BGW_ERR_ARG, "null handle");
    BGW_TRY(set_device(h));
    hipStream_t st = (hipStream_t)stream;
    ChiPlan P;
    BGW_TRY(make_plan(h, d, P, 0, 0, 0));
    if (d->use_graph) return run_graph(h, d, P, st);
    return run_eager(h, d, P, st);
}

extern "C" int bgw_autotune(bgw_handle_t h, const bgw_chi_desc *d, void *stream) {
    clear_error();
    BGW_TRY(check_chi_desc(d));
    if (!h) return fail(BGW_ERR_ARG, "null handle");
    BGW_TRY(set_device(h));
    hipStream_t st = (hipStream_t)stream;
    ChiState *s = state(h);
    load_cache(s);
    // one representative q per size class, first frequency, K cut to at most 2^17 pairs
    std::map<ClassKey, int> reps;
    for (int iq = 0; iq < d->nq; ++iq) {
        const bgw_chi_q &q = d->q[iq];
        reps.emplace(class_of(d->precision, q.ng, (long long)q.nk * q.nv * q.nc), iq);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BGW_HIP(hipEventCreate(&e0));
    BGW_HIP(hipEventCreate(&e1));
    int rc = BGW_OK;
    for (auto &kv : reps) {
        bgw_chi_q q = d->q[kv.second];
        const long long K = (long long)q.nk * q.nv * q.nc;
        // truncate along the pair index: whole (k, v) rows of nc pairs
        const long long kmax = 1ll << 17;
        if (K > kmax) {
            const long long rows = std::max<long long>(1, kmax / q.nc);
            q.nk = 1;
            q.nv = (int)std::min<long long>(rows, (long long)q.nv * d->q[kv.second].nk);
        }
        // timing writes into chi of this q (an output buffer): first frequency, no accumulation
        bgw_chi_desc one = *d;
        one.nq = 1;
        one.q = &q;
        one.nw = 1;
        one.accumulate = 0;
        one.use_graph = 0;
        std::vector<std::tuple<int, int, int>> cands;
        if (d->precision == BGW_FP64) {
            for (int tile : {32, 64})
                for (int ipc : {2, 8, 32}) cands.emplace_back(tile, ipc, 0);
        } else {
            for (int ns : {8, 16, 24, 32}) cands.emplace_back(0, 0, ns);
        }
        TuneEntry best;
        best.ms = 1e300;
        for (auto &c : cands) {
            ChiPlan P;
            rc = make_plan(h, &one, P, std::get<0>(c), std::get<1>(c), std::get<2>(c));
            if (rc != BGW_OK) break;
            float tot = 0.f;
            for (int rep = 0; rep < 3 && rc == BGW_OK; ++rep) {
                ChiPlan Q = P;
                if (rep == 1) rc = hipEventRecord(e0, st) == hipSuccess ? BGW_OK : BGW_ERR_HIP;
                if (rc == BGW_OK) rc = run_eager(h, &one, Q, st);
                if (rep == 2 && rc == BGW_OK) {
                    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&tot, e0, e1) != hipSuccess)
                        rc = fail(BGW_ERR_HIP, "autotune timing failed");
                }
            }
            if (rc != BGW_OK) break;
            const double ms = tot / 2.0;
            if (ms < best.ms) {
                best.ms = ms;
                best.tile = std::get<0>(c) ? std::get<0>(c) : 64;
                best.ipc = std::get<1>(c) ? std::get<1>(c) : 8;
                best.nsplit = std::get<2>(c);
            }
        }
        if (rc != BGW_OK) break;
        s->tune[kv.first] = best;
        append_cache(kv.first, best);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ++s->generation;  // captured graphs of older choices are not reused
    return rc;
}

extern "C" int bgw_tuned_config(bgw_handle_t h, int precision, int ng, long long K, int *cfg) {
    clear_error();
    if (!h || !cfg || ng < 1 || K < 1 || (precision != BGW_FP64 && precision != BGW_SPLIT_BF16))
        return fail(BGW_ERR_ARG, "bad arguments to bgw_tuned_config");
    ChiState *s = state(h);
    load_cache(s);
    const bool tuned = s->tune.count(class_of(precision, ng, K)) != 0;
    const TuneEntry e = lookup(s, precision, ng, K);
    cfg[0] = e.tile;
    cfg[1] = e.ipc;
    cfg[2] = e.nsplit;
    cfg[3] = tuned ? 1 : 0;
    return BGW_OK;
}
