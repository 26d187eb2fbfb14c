// bgw_chi0 and bgw_autotune: planning of a batched chi0 call (all q of the
// descriptor, all frequencies, both frequency axes), its launch sequence,
// HIP-graph capture and replay, and the tile autotuner with its optional
// JSON-lines cache.
//
// A weight vector is one (q, frequency) on the imaginary axis and one
// (q, frequency, Re w / Im w) on the real axis.  FP64 path: one weights
// launch, one persistent rank-K-update launch per tile size over every
// (vector, tile, K-split) work item and one finalize launch, whatever the
// number of q and frequencies.  Split path: one weights launch; per q the
// frequency-independent digit slices; one persistent launch over every
// (q, vector, tile, K-split) item of the q whose slices fit together (one
// launch for the whole batch unless the device memory runs out); the FP64
// head rows of every q; one finalize launch.
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

constexpr size_t kMaxGraphs = 64;
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
    if (d->axis != BGW_AXIS_IMAG && d->axis != BGW_AXIS_RETARDED && d->axis != BGW_AXIS_ADVANCED)
        return fail(BGW_ERR_ARG, "unknown frequency axis");
    if (d->axis != BGW_AXIS_IMAG && !(d->broadening > 0.0))
        return fail(BGW_ERR_ARG, "the real frequency axis needs a broadening > 0");
    const long long nvec = (long long)d->nq * d->nw * (d->axis == BGW_AXIS_IMAG ? 1 : 2);
    if (nvec > 65535) return fail(BGW_ERR_UNSUPPORTED, "more than 65535 weight vectors (q x frequencies)");
    for (int i = 0; i < d->nw; ++i)
        if (!(d->omega[i] >= 0.0)) return fail(BGW_ERR_ARG, "frequencies must be >= 0");
    for (int i = 0; i < d->nq; ++i) {
        const bgw_chi_q &q = d->q[i];
        if (q.ng < 1 || q.nk < 1 || q.nv < 1 || q.nc < 1) return fail(BGW_ERR_ARG, "chi q entry: sizes must be >= 1");
        if (q.ng > kMaxNg) return fail(BGW_ERR_UNSUPPORTED, "chi q entry: ng > 12288");
        if (!q.M || !q.ev || !q.ec || !q.chi) return fail(BGW_ERR_ARG, "chi q entry: null pointer");
        if (q.head < -1 || q.head >= q.ng) return fail(BGW_ERR_ARG, "chi q entry: head index out of range");
    }
    return BGW_OK;
}

size_t al256(size_t b) { return (b + 255) / 256 * 256; }

constexpr int kHeadSplits = 128;  // K ranges of the FP64 head rows (enough blocks to stream M at full rate)

// One launch of the persistent split-precision GEMM: entries (q, chunk range).
struct SplitLaunch {
    std::vector<SplitQ> qs;      // table entries (pointers bound later)
    std::vector<int> qidx;       // q of each entry
    std::vector<size_t> sb_off;  // slices of each entry (offset in the slice region)
    std::vector<size_t> ew_off;  // weighted-side exponents of each entry (offset in the EA region)
    long long nitems = 0;
    size_t tab_off = 0;          // offset of the entries in the device table
};

// Everything one chi0 call launches, decided on the host.  A weight vector
// is one (q, frequency) on the imaginary axis and one (q, frequency, Re/Im)
// on the real axis; an output matrix is one (q, frequency).
struct ChiPlan {
    int precision = 0, axis = 0;
    int vpq = 1;                 // weight vectors per (q, frequency): 1 or 2
    int nvec = 0, nout = 0;
    std::vector<WProb> wts;      // per vector, q-major, then frequency, then Re/Im
    std::vector<size_t> w_off;   // per vector
    std::vector<FinProb> fin;    // per output matrix
    long long maxK = 0;
    int maxng = 0;
    // FP64
    std::vector<HerkProb> herk;  // ordered by first work item (tile 64, then tile 32)
    std::vector<int> herk_vec;   // vector of each herk entry
    std::vector<size_t> vpart_off;  // FP64: per vector partial sums ((size_t)-1: in place)
    long long nitems64 = 0, nitems = 0;
    int grid = 0;
    // split
    std::vector<SplitLaunch> launches;
    std::vector<std::vector<unsigned>> tiles;  // per q
    std::vector<size_t> tiles_off;             // per q, in the device table
    std::vector<size_t> qpart_off;             // per q: [nvec_q][ns][ng][ng] partial sums ((size_t)-1: in place)
    std::vector<int> q_ns;
    size_t off_slices = 0, off_ew = 0, off_hw = 0;
    // workspace and table sizes
    size_t ws_bytes = 0, table_bytes = 0;
    size_t off_fin = 0, off_wts = 0, off_split = 0;  // table offsets
};

long long q_pairs(const bgw_chi_q &q) { return (long long)q.nk * q.nv * q.nc; }

// Wave-filling rule shared by both precisions: at least `ipc` items per CU,
// then the count whose last round of items fills the resident slots best
// (smallest such count within 3% of the best makespan).
long long choose_splits(long long base_items, long long slots, int ipc, long long cap) {
    const long long cus = device_cus();
    long long lo = std::max<long long>(1, ((long long)ipc * cus + base_items - 1) / base_items);
    lo = std::min(lo, std::max<long long>(1, cap));
    const long long hi = std::max(lo, std::min<long long>(cap, 32));
    auto makespan = [&](long long n) { return (double)((base_items * n + slots - 1) / slots) / (double)n; };
    double best = makespan(lo);
    for (long long n = lo; n <= hi; ++n) best = std::min(best, makespan(n));
    long long ns = lo;
    while (ns < hi && makespan(ns) > 1.03 * best) ++ns;
    return ns;
}

// prefix: workspace bytes kept free at the start (the Bethe-Salpeter exchange
// kernel keeps its transposed pair matrix there); given: the q entries' ev
// arrays are the weights themselves (one vector per q, imaginary axis, one
// frequency).
int make_plan(bgw_handle_t h, const bgw_chi_desc *d, ChiPlan &P, int force_tile, int force_ipc, int force_nsplit,
              size_t prefix = 0, bool given = false) {
    ChiState *s = state(h);
    load_cache(s);
    P.precision = d->precision;
    P.axis = d->axis;
    P.vpq = d->axis == BGW_AXIS_IMAG ? 1 : 2;
    P.nvec = d->nq * d->nw * P.vpq;
    P.nout = d->nq * d->nw;
    const bool real_axis = d->axis != BGW_AXIS_IMAG;
    const int cus = device_cus();
    size_t off = al256(prefix);
    // weight vectors
    for (int iq = 0; iq < d->nq; ++iq) {
        const bgw_chi_q &q = d->q[iq];
        const long long K = q_pairs(q);
        P.maxK = std::max(P.maxK, K);
        P.maxng = std::max(P.maxng, q.ng);
        for (int iw = 0; iw < d->nw; ++iw)
            for (int part = 0; part < P.vpq; ++part) {
                WProb wp;
                wp.ev = q.ev;
                wp.ec = q.ec;
                wp.w = nullptr;
                wp.omega_ha = d->omega[iw] / kHartreeEv;
                wp.delta_ha = real_axis ? d->broadening / kHartreeEv : 0.0;
                wp.nk = q.nk;
                wp.nv = q.nv;
                wp.nc = q.nc;
                wp.kind = given ? kWeightGiven
                          : !real_axis ? kWeightImag
                                     : (part == 0 ? kWeightRealRe
                                                  : (d->axis == BGW_AXIS_RETARDED ? kWeightRetIm : kWeightAdvIm));
                P.wts.push_back(wp);
                P.w_off.push_back(off);
                off += al256(sizeof(double) * (K + 128));  // padded: the split GEMM stages whole 16-pair steps
            }
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) total_b = (size_t)64 << 30;
    if (d->precision == BGW_FP64) {
        // tiles per vector, then one K-split count for the batch
        long long total_tiles = 0;
        int ipc = 0;
        std::vector<int> tile(P.nvec);
        if (!force_tile) {  // BGW_HERK_TILE=32|64 pins the FP64 output tile
            const char *env = std::getenv("BGW_HERK_TILE");
            if (env && (std::atoi(env) == 32 || std::atoi(env) == 64)) force_tile = std::atoi(env);
        }
        for (int v = 0; v < P.nvec; ++v) {
            const bgw_chi_q &q = d->q[v / (d->nw * P.vpq)];
            const TuneEntry e = lookup(s, BGW_FP64, q.ng, q_pairs(q));
            tile[v] = force_tile ? force_tile : e.tile;
            ipc = std::max(ipc, force_ipc ? force_ipc : e.ipc);
            const long long nt = (q.ng + tile[v] - 1) / tile[v];
            total_tiles += nt * (nt + 1) / 2;
        }
        const long long slots = (long long)cus * herk_blocks_per_cu();
        long long ns = choose_splits(total_tiles, slots, ipc, 64);
        // keep the partial sums within a quarter of the device memory
        for (;;) {
            size_t part = 0;
            for (int v = 0; v < P.nvec; ++v) {
                const bgw_chi_q &q = d->q[v / (d->nw * P.vpq)];
                const long long nsp = std::min<long long>(ns, std::max<long long>(1, q_pairs(q) / (8 * kHerkKC)));
                if (nsp > 1 || d->accumulate || real_axis) part += al256(sizeof(double2) * (size_t)nsp * q.ng * q.ng);
            }
            if (ns == 1 || part <= total_b / 4) break;
            ns = std::max<long long>(1, ns / 2);
        }
        std::vector<HerkProb> hps(P.nvec);
        for (int v = 0; v < P.nvec; ++v) {
            const int iq = v / (d->nw * P.vpq), iw = (v / P.vpq) % d->nw;
            const bgw_chi_q &q = d->q[iq];
            const long long K = q_pairs(q);
            long long nsp = std::min<long long>(ns, std::max<long long>(1, K / (8 * kHerkKC)));
            long long kper = (K + nsp - 1) / nsp;
            kper = (kper + kHerkKC - 1) / kHerkKC * kHerkKC;
            nsp = (K + kper - 1) / kper;
            const bool inplace = nsp == 1 && !d->accumulate && !real_axis;
            HerkProb hp;
            hp.M = (const double2 *)q.M;
            hp.w = nullptr;  // set once the workspace base is known
            hp.K = K;
            hp.kper = kper;
            hp.item0 = 0;
            hp.ng = q.ng;
            hp.tile = tile[v];
            hp.nt = (q.ng + tile[v] - 1) / tile[v];
            hp.ns = (int)nsp;
            if (inplace) {
                hp.out = (double2 *)q.chi + (size_t)iw * q.ng * q.ng;
                P.vpart_off.push_back((size_t)-1);
            } else {
                hp.out = nullptr;
                P.vpart_off.push_back(off);
                off += al256(sizeof(double2) * (size_t)nsp * q.ng * q.ng);
            }
            hps[v] = hp;
        }
        for (int o = 0; o < P.nout; ++o) {
            const int iq = o / d->nw, iw = o % d->nw;
            const bgw_chi_q &q = d->q[iq];
            const int va = o * P.vpq;
            FinProb fp;
            fp.part = nullptr;
            fp.part_im = nullptr;
            fp.chi = (double2 *)q.chi + (size_t)iw * q.ng * q.ng;
            fp.pf = q.prefactor;
            fp.ns = hps[va].ns;
            fp.ng = q.ng;
            fp.accumulate = d->accumulate;
            fp.skip = -1;
            fp.inplace = P.vpart_off[va] == (size_t)-1 ? 1 : 0;
            fp.pad = 0;
            P.fin.push_back(fp);
        }
        long long item0 = 0;
        for (int t : {64, 32}) {
            for (int v = 0; v < P.nvec; ++v) {
                if (hps[v].tile != t) continue;
                hps[v].item0 = item0;
                hps[v].nitems = ((long long)hps[v].nt * (hps[v].nt + 1) / 2 * hps[v].ns + 7) / 8 * 8;
                item0 += hps[v].nitems;
                P.herk.push_back(hps[v]);
                P.herk_vec.push_back(v);
            }
            if (t == 64) P.nitems64 = item0;
        }
        P.nitems = item0;
        P.grid = (int)(slots / 8 * 8);  // a multiple of 8: item i stays on XCD i % 8
    } else {
        // ---- split precision: per q the K-split count, the partial sums and the tile walk
        const int vq = d->nw * P.vpq;  // weight vectors per q
        const long long slots = split_grid();
        long long base_items = 0;
        for (int iq = 0; iq < d->nq; ++iq) {
            P.tiles.emplace_back();
            split_tiles(d->q[iq].ng, P.tiles.back());
            base_items += (long long)P.tiles.back().size() * vq;
        }
        // K splits per q: the wave-filling rule over the whole batch (or the tuned count)
        P.q_ns.assign(d->nq, 1);
        for (int iq = 0; iq < d->nq; ++iq) {
            const bgw_chi_q &q = d->q[iq];
            const TuneEntry e = lookup(s, BGW_SPLIT_BF16, q.ng, q_pairs(q));
            const int nso = force_nsplit ? force_nsplit : e.nsplit;
            const long long ns = nso > 0 ? nso : choose_splits(base_items, slots, 4, 64);
            P.q_ns[iq] = (int)std::max<long long>(1, std::min<long long>(ns, split_chunks(q_pairs(q))));
        }
        // partial sums per q (none when the raw sums can go straight into chi)
        auto part_bytes = [&](int iq) {
            return al256(sizeof(double2) * (size_t)vq * P.q_ns[iq] * d->q[iq].ng * d->q[iq].ng);
        };
        P.qpart_off.assign(d->nq, (size_t)-1);
        for (int iq = 0; iq < d->nq; ++iq) {
            if (P.q_ns[iq] == 1 && !d->accumulate && !real_axis) continue;
            P.qpart_off[iq] = off;
            off += part_bytes(iq);
        }
        size_t hw = 0, ew_all = 0;
        for (int iq = 0; iq < d->nq; ++iq) {
            if (d->q[iq].head >= 0) hw = std::max(hw, sizeof(double2) * (size_t)kHeadSplits * vq * d->q[iq].ng);
            ew_all += al256((size_t)vq * split_chunks(q_pairs(d->q[iq])) * split_gpad(d->q[iq].ng));
        }
        // slice budget: what the device holds next to everything else of the call
        const size_t other = off + al256(hw) + ew_all + ((size_t)2 << 30);
        const size_t avail = (size_t)(0.9 * (double)(free_b + h->ws.bytes));
        size_t budget = avail > other + ((size_t)1 << 30) ? avail - other : ((size_t)1 << 30);
        if (const char *env = std::getenv("BGW_SPLIT_SLICE_BYTES"))
            budget = std::max<size_t>(1, std::strtoull(env, nullptr, 10));
        // launches: consecutive q whose slices fit together; a q too large alone
        // is cut into chunk ranges (one launch each, later ones adding)
        std::vector<std::pair<int, std::pair<long long, long long>>> ranges;  // (q, [c0, c1))
        for (int iq = 0; iq < d->nq; ++iq) {
            const long long nch = split_chunks(q_pairs(d->q[iq]));
            const size_t per_chunk = split_slice_bytes(1, d->q[iq].ng);
            long long fit = std::max<long long>(1, (long long)(budget / per_chunk));
            if (fit < nch) fit = std::max<long long>(fit, P.q_ns[iq]);  // the first range initialises every split
            for (long long c0 = 0; c0 < nch; c0 += fit) ranges.push_back({iq, {c0, std::min(nch, c0 + fit)}});
        }
        size_t slice_max = 0, ew_max = 0;
        {
            SplitLaunch cur;
            size_t cur_bytes = 0, cur_ew = 0;
            auto close = [&]() {
                if (cur.qs.empty()) return;
                slice_max = std::max(slice_max, cur_bytes);
                ew_max = std::max(ew_max, cur_ew);
                P.launches.push_back(cur);
                cur = SplitLaunch();
                cur_bytes = cur_ew = 0;
            };
            for (auto &r : ranges) {
                const int iq = r.first;
                const long long nchr = r.second.second - r.second.first;
                const size_t b = al256(split_slice_bytes(nchr, d->q[iq].ng));
                const bool whole = r.second.first == 0 && r.second.second == split_chunks(q_pairs(d->q[iq]));
                if (!cur.qs.empty() && (!whole || cur_bytes + b > budget)) close();
                SplitQ e;
                std::memset(&e, 0, sizeof(e));
                e.chunk0 = (int)r.second.first;
                e.nch = (int)nchr;
                cur.qs.push_back(e);
                cur.qidx.push_back(iq);
                cur.sb_off.push_back(cur_bytes);
                cur.ew_off.push_back(cur_ew);
                cur_bytes += b;
                cur_ew += al256((size_t)vq * nchr * split_gpad(d->q[iq].ng));
                if (!whole) close();
                if (!whole && P.qpart_off[iq] == (size_t)-1) {  // several launches: sums through partials
                    P.qpart_off[iq] = off;
                    off += part_bytes(iq);
                }
            }
            close();
        }
        // fill the launch entries (workspace pointers are bound later)
        std::vector<int> seen(d->nq, 0);
        for (auto &L : P.launches) {
            long long item0 = 0;
            for (size_t i = 0; i < L.qs.size(); ++i) {
                const int iq = L.qidx[i];
                const bgw_chi_q &q = d->q[iq];
                SplitQ &e = L.qs[i];
                e.M = (const double2 *)q.M;
                e.K = q_pairs(q);
                e.ng = q.ng;
                e.gpad = split_gpad(q.ng);
                e.nvec = vq;
                e.ntiles = (int)P.tiles[iq].size();
                // every split non-empty; the first range of a q holds >= q_ns chunks, so it
                // writes all q_ns partial sums that the finalize reads
                e.ns = std::min<int>(P.q_ns[iq], e.nch);
                e.add = seen[iq] ? 1 : 0;
                seen[iq] = 1;
                e.item0 = item0;
                e.nitems = ((long long)e.ntiles * e.ns * e.nvec + 7) / 8 * 8;
                item0 += e.nitems;
            }
            L.nitems = item0;
        }
        for (int o = 0; o < P.nout; ++o) {
            const int iq = o / d->nw, iw = o % d->nw;
            const bgw_chi_q &q = d->q[iq];
            FinProb fp;
            fp.part = nullptr;  // bound later
            fp.part_im = nullptr;
            fp.chi = (double2 *)q.chi + (size_t)iw * q.ng * q.ng;
            fp.pf = q.prefactor;
            fp.ns = P.q_ns[iq];
            fp.ng = q.ng;
            fp.accumulate = d->accumulate;
            fp.skip = q.head;
            fp.inplace = P.qpart_off[iq] == (size_t)-1 ? 1 : 0;
            fp.pad = 0;
            P.fin.push_back(fp);
        }
        P.off_slices = off;
        off += al256(slice_max);
        P.off_ew = off;
        off += al256(ew_max);
        P.off_hw = off;
        off += al256(hw);
    }
    // device table: [HerkProb * nvec][FinProb * nout][WProb * nvec][SplitQ ...][tile walks]
    size_t t = al256(sizeof(HerkProb) * P.herk.size());
    P.off_fin = t;
    t += al256(sizeof(FinProb) * P.nout);
    P.off_wts = t;
    t += al256(sizeof(WProb) * P.nvec);
    P.off_split = t;
    for (auto &L : P.launches) {
        L.tab_off = t;
        t += al256(sizeof(SplitQ) * L.qs.size());
    }
    for (auto &tl : P.tiles) {
        P.tiles_off.push_back(t);
        t += al256(sizeof(unsigned) * tl.size());
    }
    P.table_bytes = std::max<size_t>(t, 256);
    P.ws_bytes = off + 256;
    return BGW_OK;
}

// Fill the workspace- and table-dependent pointers: ws is the workspace base,
// tab the device table base the kernels will read.
void bind_plan(const bgw_chi_desc *d, ChiPlan &P, char *ws, char *tab) {
    for (int v = 0; v < P.nvec; ++v) P.wts[v].w = (double *)(ws + P.w_off[v]);
    const int vq = d->nw * P.vpq;
    if (P.precision == BGW_FP64) {
        std::vector<double2 *> vout(P.nvec, nullptr);
        for (size_t i = 0; i < P.herk.size(); ++i) {
            const int v = P.herk_vec[i];
            P.herk[i].w = P.wts[v].w;
            if (P.vpart_off[v] != (size_t)-1) P.herk[i].out = (double2 *)(ws + P.vpart_off[v]);
            vout[v] = P.herk[i].out;
        }
        for (int o = 0; o < P.nout; ++o) {
            const int va = o * P.vpq;
            if (!P.fin[o].inplace) P.fin[o].part = vout[va];
            if (P.vpq == 2) P.fin[o].part_im = vout[va + 1];
        }
        return;
    }
    for (auto &L : P.launches)
        for (size_t i = 0; i < L.qs.size(); ++i) {
            const int iq = L.qidx[i];
            const bgw_chi_q &q = d->q[iq];
            SplitQ &e = L.qs[i];
            e.w = P.wts[iq * vq].w;
            e.wstride = vq > 1 ? (long long)((P.w_off[iq * vq + 1] - P.w_off[iq * vq]) / sizeof(double)) : 0;
            e.SB = (const unsigned short *)(ws + P.off_slices + L.sb_off[i]);
            e.EB = (const int *)(ws + P.off_slices + L.sb_off[i] + split_slices_only_bytes(e.nch, e.ng));
            e.EA = (const signed char *)(ws + P.off_ew + L.ew_off[i]);
            e.out = P.qpart_off[iq] == (size_t)-1 ? (double2 *)q.chi : (double2 *)(ws + P.qpart_off[iq]);
            e.vstride = (long long)(P.qpart_off[iq] == (size_t)-1 ? 1 : P.q_ns[iq]) * q.ng * q.ng;
            e.tiles = (const unsigned *)(tab + P.tiles_off[iq]);
        }
    for (int o = 0; o < P.nout; ++o) {
        const int iq = o / d->nw, iw = o % d->nw;
        if (P.qpart_off[iq] == (size_t)-1) continue;
        const bgw_chi_q &q = d->q[iq];
        double2 *base = (double2 *)(ws + P.qpart_off[iq]);
        const size_t blk = (size_t)P.q_ns[iq] * q.ng * q.ng;
        P.fin[o].part = base + (size_t)(iw * P.vpq) * blk;
        if (P.vpq == 2) P.fin[o].part_im = base + (size_t)(iw * P.vpq + 1) * blk;
    }
}

void write_tables(const ChiPlan &P, void *host) {
    char *b = (char *)host;
    std::memset(b, 0, P.table_bytes);
    if (!P.herk.empty()) std::memcpy(b, P.herk.data(), sizeof(HerkProb) * P.herk.size());
    std::memcpy(b + P.off_fin, P.fin.data(), sizeof(FinProb) * P.nout);
    std::memcpy(b + P.off_wts, P.wts.data(), sizeof(WProb) * P.nvec);
    for (auto &L : P.launches) std::memcpy(b + L.tab_off, L.qs.data(), sizeof(SplitQ) * L.qs.size());
    for (size_t i = 0; i < P.tiles.size(); ++i)
        std::memcpy(b + P.tiles_off[i], P.tiles[i].data(), sizeof(unsigned) * P.tiles[i].size());
}

// The launch sequence of one chi0 call (tables already in device memory at tab).
int enqueue(bgw_handle_t h, const bgw_chi_desc *d, ChiPlan &P, char *ws, char *tab, hipStream_t st) {
    const HerkProb *dherk = (const HerkProb *)tab;
    const FinProb *dfin = (const FinProb *)(tab + P.off_fin);
    const WProb *dw = (const WProb *)(tab + P.off_wts);
    {
        Timed tm(h, BGW_KERNEL_WEIGHTS, st);
        BGW_TRY(launch_weights_batch(dw, P.nvec, P.maxK, st));
    }
    if (P.precision == BGW_FP64) {
        {
            Timed tm(h, BGW_KERNEL_HERK, st);
            const int nh = (int)P.herk.size();
            BGW_TRY(launch_herk_batch(dherk, nh, 0, P.nitems64, 64, P.grid, st));
            BGW_TRY(launch_herk_batch(dherk, nh, P.nitems64, P.nitems, 32, P.grid, st));
        }
        Timed tm(h, BGW_KERNEL_FINALIZE, st);
        BGW_TRY(launch_finalize_batch(dfin, P.nout, P.maxng, st));
        return BGW_OK;
    }
    const int vq = d->nw * P.vpq;
    std::vector<int> remaining(d->nq, 0);
    for (auto &L : P.launches)
        for (int qi : L.qidx) ++remaining[qi];
    for (auto &L : P.launches) {
        {
            Timed tm(h, BGW_KERNEL_SPLIT_SLICE, st);
            for (size_t i = 0; i < L.qs.size(); ++i) {
                const SplitQ &e = L.qs[i];
                BGW_TRY(launch_split_slices(e.M, e.K, e.ng, e.chunk0, e.nch, (unsigned short *)e.SB, (int *)e.EB, e.w,
                                            e.wstride, e.nvec, (signed char *)e.EA, st));
            }
        }
        {
            Timed tm(h, BGW_KERNEL_SPLIT_HERK, st);
            BGW_TRY(launch_chi_split((const SplitQ *)(tab + L.tab_off), (int)L.qs.size(), L.nitems, st));
        }
        // FP64 head rows of every q whose sums are complete
        for (size_t i = 0; i < L.qs.size(); ++i) {
            const int iq = L.qidx[i];
            if (--remaining[iq] > 0) continue;
            const bgw_chi_q &q = d->q[iq];
            if (q.head < 0) continue;
            const SplitQ &e = L.qs[i];
            Timed tm(h, BGW_KERNEL_HEADWING, st);
            double2 *hw = (double2 *)(ws + P.off_hw);
            BGW_TRY(launch_headwing(e.M, e.K, q.ng, q.head, e.w, e.wstride, vq, kHeadSplits, hw, st));
            // the finalize skips row/column head, so these writes may come first
            BGW_TRY(launch_headwing_write(hw, kHeadSplits, vq, q.ng, q.head, q.prefactor, (double2 *)q.chi, d->nw,
                                          P.vpq == 2 ? 1 : 0, d->accumulate, st));
        }
    }
    Timed tm(h, BGW_KERNEL_FINALIZE, st);
    BGW_TRY(launch_finalize_batch(dfin, P.nout, P.maxng, st));
    return BGW_OK;
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
    k = fnv(k, &d->axis, sizeof(int));
    k = fnv(k, &d->broadening, sizeof(double));
    k = fnv(k, &h->ws.p, sizeof(void *));
    k = fnv(k, &h->ws.bytes, sizeof(size_t));
    k = fnv(k, &h->chi->generation, sizeof(unsigned));
    return k;
}

int run_eager(bgw_handle_t h, const bgw_chi_desc *d, ChiPlan &P, hipStream_t st) {
    ChiState *s = state(h);
    BGW_TRY(ensure_ws(h, P.ws_bytes, st));
    char *ws = (char *)h->ws.p;
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
    bind_plan(d, P, ws, (char *)s->tables.p);
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
    auto g = std::make_unique<GraphEntry>();
    g->key = key;
    BGW_HIP(hipMalloc(&g->tables.p, P.table_bytes));
    g->tables.bytes = P.table_bytes;
    bind_plan(d, P, ws, (char *)g->tables.p);
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

extern "C" int bgw_chi0_workspace(bgw_handle_t h, const bgw_chi_desc *d, size_t *bytes) {
    clear_error();
    BGW_TRY(check_chi_desc(d));
    if (!h || !bytes) return fail(BGW_ERR_ARG, "null handle or output");
    BGW_TRY(set_device(h));
    ChiPlan P;
    BGW_TRY(make_plan(h, d, P, 0, 0, 0));
    *bytes = P.ws_bytes;
    return BGW_OK;
}

namespace bgw {
namespace {
constexpr long long kMaxKxPairs = 65536;

int check_kx_desc(const bgw_kx_desc *d) {
    if (!d || !d->M || !d->v || !d->kx) return fail(BGW_ERR_ARG, "bad exchange-kernel descriptor");
    if (d->K < 1 || d->K > kMaxKxPairs) return fail(BGW_ERR_UNSUPPORTED, "exchange kernel: K outside 1 .. 65536");
    if (d->ng < 1) return fail(BGW_ERR_ARG, "exchange kernel: ng must be >= 1");
    if (d->head < -1 || d->head >= d->ng) return fail(BGW_ERR_ARG, "exchange kernel: head index out of range");
    if (d->precision != BGW_FP64 && d->precision != BGW_SPLIT_BF16) return fail(BGW_ERR_ARG, "unknown precision");
    return BGW_OK;
}

// The chi-sum problem of the exchange kernel: "pairs" are the ng G vectors
// of the transposed MT [ng][K], the output index runs over the K pairs, the
// weights are v (given), and no output row needs the FP64 head treatment.
struct KxProblem {
    bgw_chi_q q;
    bgw_chi_desc cd;
    double omega = 0.0;
    void set(const bgw_kx_desc *d, const void *MT) {
        std::memset(&q, 0, sizeof(q));
        q.ng = (int)d->K;
        q.nk = 1;
        q.nv = 1;
        q.nc = d->ng;
        q.M = (const double *)MT;
        q.ev = d->v;
        q.ec = d->v;
        q.head = -1;
        q.prefactor = d->prefactor;
        q.chi = d->kx;
        std::memset(&cd, 0, sizeof(cd));
        cd.nq = 1;
        cd.q = &q;
        cd.nw = 1;
        cd.omega = &omega;
        cd.precision = d->precision;
        cd.axis = BGW_AXIS_IMAG;
    }
};
}  // namespace
}  // namespace bgw

extern "C" int bgw_bse_kx_workspace(bgw_handle_t h, const bgw_kx_desc *d, size_t *bytes) {
    clear_error();
    BGW_TRY(check_kx_desc(d));
    if (!h || !bytes) return fail(BGW_ERR_ARG, "null handle or output");
    BGW_TRY(set_device(h));
    KxProblem kp;
    kp.set(d, d->M);  // any non-null placeholder: sizes only
    ChiPlan P;
    BGW_TRY(make_plan(h, &kp.cd, P, 0, 0, 0, sizeof(double2) * (size_t)d->K * d->ng, true));
    *bytes = P.ws_bytes;
    return BGW_OK;
}

extern "C" int bgw_bse_kx(bgw_handle_t h, const bgw_kx_desc *d, void *stream) {
    clear_error();
    BGW_TRY(check_kx_desc(d));
    if (!h) return fail(BGW_ERR_ARG, "null handle");
    BGW_TRY(set_device(h));
    hipStream_t st = (hipStream_t)stream;
    const size_t mt_bytes = sizeof(double2) * (size_t)d->K * d->ng;
    KxProblem kp;
    ChiPlan P0;
    kp.set(d, d->M);
    BGW_TRY(make_plan(h, &kp.cd, P0, 0, 0, 0, mt_bytes, true));
    BGW_TRY(ensure_ws(h, P0.ws_bytes, st));
    double2 *MT = (double2 *)h->ws.p;  // the plan keeps the first mt_bytes free
    BGW_TRY(launch_transpose_pairs((const double2 *)d->M, d->K, d->ng, d->head, MT, st));
    kp.set(d, MT);
    ChiPlan P;
    BGW_TRY(make_plan(h, &kp.cd, P, 0, 0, 0, mt_bytes, true));
    return run_eager(h, &kp.cd, P, st);
}

namespace bgw {
namespace {
int check_sigma_desc(const bgw_sigma_desc *d) {
    if (!d || !d->M || !d->v || !d->sigma) return fail(BGW_ERR_ARG, "bad self-energy descriptor");
    if (d->kind != BGW_SIGMA_X && d->kind != BGW_SIGMA_SX && d->kind != BGW_SIGMA_CH)
        return fail(BGW_ERR_ARG, "unknown self-energy kind");
    if (d->ninner < 1 || d->nouter < 1 || d->nouter > 65536 || d->ng < 1)
        return fail(BGW_ERR_ARG, "self-energy: sizes out of range");
    if (d->ng > kMaxNg) return fail(BGW_ERR_UNSUPPORTED, "self-energy: ng > 12288");
    if ((long long)d->ninner * d->ng > 0x7fffffffll) return fail(BGW_ERR_UNSUPPORTED, "self-energy: ninner * ng too large");
    if (d->precision != BGW_FP64 && d->precision != BGW_SPLIT_BF16) return fail(BGW_ERR_ARG, "unknown precision");
    if (d->kind != BGW_SIGMA_X) {
        if (!d->epsinv) return fail(BGW_ERR_ARG, "self-energy: screened kinds need eps^-1");
        if (d->precision != BGW_FP64) return fail(BGW_ERR_UNSUPPORTED, "self-energy: SX and CH are FP64 only");
    } else if (d->head < -1 || d->head >= d->ng) {
        return fail(BGW_ERR_ARG, "self-energy: head index out of range");
    }
    return BGW_OK;
}

// The bare exchange as a chi-sum: "pairs" are the (inner state, G) rows of
// MT2[i ng + G][n] = M[i][n][G], the weights v(G) repeated per inner state,
// the output over the outer states, prefactor -pf.
struct SigmaXProblem {
    bgw_chi_q q;
    bgw_chi_desc cd;
    double omega = 0.0;
    void set(const bgw_sigma_desc *d, const void *MT2, const double *w) {
        std::memset(&q, 0, sizeof(q));
        q.ng = d->nouter;
        q.nk = 1;
        q.nv = 1;
        q.nc = d->ninner * d->ng;
        q.M = (const double *)MT2;
        q.ev = w;
        q.ec = w;
        q.head = -1;
        q.prefactor = -d->prefactor;
        q.chi = d->sigma;
        std::memset(&cd, 0, sizeof(cd));
        cd.nq = 1;
        cd.q = &q;
        cd.nw = 1;
        cd.omega = &omega;
        cd.precision = d->precision;
        cd.accumulate = d->accumulate;
        cd.axis = BGW_AXIS_IMAG;
    }
};

// One P^H Q product: tile edge, K-split count and the split ranges.
GemmProb gemm_plan(const double2 *P, long long ldp, int m, const double2 *Q, long long ldq, int n, long long K,
                   int &tile) {
    GemmProb g;
    std::memset(&g, 0, sizeof(g));
    tile = std::min(m, n) >= 64 ? 64 : 32;
    g.P = P;
    g.Q = Q;
    g.K = K;
    g.ldp = ldp;
    g.ldq = ldq;
    g.m = m;
    g.n = n;
    g.ntr = (m + tile - 1) / tile;
    g.ntc = (n + tile - 1) / tile;
    const long long tiles = (long long)g.ntr * g.ntc;
    long long ns = std::max<long long>(1, (3LL * device_cus() + tiles - 1) / tiles);
    ns = std::min<long long>(ns, std::max<long long>(1, K / 64));
    ns = std::min<long long>(ns, 256);
    long long kper = (K + ns - 1) / ns;
    kper = (kper + 15) / 16 * 16;
    g.kper = kper;
    g.ns = (int)((K + kper - 1) / kper);
    return g;
}

// Workspace carve-up of the screened kinds: WT, M^T, W M, the regrouped
// operands and the partial sums of the two products.
struct SigmaWLayout {
    size_t wt = 0, mt = 0, b = 0, mt2 = 0, b2 = 0, p1 = 0, p2 = 0, total = 0;
    int tile1 = 64, tile2 = 32;
    GemmProb g1, g2;
};

SigmaWLayout sigma_w_layout(const bgw_sigma_desc *d, char *ws) {
    SigmaWLayout L;
    const long long ng = d->ng, K = (long long)d->ninner * d->nouter;
    size_t off = 0;
    L.wt = off;
    off += al256(sizeof(double2) * ng * ng);
    L.mt = off;
    off += al256(sizeof(double2) * ng * K);
    L.b = off;
    off += al256(sizeof(double2) * ng * K);
    L.mt2 = off;
    off += al256(sizeof(double2) * ng * K);
    L.b2 = off;
    off += al256(sizeof(double2) * ng * K);
    L.g1 = gemm_plan((const double2 *)(ws + L.wt), ng, d->ng, (const double2 *)(ws + L.mt), K, (int)K, ng, L.tile1);
    L.p1 = off;
    if (L.g1.ns > 1) off += al256(sizeof(double2) * (size_t)L.g1.ns * ng * K);
    L.g1.out = (double2 *)(ws + (L.g1.ns > 1 ? L.p1 : L.b));
    L.g2 = gemm_plan((const double2 *)(ws + L.mt2), d->nouter, d->nouter, (const double2 *)(ws + L.b2), d->nouter,
                     d->nouter, (long long)d->ninner * ng, L.tile2);
    L.p2 = off;
    off += al256(sizeof(double2) * (size_t)L.g2.ns * d->nouter * d->nouter);
    L.g2.out = (double2 *)(ws + L.p2);
    L.total = off + 256;
    return L;
}
}  // namespace
}  // namespace bgw

extern "C" int bgw_sigma_workspace(bgw_handle_t h, const bgw_sigma_desc *d, size_t *bytes) {
    clear_error();
    BGW_TRY(check_sigma_desc(d));
    if (!h || !bytes) return fail(BGW_ERR_ARG, "null handle or output");
    BGW_TRY(set_device(h));
    if (d->kind == BGW_SIGMA_X) {
        const size_t pre = al256(sizeof(double2) * (size_t)d->ninner * d->ng * d->nouter) +
                           al256(sizeof(double) * (size_t)d->ninner * d->ng);
        SigmaXProblem sp;
        sp.set(d, d->M, d->v);
        ChiPlan P;
        BGW_TRY(make_plan(h, &sp.cd, P, 0, 0, 0, pre, true));
        *bytes = P.ws_bytes;
    } else {
        *bytes = sigma_w_layout(d, nullptr).total;
    }
    return BGW_OK;
}

extern "C" int bgw_sigma(bgw_handle_t h, const bgw_sigma_desc *d, void *stream) {
    clear_error();
    BGW_TRY(check_sigma_desc(d));
    if (!h) return fail(BGW_ERR_ARG, "null handle");
    BGW_TRY(set_device(h));
    hipStream_t st = (hipStream_t)stream;
    const long long ng = d->ng, ni = d->ninner, no = d->nouter;
    if (d->kind == BGW_SIGMA_X) {
        const size_t mt2 = al256(sizeof(double2) * (size_t)ni * ng * no);
        const size_t pre = mt2 + al256(sizeof(double) * (size_t)ni * ng);
        SigmaXProblem sp;
        ChiPlan P0;
        sp.set(d, d->M, d->v);
        BGW_TRY(make_plan(h, &sp.cd, P0, 0, 0, 0, pre, true));
        BGW_TRY(ensure_ws(h, P0.ws_bytes, st));
        char *ws = (char *)h->ws.p;
        double2 *MT2 = (double2 *)ws;
        double *w = (double *)(ws + mt2);
        BGW_TRY(launch_transpose_pairs((const double2 *)d->M, no, d->ng, d->head, MT2, st, d->ninner));
        BGW_TRY(launch_sigma_weights(d->v, d->ng, d->ninner, w, st));
        sp.set(d, MT2, w);
        ChiPlan P;
        BGW_TRY(make_plan(h, &sp.cd, P, 0, 0, 0, pre, true));
        return run_eager(h, &sp.cd, P, st);
    }
    BGW_TRY(ensure_ws(h, sigma_w_layout(d, nullptr).total, st));
    char *ws = (char *)h->ws.p;
    SigmaWLayout L = sigma_w_layout(d, ws);
    const double2 *M = (const double2 *)d->M;
    BGW_TRY(launch_sigma_wt((const double2 *)d->epsinv, d->v, d->ng, d->kind == BGW_SIGMA_CH, (double2 *)(ws + L.wt), st));
    BGW_TRY(launch_transpose_pairs(M, ni * no, d->ng, -1, (double2 *)(ws + L.mt), st));
    BGW_TRY(launch_gemm_phq(L.g1, L.tile1, st));
    if (L.g1.ns > 1)
        BGW_TRY(launch_gemm_finalize(L.g1.out, L.g1.ns, ng * ni * no, 1.0, (double2 *)(ws + L.b), 0, st));
    BGW_TRY(launch_sigma_regroup((const double2 *)(ws + L.b), d->ng, d->ninner, d->nouter, (double2 *)(ws + L.b2), st));
    BGW_TRY(launch_transpose_pairs(M, no, d->ng, -1, (double2 *)(ws + L.mt2), st, d->ninner));
    BGW_TRY(launch_gemm_phq(L.g2, L.tile2, st));
    const double scale = d->kind == BGW_SIGMA_CH ? 0.5 * d->prefactor : -d->prefactor;
    return launch_gemm_finalize(L.g2.out, L.g2.ns, no * no, scale, (double2 *)d->sigma, d->accumulate, st);
}

namespace bgw {
namespace {
// Everything one real-flavor chi0 call launches: weights, the persistent real
// rank-K update over every (vector, K split, upper tile) item, the finalize.
struct RealChiPlan {
    std::vector<WProb> wts;
    std::vector<SyrkProb> sy;
    std::vector<SyrkFin> fin;
    std::vector<size_t> w_off, part_off;  // per vector ((size_t)-1: in place)
    size_t off_tab = 0, ws_bytes = 0, tab_bytes = 0;
    long long maxK = 0, nitems = 0;
    int maxng = 0, grid = 0;
};

int check_chi_real(const bgw_chi_desc *d) {
    BGW_TRY(check_chi_desc(d));
    if (d->precision != BGW_FP64) return fail(BGW_ERR_UNSUPPORTED, "real flavor: FP64 only");
    if (d->axis != BGW_AXIS_IMAG) return fail(BGW_ERR_UNSUPPORTED, "real flavor: imaginary axis only");
    if (d->use_graph) return fail(BGW_ERR_UNSUPPORTED, "real flavor: no graph capture");
    return BGW_OK;
}

void make_real_plan(const bgw_chi_desc *d, RealChiPlan &P) {
    constexpr int RT = kSyrkTile, RKC = kSyrkK;
    const int nvec = d->nq * d->nw;
    size_t off = 0;
    long long total_tiles = 0;
    for (int iq = 0; iq < d->nq; ++iq) {
        const bgw_chi_q &q = d->q[iq];
        P.maxK = std::max(P.maxK, q_pairs(q));
        P.maxng = std::max(P.maxng, q.ng);
        const long long nt = (q.ng + RT - 1) / RT;
        total_tiles += nt * (nt + 1) / 2 * d->nw;
        for (int iw = 0; iw < d->nw; ++iw) {
            WProb wp;
            wp.ev = q.ev;
            wp.ec = q.ec;
            wp.w = nullptr;
            wp.omega_ha = d->omega[iw] / kHartreeEv;
            wp.delta_ha = 0.0;
            wp.nk = q.nk;
            wp.nv = q.nv;
            wp.nc = q.nc;
            wp.kind = kWeightImag;
            P.wts.push_back(wp);
            P.w_off.push_back(off);
            off += al256(sizeof(double) * q_pairs(q));
        }
    }
    const long long slots = (long long)device_cus() * syrk_blocks_per_cu();
    const long long ns = choose_splits(total_tiles, slots, 8, 64);
    long long item0 = 0;
    for (int v = 0; v < nvec; ++v) {
        const int iq = v / d->nw, iw = v % d->nw;
        const bgw_chi_q &q = d->q[iq];
        const long long K = q_pairs(q);
        long long nsp = std::min<long long>(ns, std::max<long long>(1, K / (8 * RKC)));
        long long kper = (K + nsp - 1) / nsp;
        kper = (kper + RKC - 1) / RKC * RKC;
        nsp = (K + kper - 1) / kper;
        const bool inplace = nsp == 1 && !d->accumulate;
        SyrkProb sp;
        std::memset(&sp, 0, sizeof(sp));
        sp.M = q.M;
        sp.K = K;
        sp.kper = kper;
        sp.ng = q.ng;
        sp.nt = (q.ng + RT - 1) / RT;
        sp.ns = (int)nsp;
        sp.item0 = item0;
        sp.nitems = ((long long)sp.nt * (sp.nt + 1) / 2 * nsp + 7) / 8 * 8;
        item0 += sp.nitems;
        SyrkFin f;
        std::memset(&f, 0, sizeof(f));
        f.chi = q.chi + (size_t)iw * q.ng * q.ng;
        f.pf = q.prefactor;
        f.ns = (int)nsp;
        f.ng = q.ng;
        f.accumulate = d->accumulate;
        f.inplace = inplace ? 1 : 0;
        if (inplace) {
            P.part_off.push_back((size_t)-1);
        } else {
            P.part_off.push_back(off);
            off += al256(sizeof(double) * (size_t)nsp * q.ng * q.ng);
        }
        P.sy.push_back(sp);
        P.fin.push_back(f);
    }
    P.nitems = item0;
    P.grid = (int)(slots / 8 * 8);
    P.off_tab = off;
    P.tab_bytes = al256(sizeof(SyrkProb) * P.sy.size()) + al256(sizeof(SyrkFin) * P.fin.size()) +
                  al256(sizeof(WProb) * P.wts.size());
    P.ws_bytes = off + P.tab_bytes + 256;
}
}  // namespace
}  // namespace bgw

extern "C" int bgw_chi0_real_workspace(bgw_handle_t h, const bgw_chi_desc *d, size_t *bytes) {
    clear_error();
    BGW_TRY(check_chi_real(d));
    if (!h || !bytes) return fail(BGW_ERR_ARG, "null handle or output");
    BGW_TRY(set_device(h));
    RealChiPlan P;
    make_real_plan(d, P);
    *bytes = P.ws_bytes;
    return BGW_OK;
}

extern "C" int bgw_chi0_real(bgw_handle_t h, const bgw_chi_desc *d, void *stream) {
    clear_error();
    BGW_TRY(check_chi_real(d));
    if (!h) return fail(BGW_ERR_ARG, "null handle");
    BGW_TRY(set_device(h));
    hipStream_t st = (hipStream_t)stream;
    RealChiPlan P;
    make_real_plan(d, P);
    BGW_TRY(ensure_ws(h, P.ws_bytes, st));
    char *ws = (char *)h->ws.p;
    for (size_t v = 0; v < P.sy.size(); ++v) {
        double *w = (double *)(ws + P.w_off[v]);
        P.wts[v].w = w;
        P.sy[v].w = w;
        double *part = P.part_off[v] == (size_t)-1 ? P.fin[v].chi : (double *)(ws + P.part_off[v]);
        P.sy[v].out = part;
        P.fin[v].part = part;
    }
    // device tables: copied from host memory, then the host copies may go
    std::vector<char> host(P.tab_bytes, 0);
    const size_t o_fin = al256(sizeof(SyrkProb) * P.sy.size());
    const size_t o_w = o_fin + al256(sizeof(SyrkFin) * P.fin.size());
    std::memcpy(host.data(), P.sy.data(), sizeof(SyrkProb) * P.sy.size());
    std::memcpy(host.data() + o_fin, P.fin.data(), sizeof(SyrkFin) * P.fin.size());
    std::memcpy(host.data() + o_w, P.wts.data(), sizeof(WProb) * P.wts.size());
    char *tab = ws + P.off_tab;
    BGW_HIP(hipMemcpyAsync(tab, host.data(), P.tab_bytes, hipMemcpyHostToDevice, st));
    BGW_HIP(hipStreamSynchronize(st));
    {
        Timed tm(h, BGW_KERNEL_WEIGHTS, st);
        BGW_TRY(launch_weights_batch((const WProb *)(tab + o_w), (int)P.wts.size(), P.maxK, st));
    }
    {
        Timed tm(h, BGW_KERNEL_HERK, st);
        BGW_TRY(launch_syrk_batch((const SyrkProb *)tab, (int)P.sy.size(), P.nitems, P.grid, st));
    }
    Timed tm(h, BGW_KERNEL_FINALIZE, st);
    return launch_syrk_finalize((const SyrkFin *)(tab + o_fin), (int)P.fin.size(), P.maxng, st);
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
            for (int ns : {1, 2, 4, 8, 16}) cands.emplace_back(0, 0, ns);
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
