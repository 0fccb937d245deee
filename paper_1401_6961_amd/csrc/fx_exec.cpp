// Exchange execution: density norms, the level-synchronous hextree traversal
// of Eqs. (7a-d) with the metric query of Eq. (8), K-block work units, one
// class-kernel launch per angular-momentum class and precision, and the final
// scaling of Eq. (6).
//
// Every size the traversal produces (ADs and entries per level, units per
// class) is written and read on the device: the host launches a fixed
// sequence of kernels whose grids are host-known bounds, so a call enqueues
// its work and returns without waiting for it, and the whole sequence can be
// captured once in a hipGraph and replayed.  Buffers are sized from the
// sizes seen by earlier calls on the same tree (FxSizeHint); the first call
// on a tree learns them in a traversal-only pass.  A level that exceeds its
// capacity sets a device flag: a call that waits for its result (statistics
// requested) then splits the work into K row ranges and runs each range
// again, and a call that does not wait writes NaN into K and records the
// sizes it needed for the next call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fx.h"
#include "eri_flops.h"
#include "eri_table.h"
#include "fx_costmodel.h"
#include "fx_host.h"
#include "fx_internal.h"
#include "fx_kernels.h"

namespace {

constexpr size_t kAlign = 256;
constexpr long kEntryMax = 0xFFFFFFFFL;   // expansion positions are 32-bit
constexpr int kBins = 32;
constexpr size_t kDefaultWorkspace = size_t(4) << 30;   // default workspace budget of one call
constexpr int kDefaultMaxRanges = 64;                     // ... unless that takes more K row ranges

// shared screen per (l_a, l_d) group where the leaves allow it (process-wide
// switch, off by default: on the 1000-atom cluster the screen kernels took
// 0.87 s and the class kernels did not get faster, 15.80 s against 14.91 s)
int g_group_screen = 0;

// progress hook of long one-system calls (process-wide)
fx_progress_fn g_progress = nullptr;
void* g_progress_ctx = nullptr;

struct ProgressMsg {
    fx_progress_fn fn;
    void* ctx;
    int32_t done, total;
};

void progress_trampoline(void* p) {
    std::unique_ptr<ProgressMsg> m(static_cast<ProgressMsg*>(p));
    m->fn(m->done, m->total, m->ctx);
}

// Sequential sub-allocation of one device block; a null base only measures.
struct Carve {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    T* take(size_t n) {
        off = (off + kAlign - 1) / kAlign * kAlign;
        T* p = base ? (T*)(base + off) : nullptr;
        off += sizeof(T) * std::max<size_t>(n, 1);
        return p;
    }
};

// Host bounds of one system's device sizes.
struct Caps {
    long e_in = 0, e_leaf = 0;      // entry capacities (inner levels, leaf level)
    std::vector<long> e_lvl;        // per level: bound of its entry count
    std::vector<long> ad_lvl;       // per level: bound of its AD count
    long ad_max = 0, items = 0;     // largest AD bound; leaf items bound
    long ucap[9] = {0};             // units per (la, ld): S_la * S_ld
    long units = 0;
};

// Device buffers of one system (one traversal chunk at a time).
struct SysBufs {
    double* Pn = nullptr;
    double* Pn2 = nullptr;          // norms of a further density (several densities)
    std::vector<double*> Psq;
    int* mismatch = nullptr;
    int2* ad[2] = {nullptr, nullptr};
    long* off[2] = {nullptr, nullptr};
    int2* ebc[2] = {nullptr, nullptr};
    int* epar[2] = {nullptr, nullptr};
    int2* leafbc = nullptr;
    uint8_t* mask = nullptr;
    uint32_t* pos = nullptr;
    int* flag = nullptr;
    long* adpos = nullptr;
    int* ucnt = nullptr;
    long* upos = nullptr;
    int* units = nullptr;
    int2* sorted = nullptr;
    long* cls_off = nullptr;
    unsigned long long* cpart = nullptr;   // partition sums of the chunk being traversed
    uint32_t* screen = nullptr;            // per leaf entry: the (l_a, l_d) group's screen (one-shell-per-l leaves)
    double* acc[FX_MAX_DENS] = {nullptr, nullptr};
};

struct Sys {
    const fx_tree* T = nullptr;
    const double* P[FX_MAX_DENS] = {nullptr, nullptr};
    double* K[FX_MAX_DENS] = {nullptr, nullptr};
    Caps caps;
    SysBufs b;
    FxDevCounts* cnt = nullptr;   // element of the call's count array
    int a_lo = 0, a_hi = 0;       // K row range (tree-order shells) of the chunk being run
};

// Buffers shared by the systems of a call.
struct Shared {
    unsigned long long* counters = nullptr;   // [81][2][3] class counters, then [3][FX_PART_SLOTS] partition
    unsigned long long* part = nullptr;
    FxDevCounts* cnts = nullptr;              // one per system
    FxDevRun* run = nullptr;                  // call totals and sizes seen (next call's capacities)
    unsigned long long* rows = nullptr;       // leaf entries per leaf row (first call on a tree)
    double* beta32 = nullptr;                 // sum of beta over the quartets evaluated in FP32
    long* partial = nullptr;
    long* total = nullptr;
    // scheduling
    float4* feat = nullptr;
    float* cost = nullptr;
    uint8_t* key = nullptr;
    int* bcount = nullptr;
    long* bpos = nullptr;
    int* order = nullptr;
    float* times = nullptr;
    // batched unit lists
    int* munits = nullptr;
    int* msys = nullptr;
    long* moff = nullptr;
    long* mb = nullptr;
    FxSys* dsys = nullptr;
};

struct Opts {
    fx_exchange_opts o;
    bool wait = false;       // the call waits for its result (statistics, profile, timing probes)
    bool graph = false;
    bool sched = false;
    bool mlp = false;
};

long ipow4(long x) {
    const long y = x * x;
    return (y > 0 && y < (1L << 31)) ? y * y : (1L << 62);
}

using Ranges = std::vector<std::pair<int, int>>;

// Capacities of one system from the tree, the entry capacities and the K row
// ranges the traversal will be run over: a range's ADs have their A node
// among the level's nodes that meet it, and its units their a shell in it.
Caps make_caps(const fx_tree* T, long e_in, long e_leaf, const Ranges& ranges, const long* units_seen = nullptr) {
    Caps c;
    const int nl = (int)T->levels.size();
    c.e_in = std::max(1L, std::min(e_in, kEntryMax));
    c.e_leaf = std::max(1L, std::min(e_leaf, kEntryMax));
    c.e_lvl.resize(nl);
    c.ad_lvl.resize(nl);
    for (int k = 0; k < nl; ++k) {
        const Level& L = T->levels[k];
        const long nk = (long)L.sL.size();
        long na = 0;
        for (const auto& r : ranges) {
            // a level's nodes partition the shells in order
            const long first = std::upper_bound(L.sR.begin(), L.sR.end(), r.first) - L.sR.begin();
            const long last = std::lower_bound(L.sL.begin(), L.sL.end(), r.second) - L.sL.begin();
            na = std::max(na, last - first);
        }
        c.ad_lvl[k] = std::max(1L, na) * nk;
        c.e_lvl[k] = std::min(k == nl - 1 ? c.e_leaf : c.e_in, ipow4(nk));
        c.ad_max = std::max(c.ad_max, c.ad_lvl[k]);
    }
    c.e_in = std::max(1L, std::min(c.e_in, nl > 1 ? *std::max_element(c.e_lvl.begin(), c.e_lvl.end() - 1) : 1L));
    c.e_leaf = std::max(1L, c.e_lvl[nl - 1]);
    c.items = c.ad_lvl[nl - 1];
    std::vector<long> pre[3];
    for (int x = 0; x < 3; ++x) pre[x].assign(T->S + 1, 0);
    for (int i = 0; i < T->S; ++i)
        for (int x = 0; x < 3; ++x) pre[x][i + 1] = pre[x][i] + (T->l[i] == x);
    long nra[3] = {0, 0, 0};
    for (const auto& r : ranges)
        for (int x = 0; x < 3; ++x) nra[x] = std::max(nra[x], pre[x][r.second] - pre[x][r.first]);
    c.units = 0;
    for (int la = 0; la < 3; ++la)
        for (int ld = 0; ld < 3; ++ld) {
            long u = nra[la] * pre[ld][T->S];
            // the counts earlier calls saw per range, with a margin: launch grids
            // follow the units that exist rather than every (a, d) pair
            if (units_seen) u = std::min(u, units_seen[la * 3 + ld] + units_seen[la * 3 + ld] / 4 + 1024);
            c.ucap[la * 3 + ld] = u;
            c.units += u;
        }
    return c;
}

Ranges whole_rows(const fx_tree* T) { return Ranges{{0, T->S}}; }

long scan_tiles_max(const Caps& c) {
    long m = std::max({fx_scan_tiles(4 * c.e_in), fx_scan_tiles(4 * c.ad_max), fx_scan_tiles(9 * c.items)});
    return m;
}

// leaves with at most one shell of each l (and more than one shell): the
// class kernels of an (l_a, l_d) group read one shared screen of each entry
bool group_screen(const fx_tree* T) { return T->basis.leaf_one != nullptr && !T->single_shell_leaves; }

void carve_sys(Carve& cv, Sys& s, int ndens, bool own_acc) {
    const fx_tree* T = s.T;
    const Caps& c = s.caps;
    SysBufs& b = s.b;
    const int nl = (int)T->levels.size();
    b.Pn = cv.take<double>((size_t)T->S * T->S);
    if (ndens > 1) b.Pn2 = cv.take<double>((size_t)T->S * T->S);
    b.Psq.resize(nl);
    for (int k = 0; k < nl; ++k) {
        const size_t nk = T->levels[k].sL.size();
        b.Psq[k] = cv.take<double>(nk * nk);
    }
    b.mismatch = cv.take<int>(1);
    for (int i = 0; i < 2; ++i) {
        b.ad[i] = cv.take<int2>(c.ad_max);
        b.off[i] = cv.take<long>(c.ad_max + 1);
        b.ebc[i] = cv.take<int2>(nl > 1 ? c.e_in : 1);
        b.epar[i] = cv.take<int>(nl > 1 ? c.e_in : 1);
    }
    b.leafbc = cv.take<int2>(c.e_leaf);
    b.mask = cv.take<uint8_t>(4 * c.e_in);
    b.pos = cv.take<uint32_t>(4 * c.e_in + 1);
    b.flag = cv.take<int>(4 * c.ad_max);
    b.adpos = cv.take<long>(4 * c.ad_max + 1);
    b.ucnt = cv.take<int>(9 * c.items);
    b.upos = cv.take<long>(9 * c.items + 1);
    b.units = cv.take<int>(3 * c.units);
    if (T->single_shell_leaves) {
        b.sorted = cv.take<int2>(c.e_leaf);
        b.cls_off = cv.take<long>(10 * c.items);
    }
    b.cpart = cv.take<unsigned long long>(3 * FX_PART_SLOTS);
    if (g_group_screen && group_screen(T)) b.screen = cv.take<uint32_t>(c.e_leaf);
    for (int j = 0; j < ndens; ++j) b.acc[j] = own_acc ? cv.take<double>((size_t)T->n * T->n) : nullptr;
}

void carve_shared(Carve& cv, Shared& sh, std::vector<Sys>& sys, const Opts& op) {
    const int count = (int)sys.size();
    sh.counters = cv.take<unsigned long long>(81 * 2 * 3 + 3 * FX_PART_SLOTS);
    sh.part = sh.counters ? sh.counters + 81 * 2 * 3 : nullptr;
    sh.beta32 = cv.take<double>(1);
    sh.cnts = cv.take<FxDevCounts>(count);
    sh.run = cv.take<FxDevRun>(1);
    size_t nleaf = 1;
    for (auto& s : sys) nleaf = std::max(nleaf, s.T->levels.back().sL.size());
    sh.rows = cv.take<unsigned long long>(nleaf);
    long tiles = 1, umax = 0;
    for (auto& s : sys) tiles = std::max(tiles, scan_tiles_max(s.caps));
    for (int k = 0; k < 9; ++k) {
        long u = 0;
        for (auto& s : sys) u += s.caps.ucap[k];
        umax = std::max(umax, u);
    }
    const long nblk = fx_bin_blocks(std::max(1L, umax));
    if (op.sched || g_recording) {
        sh.feat = cv.take<float4>(umax);
        sh.cost = cv.take<float>(umax);
    }
    if (op.sched) {
        sh.key = cv.take<uint8_t>(umax);
        sh.bcount = cv.take<int>((size_t)kBins * nblk);
        sh.bpos = cv.take<long>((size_t)kBins * nblk + 1);
        sh.order = cv.take<int>(umax);
        tiles = std::max(tiles, fx_scan_tiles((long)kBins * nblk));
    }
    if (g_recording) sh.times = cv.take<float>(umax);
    sh.partial = cv.take<long>(tiles);
    sh.total = cv.take<long>(1);
    if (count > 1) {
        sh.munits = cv.take<int>(3 * umax);
        sh.msys = cv.take<int>(umax);
        sh.moff = cv.take<long>(count);
        sh.mb = cv.take<long>(2 * 9);
        sh.dsys = cv.take<FxSys>(count);
    }
}

// ---------------------------------------------------------------------------
// the steps
// ---------------------------------------------------------------------------

// Density norms (Eq. 8): shell-level Pn (the largest over the densities),
// squared block norms per level, and the bitwise symmetry test of P.
void density_norms(Sys& s, int ndens, bool allow_sym, hipStream_t st) {
    const fx_tree* T = s.T;
    SysBufs& b = s.b;
    const int S = T->S;
    const long n = T->n;
    fx_launch_pnorm(s.P[0], n, T->basis.l, T->basis.f0, S, b.Pn, st);
    for (int j = 1; j < ndens; ++j) {
        fx_launch_pnorm(s.P[j], n, T->basis.l, T->basis.f0, S, b.Pn2, st);
        fx_launch_max_inplace(b.Pn, b.Pn2, (long)S * S, st);
    }
    const int nl = (int)T->levels.size();
    for (int k = nl - 1; k >= 0; --k) {
        const int nk = (int)T->levels[k].sL.size();
        if (k == nl - 1)
            fx_launch_leaf_sq(b.Pn, S, T->d_sL[k], T->d_sR[k], nk, b.Psq[k], st);
        else
            fx_launch_level_up(b.Psq[k + 1], (int)T->levels[k + 1].sL.size(), T->d_ch0[k], T->d_nch[k], nk, b.Psq[k],
                               st);
    }
    fx_launch_fill_i32(b.mismatch, 1, 0, st);
    if (allow_sym)
        for (int j = 0; j < ndens; ++j) fx_launch_psym(s.P[j], n, b.mismatch, st);
}

// Traversal of one K row range [a_lo, a_hi): root task, then one expansion
// per level; leaves the leaf ADs and entries in the buffers.
void traverse(Sys& s, double tau, double tau_ovlp, bool allow_sym, bool count_root, hipStream_t st,
              const Shared& sh) {
    const fx_tree* T = s.T;
    const Caps& c = s.caps;
    SysBufs& b = s.b;
    const int nl = (int)T->levels.size();
    const double tau2 = tau * tau;
    FxDevCounts* cnt = s.cnt;
    fx_launch_set_sym(cnt, b.mismatch, allow_sym ? 1 : 0, st);
    fx_launch_fill_u64(b.cpart, 3 * FX_PART_SLOTS, 0ull, st);
    const unsigned long long n = (unsigned long long)T->n;
    fx_launch_root(cnt, T->d_Qsq[0], b.Psq[0], tau2, b.ad[0], b.off[0], nl > 1 ? b.ebc[0] : b.leafbc,
                   nl > 1 ? b.epar[0] : nullptr, b.cpart, n * n * n * n, nl == 1 ? 1 : 0, count_root ? 1 : 0, st);
    for (int k = 0; k + 1 < nl; ++k) {
        FxLevelArgs L{};
        L.ad = b.ad[k & 1];
        L.bc_off = b.off[k & 1];
        L.bc = b.ebc[k & 1];
        L.bc_parent = b.epar[k & 1];
        L.cnt = cnt;
        L.k = k;
        L.ch0 = T->d_ch0[k];
        L.nch = T->d_nch[k];
        L.Qsq = T->d_Qsq[k + 1];
        L.Psq = b.Psq[k + 1];
        L.nk1 = (int)T->levels[k + 1].sL.size();
        L.tau2 = tau2;
        L.Smx = T->d_Smx[k + 1];
        L.tau_ovlp = tau_ovlp;
        L.sL1 = T->d_sL[k + 1];
        L.sR1 = T->d_sR[k + 1];
        L.a_lo = s.a_lo;
        L.a_hi = s.a_hi;
        L.nf1 = T->d_nf[k + 1];
        L.leaf_next = (k + 1 == nl - 1) ? 1 : 0;
        L.part = b.cpart;
        const bool leaf = k + 1 == nl - 1;
        const long e_max = c.e_lvl[k], nad_max = c.ad_lvl[k];
        const long cap_next = leaf ? c.e_leaf : c.e_in;
        fx_launch_expand_mask(L, e_max, b.mask, st);
        fx_scan_popc_u8_dev(b.mask, &cnt->ne[k], 4, 4 * e_max, b.pos, sh.partial, &cnt->tot[0], st);
        fx_launch_commit_entries(cnt, k, &cnt->tot[0], cap_next, st);
        fx_launch_expand_adflag(L, nad_max, b.pos, b.flag, st);
        fx_scan_i32_dev(b.flag, &cnt->nad[k], 4, 4 * nad_max, b.adpos, sh.partial, &cnt->tot[1], st);
        fx_launch_commit_ads(cnt, k, &cnt->tot[1], st);
        fx_launch_expand_adwrite(L, nad_max, b.pos, b.flag, b.adpos, b.ad[(k + 1) & 1], b.off[(k + 1) & 1], st);
        fx_launch_expand_write(L, e_max, b.mask, b.pos, b.adpos, leaf ? b.leafbc : b.ebc[(k + 1) & 1],
                               leaf ? nullptr : b.epar[(k + 1) & 1], st);
    }
    fx_launch_chunk_done(cnt, nl, b.cpart, sh.part, sh.run, st);
}

// The system as the class kernels see it (host-side description: every
// pointer is fixed once the call's block is laid out).
FxSys describe(const Sys& s, int ndens, bool screen) {
    const fx_tree* T = s.T;
    const SysBufs& b = s.b;
    const int lv = (int)T->levels.size() - 1;
    FxSys Y{};
    Y.basis = T->basis;
    for (int j = 0; j < FX_MAX_DENS; ++j) {
        Y.P[j] = s.P[j < ndens ? j : 0];
        Y.acc[j] = b.acc[j < ndens ? j : 0];
    }
    Y.n = T->n;
    Y.Pn = b.Pn;
    Y.bc_off = b.off[lv & 1];
    Y.bc = T->single_shell_leaves ? b.sorted : b.leafbc;
    Y.cls_off = T->single_shell_leaves ? b.cls_off : nullptr;
    Y.mask = screen ? b.screen : nullptr;
    Y.cnt = s.cnt;
    return Y;
}

// Units of the leaf items (and, for single-shell leaves, the entries grouped
// by density-side class).
void make_units(Sys& s, hipStream_t st, const Shared& sh) {
    const fx_tree* T = s.T;
    const Caps& c = s.caps;
    SysBufs& b = s.b;
    const int lv = (int)T->levels.size() - 1;
    const int2* items = b.ad[lv & 1];
    const long* item_off = b.off[lv & 1];
    fx_launch_unit_count(items, s.cnt, lv, c.items, T->basis.leaf_lofs, T->basis.leaf_lsh, b.ucnt, st);
    fx_scan_i32(b.ucnt, 9 * c.items, b.upos, sh.partial, sh.total, st);
    FxUnitCaps uc{};
    for (int k = 0; k < 9; ++k) uc.cap[k] = c.ucap[k];
    uc.total = c.units;
    fx_launch_unit_bounds(b.upos, c.items, s.cnt, sh.run, uc, st);
    fx_launch_units_done(s.cnt, sh.run, st);
    fx_launch_unit_write(items, s.cnt, lv, c.items, T->basis.leaf_lofs, T->basis.leaf_lsh, b.upos, b.units, st);
    if (T->single_shell_leaves)
        fx_launch_class_sort(item_off, b.leafbc, s.cnt, lv, c.items, T->basis.l, b.sorted, b.cls_off, st);
}

struct Timed {
    int idx;
    hipEvent_t a, b;
};

struct CallState {
    Opts op;
    double tau = 0;
    int ndens = 1;
    fx_stats* stats = nullptr;
    std::vector<Timed> timed;
    double tick_ns = 10.0;
    ~CallState() {
        for (auto& t : timed) {
            (void)hipEventDestroy(t.a);
            (void)hipEventDestroy(t.b);
        }
    }
};

// One launch per class and precision over the units of the given systems
// (several systems: their lists concatenated on the device).
// The descriptors of several systems must be in sh.dsys (uploaded by the caller).
void run_classes(CallState& cs, std::vector<Sys*>& sys, std::vector<FxSys>& ysys, const Shared& sh, hipStream_t st) {
    const int count = (int)sys.size();
    const bool multi = count > 1;
    int lmax = 0;
    for (auto* s : sys) lmax = std::max(lmax, s->T->lmax);
    const Opts& op = cs.op;
    const int nprec = op.o.precision == FX_PREC_MIXED ? 2 : 1;
    FxClassArgs args{};
    args.boys = sys[0]->T->boys;
    args.ndens = cs.ndens;
    args.tau = cs.tau;
    args.thr = op.o.fp32_threshold;
    args.tau_ovlp = op.o.tau_ovlp;
    args.block = op.o.leaf_screen == FX_LEAF_BLOCK ? 1 : 0;
    // statistics calls only, and not those that time every launch
    args.beta32 = cs.stats && !op.o.profile ? sh.beta32 : nullptr;
    const float* mean_np = sys[0]->T->mean_np;
    std::vector<float> hfeat, htime;
    for (int la = 0; la <= lmax; ++la)
        for (int ld = 0; ld <= lmax; ++ld) {
            const int k2 = la * 3 + ld;
            long bound = 0;
            for (auto* s : sys) bound += s->caps.ucap[k2];
            if (bound == 0) continue;
            args.nbound = bound;
            if (multi) {
                fx_launch_merge_bounds(sh.cnts, count, k2, sh.moff, sh.mb + 2 * k2, st);
                for (int i = 0; i < count; ++i)
                    if (sys[i]->caps.ucap[k2])
                        fx_launch_merge_copy(sys[i]->b.units, sys[i]->cnt, k2, sys[i]->caps.ucap[k2], sh.moff, i,
                                             sh.munits, sh.msys, st);
                args.units = sh.munits;
                args.ulh = sh.mb + 2 * k2;
                args.unit_sys = sh.msys;
                args.sys = sh.dsys;
            } else {
                args.units = sys[0]->b.units;
                args.ulh = &sys[0]->cnt->ubase[k2];
                args.unit_sys = nullptr;
                args.sys = nullptr;
                args.one = ysys[0];
                if (ysys[0].mask) {
                    // the group's nine class kernels read this screen
                    const Sys& s0 = *sys[0];
                    const int lv = (int)s0.T->levels.size() - 1;
                    fx_launch_screen_group(s0.b.ad[lv & 1], s0.b.off[lv & 1], s0.b.leafbc, s0.cnt, lv, s0.caps.items,
                                           s0.T->basis, s0.b.Pn, la, ld, cs.tau, op.o.fp32_threshold, op.o.tau_ovlp,
                                           s0.b.screen, st);
                }
            }
            for (int lb = 0; lb <= lmax; ++lb)
                for (int lc = 0; lc <= lmax; ++lc) {
                    const int cls = ((la * 3 + lb) * 3 + lc) * 3 + ld;
                    const float class_cost = std::log2((float)fx_class_vrr_flops[cls] * mean_np[lb] * mean_np[lc] +
                                                       (float)fx_class_hrr_flops[cls] + 1.f);
                    args.order = nullptr;
                    args.times = nullptr;
                    if (sh.feat) {
                        for (int i = 0; i < count; ++i) {
                            const Sys& s = *sys[i];
                            if (!s.caps.ucap[k2]) continue;
                            fx_launch_unit_features(s.b.units, &s.cnt->ubase[k2], s.caps.ucap[k2], ysys[i].bc_off,
                                                    ysys[i].cls_off, lb * 3 + lc, s.T->basis.nprim, s.T->qrow,
                                                    class_cost, sh.feat, multi ? sh.moff + i : nullptr, st);
                        }
                    }
                    if (op.sched) {
                        // predicted log2 cost per unit: the learned model, or the
                        // bound-only estimate log2(class flops * nprim_a nprim_d * entries)
                        if (op.mlp)
                            fx_launch_mlp_predict(op.o.costmodel->dW, op.o.costmodel->dnorm, sh.feat, args.ulh, bound,
                                                  sh.cost, st);
                        else
                            fx_launch_bound_cost(sh.feat, args.ulh, bound, sh.cost, st);
                        fx_launch_bin_order(sh.cost, args.ulh, bound, op.mlp ? 40.f : 48.f, 1.0f, kBins, sh.key,
                                            sh.bcount, sh.bpos, sh.partial, sh.total, sh.order, st, fx_scan_i32);
                        args.order = sh.order;
                    }
                    // mixed precision in one pass (variant 2 on the FP64 entry, one density)
                    const bool dual = nprec == 2 && cs.ndens == 1 && g_variant[cls][0] == 2;
                    for (int pr = 0; pr < (dual ? 1 : nprec); ++pr) {
                        if (g_recording) args.times = sh.times;
                        args.mode = dual ? FX_MODE_DUAL
                                         : op.o.precision == FX_PREC_MIXED ? (pr ? FX_MODE_MIXED_LO : FX_MODE_MIXED_HI)
                                                                           : FX_MODE_ALL;
                        args.counters = sh.counters + (cls * 2 + pr) * 3;
                        args.counters2 = dual ? sh.counters + (cls * 2 + 1) * 3 : nullptr;
                        args.flags = g_flags[cls][pr];
                        if (op.o.profile) {
                            Timed t{cls * 2 + pr, nullptr, nullptr};
                            FX_HIP(hipEventCreate(&t.a));
                            FX_HIP(hipEventCreate(&t.b));
                            FX_HIP(hipEventRecord(t.a, st));
                            fx_class_table[cls](pr, g_variant[cls][pr], args, st);
                            FX_HIP(hipEventRecord(t.b, st));
                            cs.timed.push_back(t);
                        } else {
                            fx_class_table[cls](pr, g_variant[cls][pr], args, st);
                        }
                        if (g_recording) {
                            long lh[2];
                            FX_HIP(hipMemcpyAsync(lh, args.ulh, sizeof(lh), hipMemcpyDeviceToHost, st));
                            FX_HIP(hipStreamSynchronize(st));
                            const long n = lh[1] - lh[0];
                            hfeat.resize(4 * std::max(1L, n));
                            htime.resize(std::max(1L, n));
                            if (n > 0) {
                                FX_HIP(hipMemcpyAsync(hfeat.data(), sh.feat, sizeof(float4) * n, hipMemcpyDeviceToHost,
                                                      st));
                                FX_HIP(hipMemcpyAsync(htime.data(), sh.times, sizeof(float) * n, hipMemcpyDeviceToHost,
                                                      st));
                                FX_HIP(hipStreamSynchronize(st));
                            }
                            for (long u = 0; u < n; ++u) {
                                for (int q = 0; q < 4; ++q) g_recording->feat.push_back(hfeat[4 * u + q]);
                                g_recording->log2ns.push_back(
                                    std::log2(std::max(1.0, (double)htime[u] * cs.tick_ns)));
                                g_recording->cls.push_back(cls * 2 + pr);
                            }
                        }
                    }
                }
        }
    FX_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// graph cache: one captured call per tree (keyed on every input that the
// captured kernels bake in), replayed while the key and the capacities hold
// ---------------------------------------------------------------------------
}  // namespace

struct FxGraphCache {
    std::vector<uint64_t> key;
    hipGraphExec_t exec = nullptr;
    void* block = nullptr;
    size_t bytes = 0;
    std::vector<Caps> caps;
    ~FxGraphCache() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (block) (void)hipFree(block);
    }
};

void fx_graph_cache_free(FxGraphCache* g) {
    if (g) {
        (void)hipDeviceSynchronize();
        delete g;
    }
}

namespace {

uint64_t bits(double x) {
    uint64_t u;
    std::memcpy(&u, &x, 8);
    return u;
}

std::vector<uint64_t> graph_key(const fx_tree* const* trees, const double* const* Ps, double* const* Ks, int count,
                                int ndens, double tau, const fx_exchange_opts& o, int nchunks) {
    std::vector<uint64_t> k;
    k.push_back((uint64_t)count);
    k.push_back((uint64_t)ndens);
    k.push_back((uint64_t)nchunks);
    k.push_back((uint64_t)g_group_screen);
    for (int i = 0; i < count; ++i) {
        k.push_back(trees[i]->id);
        for (int j = 0; j < ndens; ++j) {
            k.push_back((uint64_t)(uintptr_t)Ps[i * ndens + j]);
            k.push_back((uint64_t)(uintptr_t)Ks[i * ndens + j]);
        }
    }
    k.push_back(bits(tau));
    k.push_back((uint64_t)o.precision);
    k.push_back(bits(o.fp32_threshold));
    k.push_back((uint64_t)o.schedule);
    k.push_back((uint64_t)(uintptr_t)o.costmodel);
    k.push_back(bits(o.alpha));
    k.push_back(bits(o.beta));
    k.push_back((uint64_t)o.symmetry);
    k.push_back((uint64_t)o.leaf_screen);
    k.push_back(bits(o.tau_ovlp));
    for (int c = 0; c < 81; ++c)
        k.push_back((uint64_t)(g_variant[c][0] | g_variant[c][1] << 4 | g_flags[c][0] << 8 | g_flags[c][1] << 12));
    return k;
}

void validate_exchange(const fx_tree* T, const double* P, double tau, const double* K) {
    if (!T) fx_fail(FX_ERR_INVALID_ARG, "tree is NULL");
    if (!P || !K) fx_fail(FX_ERR_INVALID_ARG, "P and K must be device pointers");
    if (P == K) fx_fail(FX_ERR_INVALID_ARG, "P must not alias K");
    if (!(tau >= 0.0) || !std::isfinite(tau)) fx_fail(FX_ERR_INVALID_ARG, "tau must be finite and >= 0");
    if (((uintptr_t)P & 7) || ((uintptr_t)K & 7)) fx_fail(FX_ERR_INVALID_ARG, "P and K must be 8-byte aligned");
}

fx_exchange_opts checked_opts(const fx_exchange_opts* opts) {
    fx_exchange_opts o;
    fx_exchange_opts_init(&o);
    if (opts) o = *opts;
    if (o.precision != FX_PREC_FP64 && o.precision != FX_PREC_MIXED) fx_fail(FX_ERR_INVALID_ARG, "bad precision");
    if (o.schedule < 0 || o.schedule > 2) fx_fail(FX_ERR_INVALID_ARG, "bad schedule");
    if (!std::isfinite(o.alpha) || !std::isfinite(o.beta)) fx_fail(FX_ERR_INVALID_ARG, "alpha/beta not finite");
    if (o.precision == FX_PREC_MIXED && !(o.fp32_threshold >= 0.0)) fx_fail(FX_ERR_INVALID_ARG, "bad fp32_threshold");
    if (o.symmetry != FX_SYM_AUTO && o.symmetry != FX_SYM_OFF) fx_fail(FX_ERR_INVALID_ARG, "bad symmetry");
    if (o.leaf_screen != FX_LEAF_SHELL && o.leaf_screen != FX_LEAF_BLOCK) fx_fail(FX_ERR_INVALID_ARG, "bad leaf_screen");
    if (o.max_frontier_entries < 0) fx_fail(FX_ERR_INVALID_ARG, "max_frontier_entries must be >= 0");
    if (!(o.tau_ovlp >= 0.0) || !std::isfinite(o.tau_ovlp)) fx_fail(FX_ERR_INVALID_ARG, "tau_ovlp must be finite and >= 0");
    return o;
}

// Split [lo, hi) at the leaf boundary nearest its middle (-1: a single leaf).
int split_rows(const fx_tree* T, int lo, int hi) {
    const Level& leaf = T->levels.back();
    int best = -1;
    double bd = 1e300;
    const double mid = 0.5 * (lo + hi);
    for (size_t i = 0; i < leaf.sL.size(); ++i) {
        const int x = leaf.sL[i];
        if (x <= lo || x >= hi) continue;
        if (std::fabs(x - mid) < bd) {
            bd = std::fabs(x - mid);
            best = x;
        }
    }
    return best;
}

// Cuts of nleaf leaves into nchunks contiguous, non-empty ranges [cut[k],
// cut[k+1]): of about equal entries when `rows` (entries per leaf) is given
// and not all zero, else of about equal leaf counts.  Cut k is the first
// leaf boundary where the running sum reaches k/nchunks of the total, moved
// only as far as keeping every range non-empty needs.
std::vector<int> leaf_cuts(const long* rows, int nleaf, int nchunks) {
    nchunks = std::max(1, std::min(nchunks, nleaf));
    std::vector<int> cut(nchunks + 1, nleaf);
    cut[0] = 0;
    long total = 0;
    if (rows)
        for (int i = 0; i < nleaf; ++i) total += rows[i];
    if (total > 0) {
        long run = 0;
        int c = 1;
        for (int i = 0; i < nleaf && c < nchunks; ++i) {
            run += rows[i];
            while (c < nchunks && (double)run >= (double)total * c / nchunks) cut[c++] = i + 1;
        }
        for (int k = 1; k < nchunks; ++k) cut[k] = std::max(cut[k], cut[k - 1] + 1);
        for (int k = nchunks - 1; k >= 1; --k) cut[k] = std::min(cut[k], cut[k + 1] - 1);
    } else {
        for (int k = 1; k < nchunks; ++k) cut[k] = (int)((long)k * nleaf / nchunks);
    }
    return cut;
}

// nchunks K row ranges at leaf boundaries: of about equal leaf entries when
// the tree has counted them, else of about equal leaf counts
Ranges row_ranges(const fx_tree* T, int nchunks) {
    const Level& leaf = T->levels.back();
    const int nleaf = (int)leaf.sL.size();
    const std::vector<long>& rows = T->hint.leaf_rows;
    const std::vector<int> cut = leaf_cuts((int)rows.size() == nleaf ? rows.data() : nullptr, nleaf, nchunks);
    Ranges r;
    for (size_t k = 0; k + 1 < cut.size(); ++k)
        r.push_back({leaf.sL[cut[k]], cut[k + 1] < nleaf ? leaf.sL[cut[k + 1]] : T->S});
    return r;
}

// fold a finished call's sizes into the tree's hint (does not wait)
void absorb_usage(const fx_tree* T) {
    if (!T->usage_pending) return;
    if (hipEventQuery(T->usage_ev) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    const FxDevRun u = *T->usage;
    T->usage_pending = false;
    FxSizeHint& h = T->hint;
    // sizes per row range of that call, scaled to the whole traversal
    const long nc = std::max(1, T->usage_nchunks);
    if (T->usage_nchunks != h.units_chunks) {
        h.units_chunks = T->usage_nchunks;
        for (int k = 0; k < 9; ++k) h.units_max[k] = 0;
    }
    for (int k = 0; k < 9; ++k) h.units_max[k] = std::max(h.units_max[k], u.ucls[k]);
    if (T->usage_nchunks == h.range_chunks) {
        h.range_e_in = std::max({h.range_e_in, u.e_in, u.need_in});
        h.range_e_leaf = std::max({h.range_e_leaf, u.e_leaf, u.need_leaf, u.need_in});
    }
    h.e_in = std::max(h.e_in, u.e_in * nc);
    h.e_leaf = std::max(h.e_leaf, u.e_leaf * nc);
    // a level that overflowed asked for need entries (later levels are unknown: at least that)
    h.e_in = std::max(h.e_in, u.need_in * nc);
    h.e_leaf = std::max(h.e_leaf, std::max(u.need_leaf, u.need_in) * nc);
}

// Row ranges for sizes (whole-traversal totals): the fewest that keep every
// level within 32-bit positions with the margin.
int chunks_for(long e_in, long e_leaf) {
    const double need = 1.25 * (double)std::max(e_in, e_leaf);
    return std::max(1, (int)std::ceil(need / (double)kEntryMax));
}

size_t free_device_bytes() {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return fr;
}

void record_usage(std::vector<Sys>& sys, const Shared& sh, int nchunks, hipStream_t st) {
    for (auto& s : sys) {
        const fx_tree* T = s.T;
        if (T->usage_pending) continue;
        FX_HIP(hipMemcpyAsync(T->usage, sh.run, sizeof(FxDevRun), hipMemcpyDeviceToHost, st));
        FX_HIP(hipEventRecord(T->usage_ev, st));
        T->usage_pending = true;
        T->usage_nchunks = nchunks;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Exchange of one or several systems (each with ndens densities).
// Ps, Ks: count * ndens device pointers, system-major.  scratch /
// scratch_bytes: a caller-provided device block (then nothing is allocated),
// or null.
// ---------------------------------------------------------------------------
void fx_exchange_run(const fx_tree* const* trees, const double* const* Ps, double* const* Ks, int count, int ndens,
                     double tau, const fx_exchange_opts* opts, fx_stats* stats, hipStream_t st, void* scratch,
                     size_t scratch_bytes) {
    auto t0 = std::chrono::steady_clock::now();
    if (ndens < 1 || ndens > FX_MAX_DENS)
        fx_fail(FX_ERR_UNSUPPORTED, "ndens must be 1.." + std::to_string(FX_MAX_DENS));
    for (int i = 0; i < count; ++i)
        for (int j = 0; j < ndens; ++j) {
            validate_exchange(trees[i], Ps[i * ndens + j], tau, Ks[i * ndens + j]);
            for (int k = 0; k < ndens; ++k) {
                if (Ps[i * ndens + j] == Ks[i * ndens + k]) fx_fail(FX_ERR_INVALID_ARG, "a density aliases a K");
                if (k != j && Ks[i * ndens + j] == Ks[i * ndens + k]) fx_fail(FX_ERR_INVALID_ARG, "two K alias");
            }
        }
    CallState cs;
    cs.op.o = checked_opts(opts);
    const fx_exchange_opts& o = cs.op.o;
    cs.tau = tau;
    cs.ndens = ndens;
    cs.stats = stats;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (count == 0) return;
    const bool noalloc = scratch != nullptr;
    cs.op.wait = stats || o.profile || g_recording;
    cs.op.graph = o.use_graph && !o.profile && !g_recording && !noalloc;
    cs.op.mlp = o.schedule == FX_SCHED_MLP && o.costmodel;
    cs.op.sched = o.schedule != FX_SCHED_NONE;
    if (g_recording) {
        int dev = 0, khz = 0;
        FX_HIP(hipGetDevice(&dev));
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            cs.tick_ns = 1e6 / (double)khz;
    }
    // tree locks in address order (a batch may repeat a tree)
    std::vector<const fx_tree*> locked(trees, trees + count);
    std::sort(locked.begin(), locked.end());
    locked.erase(std::unique(locked.begin(), locked.end()), locked.end());
    std::vector<std::unique_lock<std::mutex>> locks;
    for (auto* T : locked) locks.emplace_back(T->mu);
    for (auto* T : locked) absorb_usage(T);

    const bool own_acc = o.beta != 0.0;
    const bool allow_sym = o.symmetry == FX_SYM_AUTO;
    std::vector<Sys> sys(count);
    for (int i = 0; i < count; ++i) {
        sys[i].T = trees[i];
        for (int j = 0; j < ndens; ++j) {
            sys[i].P[j] = Ps[i * ndens + j];
            sys[i].K[j] = Ks[i * ndens + j];
        }
        if (stats) stats->levels = std::max(stats->levels, (int)trees[i]->levels.size());
    }

    // ---- the device block of the call: measure, obtain, carve ----
    Shared sh;
    auto layout = [&](char* base) {
        Carve cv;
        cv.base = base;
        carve_shared(cv, sh, sys, cs.op);
        for (auto& s : sys) carve_sys(cv, s, ndens, own_acc);
        for (int i = 0; i < count; ++i) sys[i].cnt = sh.cnts + i;
        return cv.off;
    };
    void* block = nullptr;
    size_t block_bytes = 0;
    bool block_owned = false;
    auto release = [&]() {
        if (block_owned && block) fx_dfree(block, st);
        block = nullptr;
        block_owned = false;
    };
    auto acquire = [&]() {
        release();
        const size_t need = layout(nullptr);
        if (noalloc) {
            if (need > scratch_bytes)
                fx_fail(FX_ERR_OOM, "the call needs " + std::to_string(need) + " bytes of workspace, more than the " +
                                        std::to_string(scratch_bytes) + "-byte scratch array");
            block = scratch;
        } else {
            block = fx_dalloc(need, st);
            block_owned = true;
        }
        block_bytes = need;
        layout((char*)block);
    };
    struct Guard {
        std::function<void()> f;
        ~Guard() { f(); }
    } guard{release};

    // ---- capacities ----
    auto caps_from_hint = [&](Sys& s, int nch) {
        const FxSizeHint& h = s.T->hint;
        long ei, el;
        if (o.max_frontier_entries > 0) {
            ei = el = o.max_frontier_entries;
        } else if (nch > 1 && h.range_chunks == nch && h.range_e_in > 0) {
            // measured for these row ranges (a small margin for another density)
            ei = (long)(1.125 * (double)h.range_e_in) + 1024;
            el = (long)(1.125 * (double)h.range_e_leaf) + 1024;
        } else {
            // the whole traversal's sizes, shared by nch row ranges (which are not
            // equally large: a larger margin when split)
            const double m = nch > 1 ? 1.5 : 1.25;
            ei = (long)(m * (double)h.e_in / nch) + 1024;
            el = (long)(m * (double)h.e_leaf / nch) + 1024;
        }
        // (calls that wait keep the bounds from the tree: they split a row range
        // that overflows, which the unit lists could not undo)
        const bool seen = o.max_frontier_entries == 0 && !cs.op.wait && h.units_chunks == nch &&
                          *std::max_element(h.units_max, h.units_max + 9) > 0;
        s.caps = make_caps(s.T, ei, el, nch > 1 ? row_ranges(s.T, nch) : whole_rows(s.T), seen ? h.units_max : nullptr);
    };
    int nchunks = 1;
    if (noalloc && o.max_frontier_entries == 0) {
        // the largest capacities that fit in the scratch array
        long lo = 1, hi = kEntryMax;
        while (lo < hi) {
            const long mid = lo + (hi - lo + 1) / 2;
            for (auto& s : sys) s.caps = make_caps(s.T, mid, 4 * mid, whole_rows(s.T));
            if (layout(nullptr) <= scratch_bytes) lo = mid;
            else hi = mid - 1;
        }
        for (auto& s : sys) s.caps = make_caps(s.T, lo, 4 * lo, whole_rows(s.T));
        nchunks = 1;
    } else {
        bool learn = false;
        for (auto& s : sys) learn |= o.max_frontier_entries == 0 && s.T->hint.e_in == 0;
        if (learn && count == 1) {
            // first call on a tree: traverse only, growing the capacity of the
            // level that overflowed until every level fits, over K row ranges
            // when one pass would need more than 32-bit positions or more memory
            // than the device holds; the hint is then the sizes seen, summed over
            // the ranges, and the leaf entries per row
            Sys& s = sys[0];
            const fx_tree* T = s.T;
            FxSizeHint& h = T->hint;
            const int nl = (int)T->levels.size();
            const int lv = nl - 1;
            const int nleaf = (int)T->levels.back().sL.size();
            long want_in = 1L << 16, want_leaf = 1L << 18;
            int lc = 1;
            bool learned = false;
            for (int attempt = 0; attempt < 128 && !learned; ++attempt) {
                const Ranges rr = lc > 1 ? row_ranges(T, lc) : whole_rows(T);
                s.caps = make_caps(T, want_in, want_leaf, rr);
                const size_t avail = free_device_bytes();
                if (avail > 0 && layout(nullptr) > avail / 10 * 8 && lc < nleaf) {
                    lc = std::min(nleaf, 2 * lc);
                    want_in = std::max(1L << 16, want_in / 2);
                    want_leaf = std::max(1L << 18, want_leaf / 2);
                    continue;
                }
                acquire();
                fx_launch_fill_u64((unsigned long long*)sh.run, sizeof(FxDevRun) / 8, 0ull, st);
                fx_launch_fill_u64(sh.rows, nleaf, 0ull, st);
                density_norms(s, ndens, allow_sym, st);
                std::vector<FxDevCounts> hc(rr.size());
                for (size_t r = 0; r < rr.size(); ++r) {
                    s.a_lo = rr[r].first;
                    s.a_hi = rr[r].second;
                    traverse(s, tau, o.tau_ovlp, allow_sym, r == 0, st, sh);
                    fx_launch_leaf_rows(s.b.ad[lv & 1], s.b.off[lv & 1], s.cnt, lv, s.caps.items, sh.rows, st);
                    FX_HIP(hipMemcpyAsync(&hc[r], s.cnt, sizeof(FxDevCounts), hipMemcpyDeviceToHost, st));
                }
                std::vector<unsigned long long> rows(nleaf, 0ull);
                FX_HIP(hipMemcpyAsync(rows.data(), sh.rows, sizeof(unsigned long long) * nleaf, hipMemcpyDeviceToHost,
                                      st));
                FX_HIP(hipStreamSynchronize(st));
                release();
                bool again = false, split = false;
                for (const auto& c : hc) {
                    if (!c.overflow) continue;
                    if (c.need > kEntryMax) split = true;
                    else if (c.need_level == lv) want_leaf = std::max(want_leaf, c.need);
                    else want_in = std::max(want_in, c.need);
                    again = true;
                }
                if (split) {
                    // more entries than 32-bit positions index in one range
                    if (lc >= nleaf) fx_fail(FX_ERR_OOM, "one row of leaf blocks exceeds 2^32 traversal entries");
                    lc = std::min(nleaf, 2 * lc);
                    continue;
                }
                if (again) continue;
                long ein = 1, eleaf = 0;
                for (int k = 0; k < nl; ++k) {
                    long sum = 0;
                    for (const auto& c : hc) sum += c.ne[k];
                    if (k < lv) ein = std::max(ein, sum);
                    else eleaf = sum;
                }
                h.e_in = ein;
                h.e_leaf = std::max(1L, eleaf);
                h.leaf_rows.assign(rows.begin(), rows.end());
                learned = true;
            }
            if (!learned) fx_fail(FX_ERR_OOM, "the traversal did not fit the device in any split of K rows");
        } else if (learn) {
            // first call on a batch: each system's whole traversal, growing the
            // capacity of the level that overflowed until every level fits
            std::vector<long> want_in(count, 1L << 16), want_leaf(count, 1L << 18);
            for (int attempt = 0; attempt < 64; ++attempt) {
                for (int i = 0; i < count; ++i)
                    sys[i].caps = make_caps(sys[i].T, want_in[i], want_leaf[i], whole_rows(sys[i].T));
                acquire();
                fx_launch_fill_u64((unsigned long long*)sh.run, sizeof(FxDevRun) / 8, 0ull, st);
                for (auto& s : sys) {
                    density_norms(s, ndens, allow_sym, st);
                    s.a_lo = 0;
                    s.a_hi = s.T->S;
                    traverse(s, tau, o.tau_ovlp, allow_sym, true, st, sh);
                }
                std::vector<FxDevCounts> hc(count);
                FX_HIP(hipMemcpyAsync(hc.data(), sh.cnts, sizeof(FxDevCounts) * count, hipMemcpyDeviceToHost, st));
                FX_HIP(hipStreamSynchronize(st));
                release();
                bool again = false;
                for (int i = 0; i < count; ++i) {
                    FxSizeHint& h = sys[i].T->hint;
                    const int nl = (int)sys[i].T->levels.size();
                    long ein = 1;
                    for (int k = 0; k + 1 < nl; ++k) ein = std::max(ein, hc[i].ne[k]);
                    if (hc[i].overflow) {
                        const long need = hc[i].need;
                        if (need > kEntryMax) fx_fail(FX_ERR_OOM, "a batched system exceeds the frontier capacity");
                        if (hc[i].need_level == nl - 1) want_leaf[i] = std::max(want_leaf[i], need);
                        else want_in[i] = std::max(want_in[i], need);
                        again = true;
                        continue;
                    }
                    h.e_in = ein;
                    h.e_leaf = std::max(1L, hc[i].ne[nl - 1]);
                }
                if (!again) break;
            }
        }
        if (count == 1 && o.max_frontier_entries == 0)
            nchunks = chunks_for(sys[0].T->hint.e_in, sys[0].T->hint.e_leaf);
        for (auto& s : sys) caps_from_hint(s, nchunks);
        if (count == 1 && o.max_frontier_entries == 0) {
            // K row ranges one after another when one pass would need more than
            // the workspace budget (or than the device holds)
            const fx_tree* T = sys[0].T;
            FxSizeHint& h = T->hint;
            const int nleaf = (int)T->levels.back().sL.size();
            size_t budget = o.max_workspace_bytes > 0 ? (size_t)o.max_workspace_bytes
                            : o.max_workspace_bytes == 0 ? kDefaultWorkspace : SIZE_MAX;
            const size_t avail = free_device_bytes();
            if (avail > 0) budget = std::min(budget, avail / 10 * 8);
            auto bytes_at = [&](int nch) {
                caps_from_hint(sys[0], nch);
                return layout(nullptr);
            };
            // the fewest row ranges within `limit`: doubling, then bisection
            auto fewest = [&](int from, size_t limit) {
                if (bytes_at(from) <= limit || from >= nleaf) return from;
                int lo = from, hi = from;
                while (hi < nleaf) {
                    hi = (int)std::min<long>(nleaf, 2L * hi);
                    if (bytes_at(hi) <= limit) break;
                    lo = hi;
                }
                if (bytes_at(hi) > limit) return hi;
                while (hi - lo > 1) {
                    const int mid = lo + (hi - lo) / 2;
                    if (bytes_at(mid) <= limit) hi = mid;
                    else lo = mid;
                }
                return hi;
            };
            const bool planned = h.plan_chunks > 0 && h.plan_budget == budget && h.plan_e_in == h.e_in &&
                                 h.plan_e_leaf == h.e_leaf && h.plan_range_chunks == h.range_chunks &&
                                 h.plan_screen == g_group_screen;
            if (planned) {
                nchunks = h.plan_chunks;
            } else if (layout(nullptr) > budget) {
                // a budget below the part that does not shrink with more ranges
                // (densities' norms, accumulators) is met as closely as is useful
                const size_t floor_bytes = bytes_at(nleaf);
                size_t limit = std::max(budget, floor_bytes + floor_bytes / 4);
                if (o.max_workspace_bytes == 0 && nleaf > kDefaultMaxRanges) {
                    // the default budget gives way to launch size: more ranges than this
                    // leave class launches too small to fill the device, so large systems
                    // take what 64 ranges need while 80% of the free memory holds it
                    const size_t at_max = bytes_at(kDefaultMaxRanges);
                    const size_t cap = avail > 0 ? avail / 10 * 8 : SIZE_MAX;
                    if (at_max > limit) limit = std::min(at_max, std::max(limit, cap));
                }
                nchunks = fewest(nchunks, limit);
                // the entries of each of these ranges, measured once (traversal only)
                for (int round = 0; round < 3 && nchunks > 1 && h.range_chunks != nchunks; ++round) {
                    const Ranges rr = row_ranges(T, nchunks);
                    caps_from_hint(sys[0], nchunks);
                    long ei = sys[0].caps.e_in, el = sys[0].caps.e_leaf;
                    bool measured = false;
                    for (int attempt = 0; attempt < 32 && !measured; ++attempt) {
                        sys[0].caps = make_caps(T, ei, el, rr);
                        acquire();
                        fx_launch_fill_u64((unsigned long long*)sh.run, sizeof(FxDevRun) / 8, 0ull, st);
                        density_norms(sys[0], ndens, allow_sym, st);
                        for (const auto& r : rr) {
                            sys[0].a_lo = r.first;
                            sys[0].a_hi = r.second;
                            traverse(sys[0], tau, o.tau_ovlp, allow_sym, r.first == 0, st, sh);
                        }
                        FxDevRun run;
                        FX_HIP(hipMemcpyAsync(&run, sh.run, sizeof(run), hipMemcpyDeviceToHost, st));
                        FX_HIP(hipStreamSynchronize(st));
                        release();
                        if (!run.overflow) {
                            h.range_chunks = nchunks;
                            h.range_e_in = std::max(1L, run.e_in);
                            h.range_e_leaf = std::max(1L, run.e_leaf);
                            measured = true;
                        } else if (run.need_in > kEntryMax || run.need_leaf > kEntryMax) {
                            break;
                        } else {
                            ei = std::max(ei, run.need_in + run.need_in / 8);
                            el = std::max(el, run.need_leaf + run.need_leaf / 8);
                        }
                    }
                    if (!measured) break;
                    // uneven ranges can need more than the estimate: more of them
                    if (bytes_at(nchunks) > limit && nchunks < nleaf) nchunks = fewest(nchunks + 1, limit);
                }
            }
            if (!planned) {
                h.plan_chunks = nchunks;
                h.plan_budget = budget;
                h.plan_e_in = h.e_in;
                h.plan_e_leaf = h.e_leaf;
                h.plan_range_chunks = h.range_chunks;
                h.plan_screen = g_group_screen;
            }
            caps_from_hint(sys[0], nchunks);
        }
    }

    // ---- the work: enqueued on `ls`; `check` = read each chunk's overflow
    // flag and split its K row range (only when the call waits) ----
    double seconds_eri = 0;
    int runs = 0;
    auto enqueue_all = [&](hipStream_t ls, bool check, bool report) {
        fx_launch_fill_u64(sh.counters, 81 * 2 * 3 + 3 * FX_PART_SLOTS, 0ull, ls);
        fx_launch_fill_u64((unsigned long long*)sh.beta32, 1, 0ull, ls);
        fx_launch_fill_u64((unsigned long long*)sh.run, sizeof(FxDevRun) / 8, 0ull, ls);
        for (auto& s : sys) {
            for (int j = 0; j < ndens; ++j) {
                if (!own_acc) s.b.acc[j] = s.K[j];
                fx_launch_fill(s.b.acc[j], (long)s.T->n * s.T->n, 0.0, ls);
            }
            density_norms(s, ndens, allow_sym, ls);
        }
        std::vector<FxSys> ysys(count);
        // one shared screen per (l_a, l_d) group: one system, shell-level screening
        const bool screen = g_group_screen && count == 1 && o.leaf_screen == FX_LEAF_SHELL && group_screen(sys[0].T);
        for (int i = 0; i < count; ++i) ysys[i] = describe(sys[i], ndens, screen);
        runs = 0;
        if (count > 1) {
            for (int i = 0; i < count; ++i) {
                sys[i].a_lo = 0;
                sys[i].a_hi = sys[i].T->S;
                traverse(sys[i], tau, o.tau_ovlp, allow_sym, true, ls, sh);
                make_units(sys[i], ls, sh);
            }
            if (check) {
                std::vector<FxDevCounts> hc(count);
                FX_HIP(hipMemcpyAsync(hc.data(), sh.cnts, sizeof(FxDevCounts) * count, hipMemcpyDeviceToHost, ls));
                FX_HIP(hipStreamSynchronize(ls));
                for (int i = 0; i < count; ++i)
                    if (hc[i].overflow)
                        fx_fail(FX_ERR_OOM, "batched call: system " + std::to_string(i) +
                                                " exceeded its frontier capacity; set max_frontier_entries");
            }
            std::vector<Sys*> ps;
            for (auto& s : sys) ps.push_back(&s);
            auto te = std::chrono::steady_clock::now();
            run_classes(cs, ps, ysys, sh, ls);
            seconds_eri += std::chrono::duration<double>(std::chrono::steady_clock::now() - te).count();
            runs = 1;
        } else {
            Sys& s = sys[0];
            std::vector<std::pair<int, int>> todo = row_ranges(s.T, nchunks);
            std::reverse(todo.begin(), todo.end());
            while (!todo.empty()) {
                const auto r = todo.back();
                todo.pop_back();
                s.a_lo = r.first;
                s.a_hi = r.second;
                traverse(s, tau, o.tau_ovlp, allow_sym, r.first == 0, ls, sh);
                if (check) {
                    int ovf = 0;
                    FX_HIP(hipMemcpyAsync(&ovf, &s.cnt->overflow, sizeof(int), hipMemcpyDeviceToHost, ls));
                    FX_HIP(hipStreamSynchronize(ls));
                    if (ovf) {
                        // this row range does not fit: split it (its sums were not kept)
                        const int m = split_rows(s.T, r.first, r.second);
                        if (m < 0) fx_fail(FX_ERR_OOM, "one K row block exceeds the frontier capacity");
                        todo.push_back({m, r.second});
                        todo.push_back({r.first, m});
                        continue;
                    }
                }
                make_units(s, ls, sh);
                std::vector<Sys*> ps{&s};
                auto te = std::chrono::steady_clock::now();
                run_classes(cs, ps, ysys, sh, ls);
                seconds_eri += std::chrono::duration<double>(std::chrono::steady_clock::now() - te).count();
                ++runs;
                if (report && g_progress) {
                    // reported from a runtime thread when the device reaches this point
                    auto* m = new ProgressMsg{g_progress, g_progress_ctx, runs, runs + (int32_t)todo.size()};
                    if (hipLaunchHostFunc(ls, progress_trampoline, m) != hipSuccess) {
                        (void)hipGetLastError();
                        delete m;
                    }
                }
            }
        }
        // a call that waits has run every overflowed row range again
        if (check) fx_launch_fill_i32(&sh.run->incomplete, 1, 0, ls);
        // K = alpha * acc + beta * K (NaN if a chunk overflowed and was not run again)
        for (auto& s : sys) {
            const long nn = (long)s.T->n * s.T->n;
            for (int j = 0; j < ndens; ++j)
                fx_launch_finalize(s.b.acc[j], nn, o.alpha, o.beta, s.K[j], &sh.run->incomplete, ls);
        }
        FX_HIP(hipGetLastError());
    };

    // descriptors of a batch's systems, uploaded before the work is enqueued
    // (or captured): they depend only on the block layout
    auto upload_descriptors = [&]() {
        if (count < 2) return;
        std::vector<FxSys> ys(count);
        for (int i = 0; i < count; ++i) {
            if (!own_acc)
                for (int j = 0; j < ndens; ++j) sys[i].b.acc[j] = sys[i].K[j];
            ys[i] = describe(sys[i], ndens, false);
        }
        FX_HIP(hipMemcpyAsync(sh.dsys, ys.data(), sizeof(FxSys) * count, hipMemcpyHostToDevice, st));
        FX_HIP(hipStreamSynchronize(st));
    };
    // accumulators must be set before the descriptors are built
    for (auto& s : sys)
        if (!own_acc)
            for (int j = 0; j < ndens; ++j) s.b.acc[j] = s.K[j];

    bool done = false;
    if (cs.op.graph) {
        // ---- graph: replay the cached capture, or capture and cache ----
        const std::vector<uint64_t> key = graph_key(trees, Ps, Ks, count, ndens, tau, o, nchunks);
        FxGraphCache* gc = trees[0]->gcache;
        bool hit = gc && gc->key == key && gc->caps.size() == sys.size();
        if (hit)
            for (int i = 0; i < count; ++i)
                hit &= gc->caps[i].e_in >= sys[i].caps.e_in && gc->caps[i].e_leaf >= sys[i].caps.e_leaf &&
                       std::equal(gc->caps[i].ucap, gc->caps[i].ucap + 9, sys[i].caps.ucap);
        if (hit) {
            for (int i = 0; i < count; ++i) sys[i].caps = gc->caps[i];
        } else {
            if (gc) {
                fx_graph_cache_free(gc);
                trees[0]->gcache = nullptr;
            }
            gc = new FxGraphCache();
            std::unique_ptr<FxGraphCache> own(gc);
            gc->bytes = layout(nullptr);
            if (hipMalloc(&gc->block, gc->bytes) != hipSuccess) {
                (void)hipGetLastError();
                gc->block = nullptr;
                fx_fail(FX_ERR_OOM, "graph workspace allocation failed");
            }
            layout((char*)gc->block);
            upload_descriptors();
            hipStream_t cap = nullptr;
            FX_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            hipGraph_t graph = nullptr;
            FX_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
            try {
                enqueue_all(cap, false, false);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(cap, &g);
                if (g) (void)hipGraphDestroy(g);
                (void)hipStreamDestroy(cap);
                throw;
            }
            hipError_t e = hipStreamEndCapture(cap, &graph);
            (void)hipStreamDestroy(cap);
            if (e != hipSuccess) fx_fail(FX_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&gc->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) fx_fail(FX_ERR_HIP, std::string("graph instantiation: ") + hipGetErrorString(e));
            gc->key = key;
            for (auto& s : sys) gc->caps.push_back(s.caps);
            trees[0]->gcache = own.release();
        }
        layout((char*)gc->block);
        block_bytes = gc->bytes;
        runs = nchunks;
        FX_HIP(hipGraphLaunch(gc->exec, st));
        record_usage(sys, sh, nchunks, st);
        if (stats) stats->graph_nodes = 1;
        done = true;
        if (cs.op.wait) {
            int ovf = 0;
            FX_HIP(hipMemcpyAsync(&ovf, &sh.run->overflow, sizeof(int), hipMemcpyDeviceToHost, st));
            FX_HIP(hipStreamSynchronize(st));
            if (ovf) {
                // sizes grew past the captured capacities: this call runs eagerly (and
                // splits row ranges as needed); the next capture uses the new sizes
                for (auto* T : locked) {
                    T->usage_pending = true;
                    absorb_usage(T);
                }
                for (auto& s : sys) caps_from_hint(s, nchunks);
                done = false;
                if (stats) stats->graph_nodes = 0;
            }
        }
    }
    if (!done) {
        acquire();
        upload_descriptors();
        enqueue_all(st, cs.op.wait, true);
        record_usage(sys, sh, nchunks, st);
    }
    if (!cs.op.wait) return;

    // ---- statistics (the call waits for its result) ----
    std::vector<unsigned long long> cnt(81 * 2 * 3 + 3 * FX_PART_SLOTS);
    FX_HIP(hipMemcpyAsync(cnt.data(), sh.counters, sizeof(unsigned long long) * cnt.size(), hipMemcpyDeviceToHost, st));
    std::vector<FxDevCounts> hc(count);
    FX_HIP(hipMemcpyAsync(hc.data(), sh.cnts, sizeof(FxDevCounts) * count, hipMemcpyDeviceToHost, st));
    FxDevRun run;
    FX_HIP(hipMemcpyAsync(&run, sh.run, sizeof(run), hipMemcpyDeviceToHost, st));
    double beta32 = 0.0;
    FX_HIP(hipMemcpyAsync(&beta32, sh.beta32, sizeof(double), hipMemcpyDeviceToHost, st));
    FX_HIP(hipStreamSynchronize(st));
    if (!stats) return;
    stats->fp32_beta_sum = beta32;
    for (int k = 0; k < FX_STATS_MAX_LEVELS && k < FX_MAX_LEVELS; ++k) stats->frontier[k] = run.frontier[k];
    stats->leaf_items = run.items;
    stats->units = run.units;
    stats->overflow = run.overflow;
    stats->chunks = std::max(0, runs - 1);
    for (int i = 0; i < count; ++i) stats->symmetric_systems += hc[i].sym;
    for (int q = 0; q < 3; ++q) {
        unsigned long long v = 0;
        for (int k = 0; k < FX_PART_SLOTS; ++k) v += cnt[81 * 2 * 3 + q * FX_PART_SLOTS + k];
        stats->partition[q] = (int64_t)v;
    }
    for (int c = 0; c < 81; ++c)
        for (int pr = 0; pr < 2; ++pr) {
            const unsigned long long q = cnt[(c * 2 + pr) * 3], pq = cnt[(c * 2 + pr) * 3 + 1];
            const unsigned long long qm = cnt[(c * 2 + pr) * 3 + 2];
            stats->class_quartets[c] += (int64_t)q;
            stats->quartets += (int64_t)q;
            stats->quartets_covered += (int64_t)(q + qm);
            if (pr) stats->quartets_fp32 += (int64_t)q;
            stats->prim_quartets += (double)pq;
            const double fl = (double)pq * fx_class_vrr_flops[c] + (double)q * fx_class_hrr_flops[c];
            stats->flops += fl;
            stats->class_flops[c * 2 + pr] = fl;
            stats->class_prec_quartets[c * 2 + pr] = (int64_t)q;
        }
    for (auto& t : cs.timed) {
        float ms = 0.f;
        FX_HIP(hipEventElapsedTime(&ms, t.a, t.b));
        stats->class_seconds[t.idx] += 1e-3 * ms;
        stats->class_launches[t.idx] += 1;
    }
    stats->workspace_bytes = (int64_t)block_bytes;
    stats->seconds_eri = seconds_eri;
    stats->seconds_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats->seconds_traversal = stats->seconds_total - seconds_eri;
}

// ---------------------------------------------------------------------------
// C ABI: exchange entry points
// ---------------------------------------------------------------------------
extern "C" {

fx_status fx_plan_row_cuts(const int64_t* leaf_entries, int32_t nleaf, int32_t nchunks, int32_t* cuts) {
    return fx_guard([&] {
        if (nleaf < 1 || nchunks < 1 || !cuts) fx_fail(FX_ERR_INVALID_ARG, "need nleaf >= 1, nchunks >= 1, cuts");
        std::vector<long> rows;
        if (leaf_entries) {
            rows.assign(leaf_entries, leaf_entries + nleaf);
            for (long x : rows)
                if (x < 0) fx_fail(FX_ERR_INVALID_ARG, "negative entry count");
        }
        const std::vector<int> cut = leaf_cuts(leaf_entries ? rows.data() : nullptr, nleaf, nchunks);
        for (int k = 0; k <= nchunks; ++k) cuts[k] = k < (int)cut.size() ? cut[k] : nleaf;
    });
}

fx_status fx_set_group_screen(int32_t enabled) {
    return fx_guard([&] { g_group_screen = enabled ? 1 : 0; });
}

int32_t fx_get_group_screen(void) { return g_group_screen; }

fx_status fx_set_progress(fx_progress_fn fn, void* ctx) {
    return fx_guard([&] {
        g_progress = fn;
        g_progress_ctx = ctx;
    });
}

void fx_progress_stderr(int32_t done, int32_t total, void* ctx) {
    std::fprintf(stderr, "%s: K row range %d of %d done\n", ctx ? (const char*)ctx : "fx", done, total);
    std::fflush(stderr);
}

void fx_exchange_opts_init(fx_exchange_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = FX_PREC_FP64;
    o->fp32_threshold = 1e-5;
    o->schedule = FX_SCHED_BOUND;
    o->costmodel = nullptr;
    o->alpha = 1.0;
    o->beta = 0.0;
    o->max_frontier_entries = 0;
    o->profile = 0;
    o->use_graph = 0;
    o->symmetry = FX_SYM_AUTO;
    o->leaf_screen = FX_LEAF_SHELL;
    o->tau_ovlp = 0.0;
    o->max_workspace_bytes = 0;
}

fx_status fx_exchange_ex(const fx_tree* tree, const double* P, double tau, double* K, const fx_exchange_opts* opts,
                         fx_stats* stats, void* stream) {
    return fx_guard([&] { fx_exchange_run(&tree, &P, &K, 1, 1, tau, opts, stats, (hipStream_t)stream, nullptr, 0); });
}

fx_status fx_exchange(const fx_tree* tree, const double* P, double tau, double* K, void* stream) {
    return fx_exchange_ex(tree, P, tau, K, nullptr, nullptr, stream);
}

fx_status fx_exchange_batched(const fx_tree* const* trees, const double* const* P, double* const* K, int32_t count,
                              double tau, const fx_exchange_opts* opts, fx_stats* stats, void* stream) {
    return fx_guard([&] {
        if (count < 0 || (count > 0 && (!trees || !P || !K))) fx_fail(FX_ERR_INVALID_ARG, "bad batch arrays");
        fx_exchange_run(trees, P, K, count, 1, tau, opts, stats, (hipStream_t)stream, nullptr, 0);
    });
}

fx_status fx_exchange_multi(const fx_tree* tree, const double* const* P, double* const* K, int32_t ndens, double tau,
                            const fx_exchange_opts* opts, fx_stats* stats, void* stream) {
    return fx_guard([&] {
        if (!P || !K) fx_fail(FX_ERR_INVALID_ARG, "P and K must be arrays of ndens device pointers");
        fx_exchange_run(&tree, P, K, 1, ndens, tau, opts, stats, (hipStream_t)stream, nullptr, 0);
    });
}

fx_status fx_record_task_timings(const fx_tree* tree, const double* P, double tau, const fx_exchange_opts* opts,
                                 fx_task_timings** out, void* stream) {
    return fx_guard([&] {
        if (!out) fx_fail(FX_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (!tree) fx_fail(FX_ERR_INVALID_ARG, "tree is NULL");
        hipStream_t st = (hipStream_t)stream;
        DevArena A(st);
        double* K = A.get<double>((size_t)tree->n * tree->n);
        fx_task_timings* rec = new fx_task_timings();
        g_recording = rec;
        try {
            fx_exchange_run(&tree, &P, &K, 1, 1, tau, opts, nullptr, st, nullptr, 0);
        } catch (...) {
            g_recording = nullptr;
            delete rec;
            throw;
        }
        g_recording = nullptr;
        *out = rec;
    });
}

}  // extern "C"
