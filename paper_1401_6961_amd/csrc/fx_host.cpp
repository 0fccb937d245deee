// Host planner and C ABI of the exchange library.
//
//  * tree build: normalisation of contracted shells, shell ordering along a
//    3D Hilbert curve (Section III), ragged bisection at shell boundaries
//    (Eq. 1), Schwarz factors of every shell pair and squared Frobenius
//    norms of the shell-pair quadtree at every level (Eq. 2, Eq. 8);
//  * exchange: density norms, the level-synchronous hextree traversal of
//    Eqs. (7a-d) with the metric query of Eq. (8) (chunked when a level
//    would exceed the frontier budget), K-block work units, one launch per
//    angular-momentum class and precision, deterministic final reduction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/fx.h"
#include "fx_host.h"
#include "eri_flops.h"
#include "eri_table.h"
#include "fx_costmodel.h"
#include "fx_internal.h"
#include "fx_kernels.h"

// ---------------------------------------------------------------------------
// process-wide state declared in fx_host.h
// ---------------------------------------------------------------------------
thread_local std::string g_last_error;
fx_alloc_fn g_alloc = nullptr;
fx_free_fn g_free = nullptr;
void* g_alloc_ctx = nullptr;
thread_local fx_task_timings* g_recording = nullptr;

// ---------------------------------------------------------------------------
// Boys table F_j(T_i), T_i = i/32: the convergent series
// F_j(T) = e^{-T} sum_k (2T)^k / ((2j+1)(2j+3)...(2j+2k+1)) in long double.
// ---------------------------------------------------------------------------
static std::vector<double> boys_table() {
    std::vector<double> tab((size_t)FX_BOYS_NROW * FX_BOYS_NCOL);
    for (int i = 0; i < FX_BOYS_NROW; ++i) {
        const long double T = (long double)i * (long double)FX_BOYS_DT;
        const long double eT = expl(-T);
        for (int j = 0; j < FX_BOYS_NF; ++j) {
            long double term = 1.0L / (2 * j + 1), sum = term;
            for (int k = 1; k < 4000; ++k) {
                term *= 2.0L * T / (long double)(2 * j + 2 * k + 1);
                sum += term;
                if (term < 1e-22L * sum) break;
            }
            tab[(size_t)i * FX_BOYS_NCOL + j] = (double)(eT * sum);
        }
        tab[(size_t)i * FX_BOYS_NCOL + FX_BOYS_NCOL - 1] = (double)eT;
    }
    return tab;
}

// ---------------------------------------------------------------------------
// 3D Hilbert curve: index of an integer point on a 2^bits grid (Skilling's
// transposed-axes construction: undo excess work, Gray-encode, then
// interleave the bits most significant first).
// ---------------------------------------------------------------------------
extern "C" uint64_t fx_hilbert_key3(uint32_t x, uint32_t y, uint32_t z, int32_t bits) {
    uint32_t X[3] = {x, y, z};
    const uint32_t top = 1u << (bits - 1);
    for (uint32_t q = top; q > 1; q >>= 1) {
        const uint32_t p = q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & q) {
                X[0] ^= p;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & p;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t q = top; q > 1; q >>= 1)
        if (X[2] & q) t ^= q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    uint64_t key = 0;
    for (int b = bits - 1; b >= 0; --b)
        for (int i = 0; i < 3; ++i) key = (key << 1) | ((X[i] >> b) & 1u);
    return key;
}

static void validate_shells(const fx_shells* s) {
    if (!s) fx_fail(FX_ERR_INVALID_ARG, "shells is NULL");
    if (s->nshell <= 0) fx_fail(FX_ERR_INVALID_ARG, "nshell must be positive");
    if (!s->l || !s->nprim || !s->center || !s->exps || !s->coefs)
        fx_fail(FX_ERR_INVALID_ARG, "a shell array pointer is NULL");
    long nf = 0, npt = 0;
    for (int i = 0; i < s->nshell; ++i) {
        if (s->l[i] < 0 || s->l[i] > FX_MAX_L) fx_fail(FX_ERR_UNSUPPORTED, "shell " + std::to_string(i) + ": l outside 0..2");
        if (s->nprim[i] < 1 || s->nprim[i] > FX_MAX_PRIM)
            fx_fail(FX_ERR_UNSUPPORTED, "shell " + std::to_string(i) + ": primitive count outside 1..16");
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(s->center[3 * i + k])) fx_fail(FX_ERR_INVALID_ARG, "non-finite shell centre");
        nf += ncart(s->l[i]);
        npt += s->nprim[i];
    }
    for (long p = 0; p < npt; ++p)
        if (!(s->exps[p] > 0.0) || !std::isfinite(s->exps[p]) || !std::isfinite(s->coefs[p]))
            fx_fail(FX_ERR_INVALID_ARG, "exponents must be positive and weights finite");
    if (nf > (1L << 30)) fx_fail(FX_ERR_UNSUPPORTED, "too many basis functions");
}

static Plan make_plan(const fx_shells* s, const fx_tree_opts* opts) {
    const int S = s->nshell;
    const int leaf_max = (opts && opts->leaf_max_functions > 0) ? opts->leaf_max_functions : 10;
    const int ordering = opts ? opts->ordering : 0;
    if (opts && (opts->ordering < 0 || opts->ordering > 1)) fx_fail(FX_ERR_INVALID_ARG, "ordering must be 0 or 1");
    Plan P;
    P.order.resize(S);
    std::iota(P.order.begin(), P.order.end(), 0);
    if (ordering == 0 && S > 1) {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int i = 0; i < S; ++i)
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], s->center[3 * i + k]);
                hi[k] = std::max(hi[k], s->center[3 * i + k]);
            }
        double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-30});
        const int bits = 21;
        const double scale = (double)((1u << bits) - 1) / ext;
        std::vector<uint64_t> key(S);
        for (int i = 0; i < S; ++i) {
            uint32_t q[3];
            for (int k = 0; k < 3; ++k) q[k] = (uint32_t)std::llround((s->center[3 * i + k] - lo[k]) * scale);
            key[i] = fx_hilbert_key3(q[0], q[1], q[2], bits);
        }
        std::stable_sort(P.order.begin(), P.order.end(), [&](int a, int b) { return key[a] < key[b]; });
    }
    // function prefix in tree order
    std::vector<long> fp(S + 1, 0);
    for (int i = 0; i < S; ++i) fp[i + 1] = fp[i] + ncart(s->l[P.order[i]]);
    // breadth-first ragged bisection; leaves are carried to the deepest level
    std::vector<std::pair<int, int>> cur{{0, S}};
    while (true) {
        Level L;
        std::vector<std::pair<int, int>> next;
        bool any_split = false;
        for (auto [lo, hi] : cur) {
            L.sL.push_back(lo);
            L.sR.push_back(hi);
            L.ch0.push_back((int)next.size());
            const long nf = fp[hi] - fp[lo];
            if (nf <= leaf_max || hi - lo == 1) {
                next.push_back({lo, hi});
                L.nch.push_back(1);
            } else {
                // split at the shell boundary closest to the function midpoint (ties: lower)
                const double mid = 0.5 * (double)(fp[lo] + fp[hi]);
                int best = lo + 1;
                double bd = 1e300;
                for (int m = lo + 1; m < hi; ++m) {
                    const double d = std::fabs((double)fp[m] - mid);
                    if (d < bd) {
                        bd = d;
                        best = m;
                    }
                }
                next.push_back({lo, best});
                next.push_back({best, hi});
                L.nch.push_back(2);
                any_split = true;
            }
        }
        P.levels.push_back(std::move(L));
        if (!any_split) break;
        cur.swap(next);
        if (P.levels.size() >= FX_STATS_MAX_LEVELS - 1) fx_fail(FX_ERR_INTERNAL, "tree too deep");
    }
    // the last level: every node is a leaf (nch = 1 pointing to itself, unused)
    return P;
}

static std::atomic<uint64_t> g_tree_ids{1};

static void build_tree(const fx_shells* s, const fx_tree_opts* opts, hipStream_t st, fx_tree* T) {
    validate_shells(s);
    T->id = g_tree_ids.fetch_add(1);
    if (hipHostMalloc((void**)&T->usage, sizeof(FxDevRun), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        T->usage = nullptr;
        fx_fail(FX_ERR_OOM, "pinned host allocation failed");
    }
    std::memset(T->usage, 0, sizeof(FxDevRun));
    FX_HIP(hipEventCreateWithFlags(&T->usage_ev, hipEventDisableTiming));
    Plan P = make_plan(s, opts);
    const int S = s->nshell;
    T->S = S;
    T->order = P.order;
    T->levels = P.levels;
    // caller-order offsets
    std::vector<long> cpofs(S + 1, 0), cf0(S + 1, 0);
    for (int i = 0; i < S; ++i) {
        cpofs[i + 1] = cpofs[i] + s->nprim[i];
        cf0[i + 1] = cf0[i] + ncart(s->l[i]);
    }
    T->n = (int)cf0[S];
    // tree-order shell data with normalised radial weights:
    //   c_p = d_p N_p / sqrt(sum_pq d_p d_q N_p N_q (2l-1)!! / (2 g)^l (pi/g)^{3/2}),
    //   N_p = (2a/pi)^{3/4} (4a)^{l/2} / sqrt((2l-1)!!)   (component x^l)
    std::vector<int> l(S), np(S), pofs(S), f0(S);
    std::vector<double> xyz(3 * S), ex, co;
    for (int t = 0; t < S; ++t) {
        const int i = P.order[t];
        l[t] = s->l[i];
        np[t] = s->nprim[i];
        pofs[t] = (int)ex.size();
        f0[t] = (int)cf0[i];
        for (int k = 0; k < 3; ++k) xyz[3 * t + k] = s->center[3 * i + k];
        const int L = l[t];
        double df = 1.0;
        for (int k = 2 * L - 1; k > 1; k -= 2) df *= k;
        std::vector<double> N(np[t]);
        for (int p = 0; p < np[t]; ++p) {
            const double a = s->exps[cpofs[i] + p];
            N[p] = std::pow(2.0 * a / M_PI, 0.75) * std::pow(4.0 * a, 0.5 * L) / std::sqrt(df);
        }
        double ovl = 0.0;
        for (int p = 0; p < np[t]; ++p)
            for (int q = 0; q < np[t]; ++q) {
                const double g = s->exps[cpofs[i] + p] + s->exps[cpofs[i] + q];
                ovl += s->coefs[cpofs[i] + p] * s->coefs[cpofs[i] + q] * N[p] * N[q] * df / std::pow(2.0 * g, L) *
                       std::pow(M_PI / g, 1.5);
            }
        if (!(ovl > 0.0)) fx_fail(FX_ERR_INVALID_ARG, "shell " + std::to_string(i) + " has zero norm");
        for (int p = 0; p < np[t]; ++p) {
            ex.push_back(s->exps[cpofs[i] + p]);
            co.push_back(s->coefs[cpofs[i] + p] * N[p] / std::sqrt(ovl));
        }
        T->lmax = std::max(T->lmax, L);
    }
    T->l = l;
    T->nprim = np;
    T->f0 = f0;
    // leaf shell lists per l
    const Level& leaf = P.levels.back();
    const int nleaf = (int)leaf.sL.size();
    std::vector<int> lofs(nleaf * 4), lsh;
    for (int A = 0; A < nleaf; ++A) {
        for (int L = 0; L < 3; ++L) {
            lofs[A * 4 + L] = (int)lsh.size();
            for (int t = leaf.sL[A]; t < leaf.sR[A]; ++t)
                if (l[t] == L) lsh.push_back(t);
        }
        lofs[A * 4 + 3] = (int)lsh.size();
    }
    T->leaf_lofs = lofs;
    T->single_shell_leaves = (int)leaf.sL.size() == S;
    // at most one shell per leaf and l (e.g. one atom of an s+p+d basis per
    // leaf): the class kernels map a leaf straight to its shell
    std::vector<int> one(nleaf * 3, -1);
    bool one_per_l = true;
    for (int A = 0; A < nleaf && one_per_l; ++A)
        for (int L = 0; L < 3; ++L) {
            const int k = lofs[A * 4 + L + 1] - lofs[A * 4 + L];
            if (k > 1) one_per_l = false;
            else if (k == 1) one[A * 3 + L] = lsh[lofs[A * 4 + L]];
        }

    T->arena = new DevArena(st, true);
    DevArena& A = *T->arena;
    FxDevBasis& B = T->basis;
    B.nshell = S;
    B.nbf = T->n;
    B.l = upload(A, l);
    B.nprim = upload(A, np);
    B.pofs = upload(A, pofs);
    B.f0 = upload(A, f0);
    B.xyz = upload(A, xyz);
    B.exps = upload(A, ex);
    B.coefs = upload(A, co);
    B.leaf_lofs = upload(A, lofs);
    B.leaf_lsh = upload(A, lsh.empty() ? std::vector<int>{0} : lsh);
    B.leaf_one = one_per_l ? upload(A, one) : nullptr;
    T->boys = upload(A, boys_table());
    // primitive pairs of every ordered pair of primitives
    {
        const long Nt = (long)ex.size();
        std::vector<int> prim_shell(Nt);
        for (int t = 0; t < S; ++t)
            for (int p = 0; p < np[t]; ++p) prim_shell[pofs[t] + p] = t;
        DevArena tmp(st);
        int* dps = upload(tmp, prim_shell);
        FxPrimPair* pp = A.get<FxPrimPair>((size_t)Nt * Nt);
        fx_launch_prim_pairs(B.exps, B.coefs, dps, B.xyz, Nt, pp, st);
        FX_HIP(hipGetLastError());
        FX_HIP(hipStreamSynchronize(st));
        B.ntprim = Nt;
        B.pp = pp;
    }
    std::vector<int> tfp(S + 1, 0);
    for (int t = 0; t < S; ++t) tfp[t + 1] = tfp[t] + ncart(l[t]);
    for (const Level& L : P.levels) {
        T->d_sL.push_back(upload(A, L.sL));
        T->d_sR.push_back(upload(A, L.sR));
        T->d_ch0.push_back(upload(A, L.ch0));
        T->d_nch.push_back(upload(A, L.nch));
        std::vector<int> nf(L.sL.size());
        for (size_t i = 0; i < nf.size(); ++i) nf[i] = tfp[L.sR[i]] - tfp[L.sL[i]];
        T->d_nf.push_back(upload(A, nf));
    }
    // Schwarz norms of all shell pairs
    double* Qn = A.get<double>((size_t)S * S);
    B.Qn = Qn;
    {
        std::vector<int2> pairs;
        pairs.reserve((size_t)S * (S + 1) / 2);
        for (int a = 0; a < S; ++a)
            for (int b = a; b < S; ++b) pairs.push_back(make_int2(a, b));
        DevArena tmp(st);
        int2* dp = upload(tmp, pairs);
        fx_launch_schwarz(B, T->boys, dp, (long)pairs.size(), Qn, st);
        FX_HIP(hipGetLastError());
        FX_HIP(hipStreamSynchronize(st));
    }
    // largest overlaps of the shell pairs and their block maxima per level (Eqs. 3-4)
    double* Sm = A.get<double>((size_t)S * S);
    B.Sm = Sm;
    {
        std::vector<int2> pairs;
        pairs.reserve((size_t)S * (S + 1) / 2);
        for (int a = 0; a < S; ++a)
            for (int b = a; b < S; ++b) pairs.push_back(make_int2(a, b));
        DevArena tmp(st);
        int2* dp = upload(tmp, pairs);
        fx_launch_overlap_max(B, dp, (long)pairs.size(), Sm, st);
        FX_HIP(hipGetLastError());
        FX_HIP(hipStreamSynchronize(st));
    }
    T->qrow = A.get<double>(S);
    fx_launch_qrow(Qn, S, T->qrow, st);
    {
        double sum[3] = {0, 0, 0}, cnt[3] = {0, 0, 0};
        for (int t = 0; t < S; ++t) {
            sum[l[t]] += np[t];
            cnt[l[t]] += 1;
        }
        for (int L = 0; L < 3; ++L) T->mean_np[L] = cnt[L] > 0 ? (float)(sum[L] / cnt[L]) : 1.f;
    }
    // squared block norms of Q at every level
    const int nl = (int)P.levels.size();
    T->d_Qsq.resize(nl);
    T->d_Smx.resize(nl);
    for (int k = nl - 1; k >= 0; --k) {
        const int nk = (int)P.levels[k].sL.size();
        T->d_Smx[k] = A.get<double>((size_t)nk * nk);
        if (k == nl - 1)
            fx_launch_leaf_max(Sm, S, T->d_sL[k], T->d_sR[k], nk, T->d_Smx[k], st);
        else
            fx_launch_level_max(T->d_Smx[k + 1], (int)P.levels[k + 1].sL.size(), T->d_ch0[k], T->d_nch[k], nk,
                                T->d_Smx[k], st);
        T->d_Qsq[k] = A.get<double>((size_t)nk * nk);
        if (k == nl - 1)
            fx_launch_leaf_sq(Qn, S, T->d_sL[k], T->d_sR[k], nk, T->d_Qsq[k], st);
        else
            fx_launch_level_up(T->d_Qsq[k + 1], (int)P.levels[k + 1].sL.size(), T->d_ch0[k], T->d_nch[k], nk,
                               T->d_Qsq[k], st);
    }
    FX_HIP(hipGetLastError());
    FX_HIP(hipStreamSynchronize(st));
}

// ---------------------------------------------------------------------------
// per class and precision: kernel variant (0 thread-per-quartet, 1 wave-per-
// quartet) and launch flags (FX_LAUNCH_*); thread form, no flags by default,
// the autotuner may switch
// ---------------------------------------------------------------------------
int g_variant[81][2];
int g_flags[81][2];
static bool g_variant_init = [] {
    for (int c = 0; c < 81; ++c)
        for (int p = 0; p < 2; ++p) {
            g_variant[c][p] = (fx_class_variants[c] & 1) ? ((p == 0 && fx_class_dual_default[c]) ? 2 : 0) : 1;
            g_flags[c][p] = 0;
        }
    return true;
}();

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

fx_status fx_build_quadtree(const fx_shells* shells, const fx_tree_opts* opts, void* stream, fx_tree** out) {
    return fx_guard([&] {
        if (!out) fx_fail(FX_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        fx_tree* T = new fx_tree();
        try {
            build_tree(shells, opts, (hipStream_t)stream, T);
        } catch (...) {
            delete T;
            throw;
        }
        *out = T;
    });
}





int32_t fx_nbf(const fx_tree* tree) { return tree ? tree->n : -1; }
int32_t fx_nshell(const fx_tree* tree) { return tree ? tree->S : -1; }

fx_status fx_tree_perm(const fx_tree* tree, int32_t* perm) {
    return fx_guard([&] {
        if (!tree || !perm) fx_fail(FX_ERR_INVALID_ARG, "NULL argument");
        for (int i = 0; i < tree->S; ++i) perm[i] = tree->order[i];
    });
}

int32_t fx_tree_levels(const fx_tree* tree, int64_t* nodes) {
    if (!tree) return -1;
    if (nodes)
        for (size_t k = 0; k < tree->levels.size(); ++k) nodes[k] = (int64_t)tree->levels[k].sL.size();
    return (int32_t)tree->levels.size();
}

fx_status fx_tree_schwarz(const fx_tree* tree, double* Qh) {
    return fx_guard([&] {
        if (!tree || !Qh) fx_fail(FX_ERR_INVALID_ARG, "NULL argument");
        const int S = tree->S;
        std::vector<double> q((size_t)S * S);
        FX_HIP(hipMemcpy(q.data(), tree->basis.Qn, sizeof(double) * q.size(), hipMemcpyDeviceToHost));
        for (int a = 0; a < S; ++a)
            for (int b = 0; b < S; ++b) Qh[(size_t)tree->order[a] * S + tree->order[b]] = q[(size_t)a * S + b];
    });
}

fx_status fx_tree_overlap(const fx_tree* tree, double* Sm_host) {
    return fx_guard([&] {
        if (!tree || !Sm_host) fx_fail(FX_ERR_INVALID_ARG, "NULL argument");
        const int S = tree->S;
        std::vector<double> q((size_t)S * S);
        FX_HIP(hipMemcpy(q.data(), tree->basis.Sm, sizeof(double) * q.size(), hipMemcpyDeviceToHost));
        for (int a = 0; a < S; ++a)
            for (int b = 0; b < S; ++b) Sm_host[(size_t)tree->order[a] * S + tree->order[b]] = q[(size_t)a * S + b];
    });
}

void fx_tree_free(fx_tree* tree) { delete tree; }

fx_status fx_set_allocator(fx_alloc_fn alloc, fx_free_fn free_, void* ctx) {
    return fx_guard([&] {
        if ((alloc == nullptr) != (free_ == nullptr)) fx_fail(FX_ERR_INVALID_ARG, "give both callbacks or neither");
        g_alloc = alloc;
        g_free = free_;
        g_alloc_ctx = ctx;
    });
}

const char* fx_status_string(fx_status s) {
    switch (s) {
        case FX_OK: return "FX_OK";
        case FX_ERR_INVALID_ARG: return "FX_ERR_INVALID_ARG";
        case FX_ERR_UNSUPPORTED: return "FX_ERR_UNSUPPORTED";
        case FX_ERR_OOM: return "FX_ERR_OOM";
        case FX_ERR_HIP: return "FX_ERR_HIP";
        case FX_ERR_INTERNAL: return "FX_ERR_INTERNAL";
    }
    return "FX_ERR_UNKNOWN";
}

const char* fx_last_error_message(void) { return g_last_error.c_str(); }

fx_status fx_set_class_variant(int32_t cls, int32_t prec32, int32_t variant) {
    return fx_guard([&] {
        if (cls < 0 || cls >= 81 || prec32 < 0 || prec32 > 1 || variant < 0 || variant > 2)
            fx_fail(FX_ERR_INVALID_ARG, "class 0..80, prec32 0..1, variant 0..2");
        if (variant == 2 && prec32 != 0) fx_fail(FX_ERR_INVALID_ARG, "variant 2 is set on the FP64 entry");
        if (!(fx_class_variants[cls] & (1 << variant))) fx_fail(FX_ERR_UNSUPPORTED, "variant not built for this class");
        g_variant[cls][prec32] = variant;
    });
}

fx_status fx_set_class_launch(int32_t cls, int32_t prec32, int32_t flags) {
    return fx_guard([&] {
        if (cls < 0 || cls >= 81 || prec32 < 0 || prec32 > 1 || flags < 0 || flags > 3)
            fx_fail(FX_ERR_INVALID_ARG, "class 0..80, prec32 0..1, flags 0..3");
        if (flags & 2) fx_fail(FX_ERR_UNSUPPORTED, "persistent class launches are switched off");
        g_flags[cls][prec32] = flags;
    });
}

int32_t fx_get_class_launch(int32_t cls, int32_t prec32) {
    if (cls < 0 || cls >= 81 || prec32 < 0 || prec32 > 1) return -1;
    return g_flags[cls][prec32];
}

int32_t fx_get_class_variant(int32_t cls, int32_t prec32) {
    if (cls < 0 || cls >= 81 || prec32 < 0 || prec32 > 1) return -1;
    return g_variant[cls][prec32];
}

int32_t fx_class_variants_available(int32_t cls) {
    if (cls < 0 || cls >= 81) return 0;
    return fx_class_variants[cls];
}


fx_status fx_task_timings_create(const float* feats, const float* log2_ns, const int32_t* cls, int64_t n,
                                 fx_task_timings** out) {
    return fx_guard([&] {
        if (!out || n < 0 || (n > 0 && (!feats || !log2_ns))) fx_fail(FX_ERR_INVALID_ARG, "bad arguments");
        fx_task_timings* t = new fx_task_timings();
        t->feat.assign(feats, feats + 4 * n);
        t->log2ns.assign(log2_ns, log2_ns + n);
        t->cls.resize(n, -1);
        if (cls)
            for (int64_t i = 0; i < n; ++i) t->cls[i] = cls[i];
        *out = t;
    });
}

int64_t fx_task_timings_count(const fx_task_timings* t) { return t ? (int64_t)t->log2ns.size() : -1; }

fx_status fx_task_timings_get(const fx_task_timings* t, float* feats, float* log2_ns, int32_t* cls) {
    return fx_guard([&] {
        if (!t) fx_fail(FX_ERR_INVALID_ARG, "timings is NULL");
        if (feats) std::copy(t->feat.begin(), t->feat.end(), feats);
        if (log2_ns) std::copy(t->log2ns.begin(), t->log2ns.end(), log2_ns);
        if (cls) std::copy(t->cls.begin(), t->cls.end(), cls);
    });
}

void fx_task_timings_free(fx_task_timings* t) { delete t; }

fx_status fx_costmodel_create(const float* params, const float* norm, fx_costmodel** out) {
    return fx_guard([&] {
        if (!params || !norm || !out) fx_fail(FX_ERR_INVALID_ARG, "NULL argument");
        fx_costmodel* m = new fx_costmodel();
        m->W.assign(params, params + FX_MLP_NPARAM);
        m->norm.assign(norm, norm + FX_MLP_NNORM);
        try {
            m->upload();
        } catch (...) {
            delete m;
            throw;
        }
        *out = m;
    });
}

fx_status fx_costmodel_params(const fx_costmodel* m, float* params, float* norm) {
    return fx_guard([&] {
        if (!m) fx_fail(FX_ERR_INVALID_ARG, "model is NULL");
        if (params) std::copy(m->W.begin(), m->W.end(), params);
        if (norm) std::copy(m->norm.begin(), m->norm.end(), norm);
    });
}

void fx_costmodel_free(fx_costmodel* m) { delete m; }

// File format: the 8 bytes "FXMLP001", two little-endian uint32 (parameter
// and normalisation counts), then the parameters and the normalisation as
// little-endian IEEE binary32, in the order of fx_costmodel_params.
static const char kMlpMagic[8] = {'F', 'X', 'M', 'L', 'P', '0', '0', '1'};

fx_status fx_costmodel_save(const fx_costmodel* m, const char* path) {
    return fx_guard([&] {
        if (!m || !path) fx_fail(FX_ERR_INVALID_ARG, "NULL argument");
        FILE* f = std::fopen(path, "wb");
        if (!f) fx_fail(FX_ERR_INVALID_ARG, std::string("cannot open ") + path + " for writing");
        const uint32_t np = FX_MLP_NPARAM, nn = FX_MLP_NNORM;
        bool ok = std::fwrite(kMlpMagic, 1, 8, f) == 8 && std::fwrite(&np, 4, 1, f) == 1 &&
                  std::fwrite(&nn, 4, 1, f) == 1 && std::fwrite(m->W.data(), 4, np, f) == np &&
                  std::fwrite(m->norm.data(), 4, nn, f) == nn;
        ok = (std::fclose(f) == 0) && ok;
        if (!ok) fx_fail(FX_ERR_INVALID_ARG, std::string("write to ") + path + " failed");
    });
}

fx_status fx_costmodel_load(const char* path, fx_costmodel** out) {
    return fx_guard([&] {
        if (!path || !out) fx_fail(FX_ERR_INVALID_ARG, "NULL argument");
        *out = nullptr;
        FILE* f = std::fopen(path, "rb");
        if (!f) fx_fail(FX_ERR_INVALID_ARG, std::string("cannot open ") + path);
        char magic[8];
        uint32_t np = 0, nn = 0;
        std::vector<float> W(FX_MLP_NPARAM), norm(FX_MLP_NNORM);
        bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMlpMagic, 8) == 0 &&
                  std::fread(&np, 4, 1, f) == 1 && std::fread(&nn, 4, 1, f) == 1 && np == FX_MLP_NPARAM &&
                  nn == FX_MLP_NNORM && std::fread(W.data(), 4, np, f) == np && std::fread(norm.data(), 4, nn, f) == nn;
        char extra;
        ok = ok && std::fread(&extra, 1, 1, f) == 0;
        std::fclose(f);
        if (!ok) fx_fail(FX_ERR_INVALID_ARG, std::string(path) + " is not a cost-model file of this library");
        for (float v : W)
            if (!std::isfinite(v)) fx_fail(FX_ERR_INVALID_ARG, "non-finite parameter in the cost-model file");
        for (int k = 0; k < FX_MLP_NNORM; ++k)
            if (!std::isfinite(norm[k]) || (k >= 4 && k < 8 && !(norm[k] > 0.f)) || (k == 9 && !(norm[k] > 0.f)))
                fx_fail(FX_ERR_INVALID_ARG, "invalid normalisation in the cost-model file");
        fx_costmodel* m = new fx_costmodel();
        m->W = W;
        m->norm = norm;
        try {
            m->upload();
        } catch (...) {
            delete m;
            throw;
        }
        *out = m;
    });
}

int32_t fx_costmodel_nparams(void) { return FX_MLP_NPARAM; }

fx_status fx_costmodel_predict(const fx_costmodel* m, const float* feats, int64_t n, float* out, void* stream) {
    return fx_guard([&] {
        if (!m || (n > 0 && (!feats || !out))) fx_fail(FX_ERR_INVALID_ARG, "NULL argument");
        if (n == 0) return;
        hipStream_t st = (hipStream_t)stream;
        DevArena A(st);
        float4* f = A.get<float4>(n);
        float* y = A.get<float>(n);
        FX_HIP(hipMemcpyAsync(f, feats, sizeof(float4) * n, hipMemcpyHostToDevice, st));
        fx_launch_mlp_predict(m->dW, m->dnorm, f, nullptr, n, y, st);
        FX_HIP(hipMemcpyAsync(out, y, sizeof(float) * n, hipMemcpyDeviceToHost, st));
        FX_HIP(hipStreamSynchronize(st));
    });
}

// loss = mean((y - t)^2) on standardised targets, and its gradient
static void mlp_loss_grad_dev(const fx_costmodel* m, const float4* f, const float* t, const int* idx, long n, float* act,
                              float* lterm, float* grad, float* loss, hipStream_t st) {
    fx_mlp_backprop_grad(m->dW, m->dnorm, f, t, idx, n, act, lterm, grad, loss, st);
}

fx_status fx_costmodel_loss_grad(const fx_costmodel* m, const float* feats, const float* log2_ns, int64_t n,
                                 float* loss, float* grad, void* stream) {
    return fx_guard([&] {
        if (!m || n <= 0 || !feats || !log2_ns) fx_fail(FX_ERR_INVALID_ARG, "bad arguments");
        hipStream_t st = (hipStream_t)stream;
        DevArena A(st);
        float4* f = A.get<float4>(n);
        float* t = A.get<float>(n);
        float* act = A.get<float>((size_t)n * FX_MLP_ACT);
        float* lt = A.get<float>(n);
        float* g = A.get<float>(FX_MLP_NPARAM);
        float* l = A.get<float>(1);
        FX_HIP(hipMemcpyAsync(f, feats, sizeof(float4) * n, hipMemcpyHostToDevice, st));
        FX_HIP(hipMemcpyAsync(t, log2_ns, sizeof(float) * n, hipMemcpyHostToDevice, st));
        mlp_loss_grad_dev(m, f, t, nullptr, n, act, lt, g, l, st);
        if (grad) FX_HIP(hipMemcpyAsync(grad, g, sizeof(float) * FX_MLP_NPARAM, hipMemcpyDeviceToHost, st));
        if (loss) FX_HIP(hipMemcpyAsync(loss, l, sizeof(float), hipMemcpyDeviceToHost, st));
        FX_HIP(hipStreamSynchronize(st));
    });
}

// Train a cost model on GPU: standardise inputs and targets, Glorot-uniform
// initialisation from a seeded generator, Adam on seeded minibatches.
fx_status fx_costmodel_train(const fx_task_timings* data, const fx_train_opts* opts, fx_costmodel** out,
                             float* final_loss, void* stream) {
    return fx_guard([&] {
        if (!data || !out) fx_fail(FX_ERR_INVALID_ARG, "NULL argument");
        const long n = (long)data->log2ns.size();
        if (n < 8) fx_fail(FX_ERR_INVALID_ARG, "need at least 8 samples");
        fx_train_opts o{2000, 8192, 3e-3f, 12345};
        if (opts) o = *opts;
        if (o.steps <= 0 || o.batch <= 0 || !(o.lr > 0.f)) fx_fail(FX_ERR_INVALID_ARG, "bad training options");
        hipStream_t st = (hipStream_t)stream;
        fx_costmodel* m = new fx_costmodel();
        std::unique_ptr<fx_costmodel> guard(m);
        m->norm.assign(FX_MLP_NNORM, 0.f);
        for (int k = 0; k < 4; ++k) {
            double mu = 0, s2 = 0;
            for (long i = 0; i < n; ++i) mu += data->feat[4 * i + k];
            mu /= n;
            for (long i = 0; i < n; ++i) s2 += (data->feat[4 * i + k] - mu) * (data->feat[4 * i + k] - mu);
            m->norm[k] = (float)mu;
            m->norm[4 + k] = (float)std::max(1e-3, std::sqrt(s2 / n));
        }
        {
            double mu = 0, s2 = 0;
            for (long i = 0; i < n; ++i) mu += data->log2ns[i];
            mu /= n;
            for (long i = 0; i < n; ++i) s2 += (data->log2ns[i] - mu) * (data->log2ns[i] - mu);
            m->norm[8] = (float)mu;
            m->norm[9] = (float)std::max(1e-3, std::sqrt(s2 / n));
        }
        // splitmix64 stream for initialisation and minibatches
        uint64_t state = o.seed;
        auto next = [&]() {
            uint64_t z = (state += 0x9E3779B97F4A7C15ull);
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            return z ^ (z >> 31);
        };
        auto unif = [&]() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); };
        m->W.assign(FX_MLP_NPARAM, 0.f);
        auto glorot = [&](int off, int fan_in, int fan_out) {
            const double a = std::sqrt(6.0 / (fan_in + fan_out));
            for (int i = 0; i < fan_in * fan_out; ++i) m->W[off + i] = (float)((2 * unif() - 1) * a);
        };
        glorot(FX_MLP_W1, FX_MLP_IN, FX_MLP_H);
        glorot(FX_MLP_W2, FX_MLP_H, FX_MLP_H);
        glorot(FX_MLP_W3, FX_MLP_H, 1);
        m->upload();
        DevArena A(st);
        const long B = std::min<long>(o.batch, n);
        float4* f = A.get<float4>(n);
        float* t = A.get<float>(n);
        float* act = A.get<float>((size_t)std::max(B, n < 65536 ? n : B) * FX_MLP_ACT);
        float* lt = A.get<float>(std::max(B, n));
        float* g = A.get<float>(FX_MLP_NPARAM);
        float* mo = A.get<float>(FX_MLP_NPARAM);
        float* vo = A.get<float>(FX_MLP_NPARAM);
        float* l = A.get<float>(1);
        int* idx = A.get<int>(B);
        FX_HIP(hipMemcpyAsync(f, data->feat.data(), sizeof(float) * 4 * n, hipMemcpyHostToDevice, st));
        FX_HIP(hipMemcpyAsync(t, data->log2ns.data(), sizeof(float) * n, hipMemcpyHostToDevice, st));
        FX_HIP(hipMemsetAsync(mo, 0, sizeof(float) * FX_MLP_NPARAM, st));
        FX_HIP(hipMemsetAsync(vo, 0, sizeof(float) * FX_MLP_NPARAM, st));
        std::vector<int> hidx(B);
        for (int step = 1; step <= o.steps; ++step) {
            for (long i = 0; i < B; ++i) hidx[i] = B == n ? (int)i : (int)(next() % (uint64_t)n);
            FX_HIP(hipMemcpyAsync(idx, hidx.data(), sizeof(int) * B, hipMemcpyHostToDevice, st));
            mlp_loss_grad_dev(m, f, t, idx, B, act, lt, g, l, st);
            fx_mlp_adam(m->dW, g, mo, vo, o.lr, step, st);
            FX_HIP(hipStreamSynchronize(st));   // idx host buffer is reused next step
        }
        FX_HIP(hipMemcpyAsync(m->W.data(), m->dW, sizeof(float) * FX_MLP_NPARAM, hipMemcpyDeviceToHost, st));
        if (final_loss) {
            // loss over the whole data set (minibatches of the activation buffer size)
            const long chunk = n < 65536 ? n : B;
            double acc = 0;
            for (long s0 = 0; s0 < n; s0 += chunk) {
                const long cn = std::min(chunk, n - s0);
                float lv = 0.f;
                mlp_loss_grad_dev(m, f + s0, t + s0, nullptr, cn, act, lt, g, l, st);
                FX_HIP(hipMemcpyAsync(&lv, l, sizeof(float), hipMemcpyDeviceToHost, st));
                FX_HIP(hipStreamSynchronize(st));
                acc += (double)lv * cn;
            }
            *final_loss = (float)(acc / n);
        }
        FX_HIP(hipStreamSynchronize(st));
        *out = guard.release();
    });
}

int64_t fx_xcd_block(int64_t b, int64_t nb) { return (b < 0 || b >= nb) ? -1 : fx_xcd_remap(b, nb); }

// Host-only planning (no device work): the tree order and the bisection
// levels.  perm[nshell]; nodes: 4 ints per node (level, first shell, end
// shell, children) for all levels, capacity given in node_cap.  Returns the
// number of levels through *nlevels and the node count through *nnodes.
fx_status fx_plan_tree(const fx_shells* shells, const fx_tree_opts* opts, int32_t* perm, int32_t* nlevels,
                       int32_t* nodes, int64_t node_cap, int64_t* nnodes) {
    return fx_guard([&] {
        validate_shells(shells);
        Plan P = make_plan(shells, opts);
        if (perm)
            for (int i = 0; i < shells->nshell; ++i) perm[i] = P.order[i];
        if (nlevels) *nlevels = (int32_t)P.levels.size();
        int64_t k = 0;
        for (size_t lv = 0; lv < P.levels.size(); ++lv)
            for (size_t i = 0; i < P.levels[lv].sL.size(); ++i, ++k)
                if (nodes && k < node_cap) {
                    nodes[4 * k] = (int32_t)lv;
                    nodes[4 * k + 1] = P.levels[lv].sL[i];
                    nodes[4 * k + 2] = P.levels[lv].sR[i];
                    nodes[4 * k + 3] = P.levels[lv].nch[i];
                }
        if (nnodes) *nnodes = k;
    });
}

}  // extern "C"
