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
#include "eri_flops.h"
#include "eri_table.h"
#include "fx_costmodel.h"
#include "fx_internal.h"
#include "fx_kernels.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

struct FxError {
    fx_status st;
    std::string msg;
};

[[noreturn]] static void fx_fail(fx_status st, const std::string& msg) { throw FxError{st, msg}; }

#define FX_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) fx_fail(FX_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

static fx_status fx_guard_status(const FxError& e) {
    g_last_error = e.msg;
    return e.st;
}

template <typename F>
static fx_status fx_guard(F&& f) {
    try {
        f();
        g_last_error.clear();
        return FX_OK;
    } catch (const FxError& e) {
        return fx_guard_status(e);
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return FX_ERR_OOM;
    } catch (...) {
        g_last_error = "internal error";
        return FX_ERR_INTERNAL;
    }
}

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------
static fx_alloc_fn g_alloc = nullptr;
static fx_free_fn g_free = nullptr;
static void* g_alloc_ctx = nullptr;

static void* fx_dalloc(size_t bytes, hipStream_t st, bool persistent = false) {
    if (bytes == 0) bytes = 8;
    void* p = nullptr;
    if (persistent) {
        // memory owned by a tree handle outlives the caller's stream
        if (hipMalloc(&p, bytes) != hipSuccess || !p) {
            (void)hipGetLastError();
            fx_fail(FX_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        }
        return p;
    }
    if (g_alloc) {
        p = g_alloc(bytes, (void*)st, g_alloc_ctx);
        if (!p) fx_fail(FX_ERR_OOM, "allocator callback returned NULL for " + std::to_string(bytes) + " bytes");
        return p;
    }
    hipError_t e = hipMallocAsync(&p, bytes, st);
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        fx_fail(FX_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return p;
}

static void fx_dfree(void* p, hipStream_t st, bool persistent = false) {
    if (!p) return;
    if (persistent) {
        (void)hipFree(p);
        return;
    }
    if (g_free) g_free(p, (void*)st, g_alloc_ctx);
    else (void)hipFreeAsync(p, st);
}

// RAII set of device allocations tied to a stream
struct DevArena {
    hipStream_t st;
    bool persistent;
    std::vector<void*> ptrs;
    explicit DevArena(hipStream_t s, bool pers = false) : st(s), persistent(pers) {}
    template <typename T>
    T* get(size_t count) {
        T* p = (T*)fx_dalloc(sizeof(T) * count, st, persistent);
        ptrs.push_back(p);
        return p;
    }
    void release(void* p) {
        auto it = std::find(ptrs.begin(), ptrs.end(), p);
        if (it != ptrs.end()) {
            fx_dfree(p, st, persistent);
            ptrs.erase(it);
        }
    }
    ~DevArena() {
        for (void* p : ptrs) fx_dfree(p, st, persistent);
    }
};

template <typename T>
static T* upload(DevArena& A, const std::vector<T>& v) {
    T* d = A.get<T>(v.size());
    if (!v.empty()) FX_HIP(hipMemcpyAsync(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, A.st));
    return d;
}

template <typename T>
static T read1(const T* dptr, hipStream_t st) {
    T v;
    FX_HIP(hipMemcpyAsync(&v, dptr, sizeof(T), hipMemcpyDeviceToHost, st));
    FX_HIP(hipStreamSynchronize(st));
    return v;
}

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

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

// ---------------------------------------------------------------------------
// host plan: ordering + ragged bisection
// ---------------------------------------------------------------------------
struct Level {
    std::vector<int> sL, sR, ch0, nch;  // nodes of this level; ch0/nch index level+1
};

struct Plan {
    std::vector<int> order;   // tree position -> caller shell index
    std::vector<Level> levels;
};

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

// ---------------------------------------------------------------------------
// the tree handle
// ---------------------------------------------------------------------------
struct fx_tree {
    int S = 0, n = 0, lmax = 0;
    std::vector<int> order;          // tree position -> caller shell
    std::vector<int> l, nprim;       // tree order
    std::vector<int> f0;             // tree order, caller function offset
    std::vector<Level> levels;
    std::vector<int> leaf_lofs;      // host copy
    bool single_shell_leaves = false;
    hipStream_t build_stream = nullptr;
    DevArena* arena = nullptr;
    FxDevBasis basis{};
    double* boys = nullptr;
    std::vector<int*> d_sL, d_sR, d_ch0, d_nch;
    std::vector<double*> d_Qsq;      // per level (nk x nk)
    double* qrow = nullptr;          // max_b Qn[s][b]
    float mean_np[3] = {1, 1, 1};    // mean primitive count of the shells of each l
    ~fx_tree() {
        if (arena) (void)hipDeviceSynchronize();
        delete arena;
    }
};

struct fx_costmodel {
    std::vector<float> W, norm;    // FX_MLP_NPARAM, FX_MLP_NNORM
    float* dW = nullptr;
    float* dnorm = nullptr;
    ~fx_costmodel() {
        if (dW) (void)hipFree(dW);
        if (dnorm) (void)hipFree(dnorm);
    }
    void upload() {
        if (!dW) {
            if (hipMalloc(&dW, sizeof(float) * FX_MLP_NPARAM) != hipSuccess ||
                hipMalloc(&dnorm, sizeof(float) * FX_MLP_NNORM) != hipSuccess)
                fx_fail(FX_ERR_OOM, "cost model allocation failed");
        }
        FX_HIP(hipMemcpy(dW, W.data(), sizeof(float) * FX_MLP_NPARAM, hipMemcpyHostToDevice));
        FX_HIP(hipMemcpy(dnorm, norm.data(), sizeof(float) * FX_MLP_NNORM, hipMemcpyHostToDevice));
    }
};

struct fx_task_timings {
    std::vector<float> feat;    // 4 per sample
    std::vector<float> log2ns;  // measured unit time
    std::vector<int> cls;       // cls * 2 + fp32
};

static void build_tree(const fx_shells* s, const fx_tree_opts* opts, hipStream_t st, fx_tree* T) {
    validate_shells(s);
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
    for (const Level& L : P.levels) {
        T->d_sL.push_back(upload(A, L.sL));
        T->d_sR.push_back(upload(A, L.sR));
        T->d_ch0.push_back(upload(A, L.ch0));
        T->d_nch.push_back(upload(A, L.nch));
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
    for (int k = nl - 1; k >= 0; --k) {
        const int nk = (int)P.levels[k].sL.size();
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
static int g_variant[81][2];
static int g_flags[81][2];
static bool g_variant_init = [] {
    for (int c = 0; c < 81; ++c)
        for (int p = 0; p < 2; ++p) {
            g_variant[c][p] = (fx_class_variants[c] & 1) ? ((p == 0 && fx_class_dual_default[c]) ? 2 : 0) : 1;
            g_flags[c][p] = 0;
        }
    return true;
}();

// ---------------------------------------------------------------------------
// exchange
// ---------------------------------------------------------------------------
struct Frontier {
    int2* ad;
    long* bc_off;      // absolute offsets into bc for ad[0..nad]
    int2* bc;
    int* parent;
    int nad;
    long e_begin, e_count;
    int p_base;
};

// one system of a call: tree, density, output and its per-call arrays
struct SysCtx {
    const fx_tree* T = nullptr;
    const double* P[FX_MAX_DENS] = {nullptr, nullptr};
    double* K[FX_MAX_DENS] = {nullptr, nullptr};
    double* Pn = nullptr;
    std::vector<double*> Psq;
    double* slots = nullptr;
    int sym = 0;                    // symmetric density: only K blocks a <= d are built
};

// a leaf-level traversal chunk, ready for the class launches
struct LeafSeg {
    std::unique_ptr<DevArena> arena;
    FxSys sys{};
    const fx_tree* T = nullptr;
    int* units = nullptr;
    long bounds[10] = {0};
    long nitems = 0;
};

struct ExCtx {
    double tau;
    hipStream_t st;
    int precision;
    double thr;
    int schedule;
    const fx_costmodel* cm;
    long cap;
    int L;                          // slot layout: (highest l + 1)^2 (x2 in mixed mode)
    int nslot;
    int ndens = 1;                  // densities per system, contracted with the same integrals
    bool collect = false;           // batched: keep leaf segments for one launch per class
    bool use_graph = false;
    std::vector<std::unique_ptr<LeafSeg>> segs;
    unsigned long long* counters;   // [81][2][2]: quartets, primitive quartets per class and precision
    fx_stats* stats;
    long* scan_partial;
    long scan_partial_cap;
    long* scan_total;
    double seconds_eri = 0;
    int profile = 0;
    fx_task_timings* rec = nullptr;   // timing-probe collection
    double tick_ns = 10.0;            // wall-clock tick
    struct Timed {
        int idx;
        hipEvent_t a, b;
    };
    std::vector<Timed> timed;
};

static thread_local fx_task_timings* g_recording = nullptr;

static int slot_index(const ExCtx& c, int lb, int lc, int prec32) {
    return (lb * c.L + lc) * (c.precision == FX_PREC_MIXED ? 2 : 1) + prec32;
}

static long* scan_partial(ExCtx& c, DevArena& A, long n) {
    const long need = fx_scan_tiles(n);
    if (need > c.scan_partial_cap) return A.get<long>(need);
    return c.scan_partial;
}

// Units (K blocks) of a leaf chunk and, for single-shell leaves, its entries
// grouped by density-side class.  In collect mode the chunk's entries are
// copied so that the segment outlives the traversal.
static std::unique_ptr<LeafSeg> prepare_seg(ExCtx& c, SysCtx& sc, const Frontier& f) {
    const fx_tree* T = sc.T;
    hipStream_t st = c.st;
    auto seg = std::make_unique<LeafSeg>();
    seg->arena = std::make_unique<DevArena>(st);
    DevArena& A = *seg->arena;
    seg->T = T;
    const long nitems = f.nad;
    seg->nitems = nitems;
    if (f.e_begin != 0) fx_fail(FX_ERR_INTERNAL, "leaf frontier does not start at entry 0");
    if (c.stats) c.stats->leaf_items += nitems;
    int* cnt = A.get<int>(9 * nitems);
    long* upos = A.get<long>(9 * nitems + 1);
    fx_launch_unit_count(f.ad, nitems, T->basis.leaf_lofs, T->basis.leaf_lsh, sc.sym, cnt, st);
    fx_scan_i32(cnt, 9 * nitems, upos, scan_partial(c, A, 9 * nitems), c.scan_total, st);
    for (int k = 0; k < 9; ++k)
        FX_HIP(hipMemcpyAsync(&seg->bounds[k], upos + (long)k * nitems, sizeof(long), hipMemcpyDeviceToHost, st));
    FX_HIP(hipMemcpyAsync(&seg->bounds[9], upos + 9 * nitems, sizeof(long), hipMemcpyDeviceToHost, st));
    FX_HIP(hipStreamSynchronize(st));
    const long nunits = seg->bounds[9];
    if (c.stats) c.stats->units += nunits;
    seg->units = A.get<int>(3 * std::max(1L, nunits));
    fx_launch_unit_write(f.ad, nitems, 0, T->basis.leaf_lofs, T->basis.leaf_lsh, sc.sym, upos, seg->units, st);
    A.release(cnt);
    A.release(upos);
    FxSys& Y = seg->sys;
    Y.basis = T->basis;
    for (int j = 0; j < FX_MAX_DENS; ++j) Y.P[j] = sc.P[j < c.ndens ? j : 0];
    Y.n = T->n;
    Y.Pn = sc.Pn;
    Y.bc_off = f.bc_off;
    Y.bc = f.bc;
    Y.cls_off = nullptr;
    Y.slots = sc.slots;
    Y.slot_stride = (long)c.nslot * T->n * T->n;
    Y.sym = sc.sym;
    const long ne = std::max(1L, f.e_count);
    if (T->single_shell_leaves) {
        int2* sorted = A.get<int2>(ne);
        long* cls_off = A.get<long>(10 * nitems);
        fx_launch_class_sort(f.bc_off, f.bc, nitems, T->basis.l, sorted, cls_off, st);
        Y.bc = sorted;
        Y.cls_off = cls_off;
    }
    if (c.collect) {
        long* off = A.get<long>(nitems + 1);
        FX_HIP(hipMemcpyAsync(off, f.bc_off, sizeof(long) * (nitems + 1), hipMemcpyDeviceToDevice, st));
        Y.bc_off = off;
        if (!T->single_shell_leaves) {
            int2* bc = A.get<int2>(ne);
            FX_HIP(hipMemcpyAsync(bc, f.bc, sizeof(int2) * f.e_count, hipMemcpyDeviceToDevice, st));
            Y.bc = bc;
        }
    }
    FX_HIP(hipGetLastError());
    return seg;
}

// One launch per class and precision over the units of all segments.
static void run_classes(ExCtx& c, const std::vector<LeafSeg*>& segs) {
    hipStream_t st = c.st;
    if (segs.empty()) return;
    DevArena A(st);
    const bool multi = segs.size() > 1;
    int lmax = 0;
    for (auto* g : segs) lmax = std::max(lmax, g->T->lmax);
    // per (la, ld): merged unit lists
    long total[9] = {0}, maxlist = 0;
    for (int k = 0; k < 9; ++k) {
        for (auto* g : segs) total[k] += g->bounds[k + 1] - g->bounds[k];
        maxlist = std::max(maxlist, total[k]);
    }
    if (maxlist == 0) return;
    int* munits[9] = {nullptr};
    int* msys[9] = {nullptr};
    FxSys* dsys = nullptr;
    if (multi) {
        std::vector<FxSys> hs;
        for (auto* g : segs) hs.push_back(g->sys);
        dsys = upload(A, hs);
        for (int k = 0; k < 9; ++k) {
            if (!total[k]) continue;
            munits[k] = A.get<int>(3 * total[k]);
            msys[k] = A.get<int>(total[k]);
            long o = 0;
            for (size_t j = 0; j < segs.size(); ++j) {
                const long n = segs[j]->bounds[k + 1] - segs[j]->bounds[k];
                if (!n) continue;
                FX_HIP(hipMemcpyAsync(munits[k] + 3 * o, segs[j]->units + 3 * segs[j]->bounds[k], sizeof(int) * 3 * n,
                                      hipMemcpyDeviceToDevice, st));
                fx_launch_fill_i32(msys[k] + o, n, (int)j, st);
                o += n;
            }
        }
    }
    const bool sched = c.schedule != FX_SCHED_NONE;
    const bool use_mlp = c.schedule == FX_SCHED_MLP && c.cm;
    const int nbins = 32;
    const bool graph = c.use_graph && !c.profile && !c.rec;
    // scheduling buffers (features, predicted costs, bins, launch order)
    struct Sched {
        float4* feat = nullptr;
        float* cost = nullptr;
        int* flags = nullptr;
        uint8_t* key = nullptr;
        long* bpos = nullptr;
        int* order = nullptr;
        long* bpartial = nullptr;
        long* total = nullptr;
    } ln;
    float* times = nullptr;
    if (sched || c.rec) {
        ln.feat = A.get<float4>(maxlist);
        ln.cost = A.get<float>(maxlist);
    }
    if (sched) {
        ln.flags = A.get<int>((size_t)nbins * maxlist);
        ln.key = A.get<uint8_t>(maxlist);
        ln.bpos = A.get<long>((size_t)nbins * maxlist + 1);
        ln.order = A.get<int>(maxlist);
        ln.bpartial = A.get<long>(fx_scan_tiles((long)nbins * maxlist));
        ln.total = A.get<long>(1);
    }
    if (c.rec) times = A.get<float>(maxlist);
    hipGraph_t gr = nullptr;
    // Capture on a library-owned stream (the caller's may be the legacy default
    // stream, which cannot be captured); the graph is then launched on `st`.
    hipStream_t launch_st = st;
    struct CapStream {
        hipStream_t s = nullptr;
        ~CapStream() {
            if (s) (void)hipStreamDestroy(s);
        }
    } cap;
    if (graph) {
        FX_HIP(hipStreamCreateWithFlags(&cap.s, hipStreamNonBlocking));
        FX_HIP(hipStreamBeginCapture(cap.s, hipStreamCaptureModeThreadLocal));
        st = cap.s;
    }
    std::vector<float> hfeat, htime;
    FxClassArgs args{};
    args.boys = segs[0]->T->boys;
    args.ndens = c.ndens;
    args.tau = c.tau;
    args.thr = c.thr;
    const float* mean_np = segs[0]->T->mean_np;
    for (int la = 0; la <= lmax; ++la)
        for (int ld = 0; ld <= lmax; ++ld) {
            const int k2 = la * 3 + ld;
            if (!total[k2]) continue;
            args.nunits = total[k2];
            if (multi) {
                args.units = munits[k2];
                args.unit_sys = msys[k2];
                args.sys = dsys;
            } else {
                args.units = segs[0]->units + 3 * segs[0]->bounds[k2];
                args.unit_sys = nullptr;
                args.sys = nullptr;
                args.one = segs[0]->sys;
            }
            for (int lb = 0; lb <= lmax; ++lb)
                for (int lc = 0; lc <= lmax; ++lc) {
                    const int cls = ((la * 3 + lb) * 3 + lc) * 3 + ld;
                    const int nprec = c.precision == FX_PREC_MIXED ? 2 : 1;
                    const float class_cost =
                        std::log2((float)fx_class_vrr_flops[cls] * mean_np[lb] * mean_np[lc] +
                                  (float)fx_class_hrr_flops[cls] + 1.f);
                    args.order = nullptr;
                    args.times = nullptr;
                    hipStream_t ls = st;
                    if (ln.feat) {
                        long o = 0;
                        for (auto* g : segs) {
                            const long n = g->bounds[k2 + 1] - g->bounds[k2];
                            if (n)
                                fx_launch_unit_features(g->units + 3 * g->bounds[k2], n, g->sys.bc_off, g->sys.cls_off,
                                                        lb * 3 + lc, g->T->basis.nprim, g->T->qrow, class_cost,
                                                        ln.feat + o, ls);
                            o += n;
                        }
                    }
                    if (sched) {
                        // predicted log2 cost per unit: the learned model, or the
                        // bound-only estimate log2(class flops * nprim_a nprim_d * entries)
                        if (use_mlp)
                            fx_launch_mlp_predict(c.cm->dW, c.cm->dnorm, ln.feat, args.nunits, ln.cost, ls);
                        else
                            fx_launch_bound_cost(ln.feat, args.nunits, ln.cost, ls);
                        fx_launch_bin_order(ln.cost, args.nunits, use_mlp ? 40.f : 48.f, 1.0f, nbins, ln.flags,
                                            ln.key, ln.bpos, ln.bpartial, ln.total, ln.order, ls, fx_scan_i32);
                        args.order = ln.order;
                    }
                    // mixed precision in one pass (variant 2 on the FP64 entry, one density)
                    const bool dual = nprec == 2 && c.ndens == 1 && g_variant[cls][0] == 2;
                    for (int pr = 0; pr < (dual ? 1 : nprec); ++pr) {
                        if (c.rec) args.times = times;
                        args.mode = dual ? FX_MODE_DUAL
                                         : c.precision == FX_PREC_MIXED ? (pr ? FX_MODE_MIXED_LO : FX_MODE_MIXED_HI)
                                                                        : FX_MODE_ALL;
                        args.slot_index = slot_index(c, lb, lc, pr);
                        args.counters = c.counters + (cls * 2 + pr) * 3;
                        args.counters2 = dual ? c.counters + (cls * 2 + 1) * 3 : nullptr;
                        args.flags = g_flags[cls][pr];
                        if (c.profile) {
                            // events on the stream the kernel is launched on
                            ExCtx::Timed t{cls * 2 + pr, nullptr, nullptr};
                            FX_HIP(hipEventCreate(&t.a));
                            FX_HIP(hipEventCreate(&t.b));
                            FX_HIP(hipEventRecord(t.a, ls));
                            fx_class_table[cls](pr, g_variant[cls][pr], args, ls);
                            FX_HIP(hipEventRecord(t.b, ls));
                            c.timed.push_back(t);
                        } else {
                            fx_class_table[cls](pr, g_variant[cls][pr], args, ls);
                        }
                        if (c.rec) {
                            const long n = args.nunits;
                            hfeat.resize(4 * n);
                            htime.resize(n);
                            FX_HIP(hipMemcpyAsync(hfeat.data(), ln.feat, sizeof(float4) * n, hipMemcpyDeviceToHost, ls));
                            FX_HIP(hipMemcpyAsync(htime.data(), times, sizeof(float) * n, hipMemcpyDeviceToHost, ls));
                            FX_HIP(hipStreamSynchronize(ls));
                            for (long u = 0; u < n; ++u) {
                                for (int q = 0; q < 4; ++q) c.rec->feat.push_back(hfeat[4 * u + q]);
                                c.rec->log2ns.push_back(std::log2(std::max(1.0, (double)htime[u] * c.tick_ns)));
                                c.rec->cls.push_back(cls * 2 + pr);
                            }
                        }
                    }
                }
        }
    if (graph) {
        FX_HIP(hipStreamEndCapture(cap.s, &gr));
        st = launch_st;
        hipGraphExec_t ge = nullptr;
        hipError_t e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
        if (e == hipSuccess) e = hipGraphLaunch(ge, st);
        if (ge) (void)hipGraphExecDestroy(ge);
        (void)hipGraphDestroy(gr);
        if (e != hipSuccess) fx_fail(FX_ERR_HIP, std::string("class-launch graph: ") + hipGetErrorString(e));
        if (c.stats) c.stats->graph_nodes += 1;
    }
    FX_HIP(hipGetLastError());
    FX_HIP(hipStreamSynchronize(st));
}

static void leaf_work(ExCtx& c, SysCtx& sc, const Frontier& f) {
    if (f.nad == 0) return;
    auto seg = prepare_seg(c, sc, f);
    if (c.collect) {
        c.segs.push_back(std::move(seg));
        return;
    }
    run_classes(c, {seg.get()});
}

static void traverse(ExCtx& c, SysCtx& sc, int k, const Frontier& f) {
    const fx_tree* T = sc.T;
    hipStream_t st = c.st;
    const int nl = (int)T->levels.size();
    if (c.stats) c.stats->frontier[k] += f.e_count;
    if (k == nl - 1) {
        auto t0 = std::chrono::steady_clock::now();
        leaf_work(c, sc, f);
        c.seconds_eri += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return;
    }
    if (f.e_count == 0) return;
    DevArena A(st);
    FxLevelArgs L{};
    L.ad = f.ad;
    L.bc_off = f.bc_off;
    L.bc = f.bc;
    L.bc_parent = f.parent;
    L.e_begin = f.e_begin;
    L.e_count = f.e_count;
    L.p_base = f.p_base;
    L.nad = f.nad;
    L.ch0 = T->d_ch0[k];
    L.nch = T->d_nch[k];
    L.Qsq = T->d_Qsq[k + 1];
    L.Psq = sc.Psq[k + 1];
    L.nk1 = (int)T->levels[k + 1].sL.size();
    L.tau2 = c.tau * c.tau;
    L.sym = sc.sym;
    const long nm = 4 * f.e_count;
    uint8_t* mask = A.get<uint8_t>(nm);
    long* pos = A.get<long>(nm + 1);
    fx_launch_expand_mask(L, mask, st);
    fx_scan_popc_u8(mask, nm, pos, scan_partial(c, A, nm), c.scan_total, st);
    FX_HIP(hipGetLastError());
    const long total = read1(c.scan_total, st);
    if (total > c.cap && f.nad > 1) {
        // chunk: split this level's ADs in two halves and traverse each
        A.release(mask);
        A.release(pos);
        const int h = f.nad / 2;
        const long mid = read1(f.bc_off + h, st);
        Frontier f1 = f, f2 = f;
        f1.nad = h;
        f1.e_count = mid - f.e_begin;
        f2.ad = f.ad + h;
        f2.bc_off = f.bc_off + h;
        f2.nad = f.nad - h;
        f2.e_begin = mid;
        f2.e_count = f.e_begin + f.e_count - mid;
        f2.p_base = f.p_base + h;
        if (c.stats) {
            c.stats->chunks += 1;
            c.stats->frontier[k] -= f.e_count;   // re-counted by the halves
        }
        traverse(c, sc, k, f1);
        traverse(c, sc, k, f2);
        return;
    }
    if (total > (1L << 31) - 1) fx_fail(FX_ERR_OOM, "a single K block pair exceeds the frontier capacity");
    int* flag = A.get<int>(4L * f.nad);
    long* adpos = A.get<long>(4L * f.nad + 1);
    fx_launch_expand_adflag(L, pos, flag, st);
    fx_scan_i32(flag, 4L * f.nad, adpos, scan_partial(c, A, 4L * f.nad), c.scan_total, st);
    const long nads = read1(c.scan_total, st);
    DevArena N(st);
    Frontier g{};
    g.ad = N.get<int2>(std::max(1L, nads));
    g.bc_off = N.get<long>(nads + 1);
    g.bc = N.get<int2>(std::max(1L, total));
    const bool last = (k + 1 == nl - 1);   // the leaf level needs no parent links
    g.parent = last ? nullptr : N.get<int>(std::max(1L, total));
    g.nad = (int)nads;
    g.e_begin = 0;
    g.e_count = total;
    g.p_base = 0;
    fx_launch_expand_adwrite(L, pos, flag, adpos, g.ad, g.bc_off, total, nads, st);
    fx_launch_expand_write(L, mask, pos, adpos, g.bc, g.parent, st);
    FX_HIP(hipGetLastError());
    A.release(mask);
    A.release(pos);
    A.release(flag);
    A.release(adpos);
    traverse(c, sc, k + 1, g);
}

static void validate_exchange(const fx_tree* T, const double* P, double tau, const double* K) {
    if (!T) fx_fail(FX_ERR_INVALID_ARG, "tree is NULL");
    if (!P || !K) fx_fail(FX_ERR_INVALID_ARG, "P and K must be device pointers");
    if (P == K) fx_fail(FX_ERR_INVALID_ARG, "P must not alias K");
    if (!(tau >= 0.0) || !std::isfinite(tau)) fx_fail(FX_ERR_INVALID_ARG, "tau must be finite and >= 0");
    if (((uintptr_t)P & 7) || ((uintptr_t)K & 7)) fx_fail(FX_ERR_INVALID_ARG, "P and K must be 8-byte aligned");
}

static fx_exchange_opts checked_opts(const fx_exchange_opts* opts) {
    fx_exchange_opts o{};
    o.precision = FX_PREC_FP64;
    o.fp32_threshold = 1e-5;
    o.schedule = FX_SCHED_BOUND;
    o.alpha = 1.0;
    o.beta = 0.0;
    if (opts) o = *opts;
    if (o.precision != FX_PREC_FP64 && o.precision != FX_PREC_MIXED) fx_fail(FX_ERR_INVALID_ARG, "bad precision");
    if (o.schedule < 0 || o.schedule > 2) fx_fail(FX_ERR_INVALID_ARG, "bad schedule");
    if (!std::isfinite(o.alpha) || !std::isfinite(o.beta)) fx_fail(FX_ERR_INVALID_ARG, "alpha/beta not finite");
    if (o.precision == FX_PREC_MIXED && !(o.fp32_threshold >= 0.0)) fx_fail(FX_ERR_INVALID_ARG, "bad fp32_threshold");
    if (o.symmetry != FX_SYM_AUTO && o.symmetry != FX_SYM_OFF) fx_fail(FX_ERR_INVALID_ARG, "bad symmetry");
    return o;
}

// Exchange of one or several systems.  Several systems are traversed one
// after another, their leaf segments kept, and every class kernel is then
// launched once over the units of all systems.
// Ps, Ks: count * ndens device pointers, system-major.
static void exchange_many(const fx_tree* const* trees, const double* const* Ps, double* const* Ks, int count,
                          int ndens, double tau, const fx_exchange_opts* opts, fx_stats* stats, hipStream_t st) {
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
    const fx_exchange_opts o = checked_opts(opts);
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (count == 0) return;
    DevArena A(st);
    ExCtx c{};
    c.tau = tau;
    c.st = st;
    c.precision = o.precision;
    c.thr = o.fp32_threshold;
    c.schedule = o.schedule;
    c.cm = o.costmodel;
    c.cap = o.max_frontier_entries > 0 ? o.max_frontier_entries : (1L << 30);
    c.stats = stats;
    c.profile = o.profile;
    c.ndens = ndens;
    c.collect = count > 1;
    c.use_graph = o.use_graph != 0;
    c.rec = g_recording;
    if (c.rec) {
        int dev = 0, khz = 0;
        FX_HIP(hipGetDevice(&dev));
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            c.tick_ns = 1e6 / (double)khz;
    }
    if (o.schedule == FX_SCHED_MLP && !o.costmodel) c.schedule = FX_SCHED_BOUND;
    int lmax = 0;
    for (int i = 0; i < count; ++i) lmax = std::max(lmax, trees[i]->lmax);
    c.L = lmax + 1;
    c.nslot = c.L * c.L * (o.precision == FX_PREC_MIXED ? 2 : 1);
    c.counters = A.get<unsigned long long>(81 * 2 * 3);
    FX_HIP(hipMemsetAsync(c.counters, 0, sizeof(unsigned long long) * 81 * 2 * 3, st));
    c.scan_partial_cap = 1 << 16;
    c.scan_partial = A.get<long>(c.scan_partial_cap);
    c.scan_total = A.get<long>(1);
    std::vector<SysCtx> sys(count);
    for (int i = 0; i < count; ++i) {
        SysCtx& sc = sys[i];
        const fx_tree* T = trees[i];
        sc.T = T;
        for (int j = 0; j < ndens; ++j) {
            sc.P[j] = Ps[i * ndens + j];
            sc.K[j] = Ks[i * ndens + j];
        }
        const int S = T->S;
        const long n = T->n, nn = n * n;
        if (stats) stats->levels = std::max(stats->levels, (int)T->levels.size());
        // density norms; with several densities the largest, so that the
        // screening bounds every density's contribution
        sc.Pn = A.get<double>((size_t)S * S);
        fx_launch_pnorm(sc.P[0], n, T->basis.l, T->basis.f0, S, sc.Pn, st);
        if (ndens > 1) {
            double* Pn2 = A.get<double>((size_t)S * S);
            for (int j = 1; j < ndens; ++j) {
                fx_launch_pnorm(sc.P[j], n, T->basis.l, T->basis.f0, S, Pn2, st);
                fx_launch_max_inplace(sc.Pn, Pn2, (long)S * S, st);
            }
            A.release(Pn2);
        }
        const int nl = (int)T->levels.size();
        sc.Psq.resize(nl);
        for (int k = nl - 1; k >= 0; --k) {
            const int nk = (int)T->levels[k].sL.size();
            sc.Psq[k] = A.get<double>((size_t)nk * nk);
            if (k == nl - 1)
                fx_launch_leaf_sq(sc.Pn, S, T->d_sL[k], T->d_sR[k], nk, sc.Psq[k], st);
            else
                fx_launch_level_up(sc.Psq[k + 1], (int)T->levels[k + 1].sL.size(), T->d_ch0[k], T->d_nch[k], nk,
                                   sc.Psq[k], st);
        }
        // K symmetry: with a bitwise symmetric P, K_da = K_ad^T, so only the
        // K blocks on and above the diagonal (tree order) are built.
        sc.sym = 0;
        if (o.symmetry == FX_SYM_AUTO && (n + 31) / 32 <= 65535) {
            int* flag = A.get<int>(1);
            fx_launch_fill_i32(flag, 1, 0, st);
            for (int j = 0; j < ndens; ++j) fx_launch_psym(sc.P[j], n, flag, st);
            sc.sym = read1(flag, st) == 0 ? 1 : 0;
            A.release(flag);
        }
        if (stats) stats->symmetric_systems += sc.sym;
        sc.slots = A.get<double>((size_t)c.nslot * nn * ndens);
        fx_launch_fill(sc.slots, (long)c.nslot * nn * ndens, 0.0, st);
        FX_HIP(hipGetLastError());
        // root task
        const double q0 = read1(T->d_Qsq[0], st), p0 = read1(sc.Psq[0], st);
        if ((q0 * q0) * p0 * (1.0 + 1e-12) > tau * tau) {
            DevArena R(st);
            Frontier f{};
            f.ad = upload(R, std::vector<int2>{make_int2(0, 0)});
            f.bc_off = upload(R, std::vector<long>{0, 1});
            f.bc = upload(R, std::vector<int2>{make_int2(0, 0)});
            f.parent = upload(R, std::vector<int>{0});
            f.nad = 1;
            f.e_begin = 0;
            f.e_count = 1;
            f.p_base = 0;
            traverse(c, sc, 0, f);
        }
    }
    if (c.collect) {
        auto t1 = std::chrono::steady_clock::now();
        std::vector<LeafSeg*> segs;
        for (auto& g : c.segs) segs.push_back(g.get());
        run_classes(c, segs);
        c.segs.clear();
        c.seconds_eri += std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count();
    }
    for (int i = 0; i < count; ++i) {
        const long nn = (long)sys[i].T->n * sys[i].T->n;
        for (int j = 0; j < ndens; ++j)
            fx_launch_finalize(sys[i].slots + (long)j * c.nslot * nn, c.nslot, nn, o.alpha, o.beta, sys[i].K[j], st);
    }
    FX_HIP(hipGetLastError());
    struct EvGuard {
        ExCtx& c;
        ~EvGuard() {
            for (auto& t : c.timed) {
                (void)hipEventDestroy(t.a);
                (void)hipEventDestroy(t.b);
            }
        }
    } evguard{c};
    std::vector<unsigned long long> cnt(81 * 2 * 3);
    FX_HIP(hipMemcpyAsync(cnt.data(), c.counters, sizeof(unsigned long long) * cnt.size(), hipMemcpyDeviceToHost, st));
    FX_HIP(hipStreamSynchronize(st));
    if (stats) {
        for (int cls = 0; cls < 81; ++cls)
            for (int pr = 0; pr < 2; ++pr) {
                const unsigned long long q = cnt[(cls * 2 + pr) * 3], pq = cnt[(cls * 2 + pr) * 3 + 1];
                const unsigned long long qm = cnt[(cls * 2 + pr) * 3 + 2];
                stats->class_quartets[cls] += (int64_t)q;
                stats->quartets += (int64_t)q;
                stats->quartets_covered += (int64_t)(q + qm);
                if (pr) stats->quartets_fp32 += (int64_t)q;
                stats->prim_quartets += (double)pq;
                const double fl = (double)pq * fx_class_vrr_flops[cls] + (double)q * fx_class_hrr_flops[cls];
                stats->flops += fl;
                stats->class_flops[cls * 2 + pr] = fl;
                stats->class_prec_quartets[cls * 2 + pr] = (int64_t)q;
            }
        for (auto& t : c.timed) {
            float ms = 0.f;
            FX_HIP(hipEventElapsedTime(&ms, t.a, t.b));
            stats->class_seconds[t.idx] += 1e-3 * ms;
            stats->class_launches[t.idx] += 1;
        }
        stats->seconds_eri = c.seconds_eri;
        stats->seconds_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        stats->seconds_traversal = stats->seconds_total - c.seconds_eri;
    }
}

static void exchange_impl(const fx_tree* T, const double* P, double tau, double* K, const fx_exchange_opts* opts,
                          fx_stats* stats, hipStream_t st) {
    exchange_many(&T, &P, &K, 1, 1, tau, opts, stats, st);
}

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

fx_status fx_exchange_ex(const fx_tree* tree, const double* P, double tau, double* K, const fx_exchange_opts* opts,
                         fx_stats* stats, void* stream) {
    return fx_guard([&] { exchange_impl(tree, P, tau, K, opts, stats, (hipStream_t)stream); });
}

fx_status fx_exchange(const fx_tree* tree, const double* P, double tau, double* K, void* stream) {
    return fx_exchange_ex(tree, P, tau, K, nullptr, nullptr, stream);
}

fx_status fx_exchange_batched(const fx_tree* const* trees, const double* const* P, double* const* K, int32_t count,
                              double tau, const fx_exchange_opts* opts, fx_stats* stats, void* stream) {
    return fx_guard([&] {
        if (count < 0 || (count > 0 && (!trees || !P || !K))) fx_fail(FX_ERR_INVALID_ARG, "bad batch arrays");
        exchange_many(trees, P, K, count, 1, tau, opts, stats, (hipStream_t)stream);
    });
}

fx_status fx_exchange_multi(const fx_tree* tree, const double* const* P, double* const* K, int32_t ndens, double tau,
                            const fx_exchange_opts* opts, fx_stats* stats, void* stream) {
    return fx_guard([&] {
        if (!P || !K) fx_fail(FX_ERR_INVALID_ARG, "P and K must be arrays of ndens device pointers");
        exchange_many(&tree, P, K, 1, ndens, tau, opts, stats, (hipStream_t)stream);
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
            exchange_impl(tree, P, tau, K, opts, nullptr, st);
        } catch (...) {
            g_recording = nullptr;
            delete rec;
            throw;
        }
        g_recording = nullptr;
        *out = rec;
    });
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
        fx_launch_mlp_predict(m->dW, m->dnorm, f, n, y, st);
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
