// Device-side building blocks shared by the generated shell-quartet class
// kernels: the Boys function, shell references, and the work-unit loop that
// screens, compacts and evaluates the quartets of one exchange K block.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fx_internal.h"

#define FX_TWO_PI_POW_2_5 34.98683665524972497   // 2 pi^{5/2}

// loop over the densities contracted with every quartet (NDENS, a template
// parameter of the quartet routines and kernels)
#define FX_FOR_DENS _Pragma("unroll") for (int _d = 0; _d < NDENS; ++_d)

// compile-time flag of the staged routines: store (false) or add (true)
template <bool B>
struct FxAcc {
    static constexpr bool value = B;
};

struct FxShellRef {
    double x, y, z;
    int nprim, pofs, idx;
};

__device__ __forceinline__ FxShellRef fx_shell(const FxDevBasis& B, int s) {
    FxShellRef r;
    r.x = B.xyz[3 * s];
    r.y = B.xyz[3 * s + 1];
    r.z = B.xyz[3 * s + 2];
    r.nprim = B.nprim[s];
    r.pofs = B.pofs[s];
    r.idx = s;
    return r;
}

// ---------------------------------------------------------------------------
// Boys function F_m(T), m = 0..M, FP64.
//   T < FX_BOYS_TMAX: 6th-order Taylor expansion of F_M about the nearest
//   tabulated point T_i = i/32 (dF_m/dT = -F_{m+1}), then the downward
//   recursion F_m = (2T F_{m+1} + e^{-T}) / (2m+1).
//   T >= FX_BOYS_TMAX (60): F_0 = (1/2) sqrt(pi/T) (erf(sqrt T) = 1 to FP64)
//   and the upward recursion F_{m+1} = ((2m+1) F_m - e^{-T}) / (2T), in which
//   e^{-T} is negligible.
// The table (F_j(T_i) and e^{-T_i}) is built on the host.
// ---------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ void fx_boys(double T, const double* __restrict__ tab, double* F) {
    if (T < FX_BOYS_TMAX) {
        const int i = (int)(T * FX_BOYS_INV_DT + 0.5);
        const double dt = (double)i * FX_BOYS_DT - T;   // T_i - T, |dt| <= 1/64
        const double* row = tab + i * FX_BOYS_NCOL;
        const double* r = row + M;
        double f = r[6] * (dt * (1.0 / 6.0));
        f = (r[5] + f) * (dt * (1.0 / 5.0));
        f = (r[4] + f) * (dt * (1.0 / 4.0));
        f = (r[3] + f) * (dt * (1.0 / 3.0));
        f = (r[2] + f) * (dt * 0.5);
        f = (r[1] + f) * dt;
        F[M] = r[0] + f;
        if (M > 0) {
            // e^{-T} = e^{-T_i} e^{dt}, e^{dt} by its Taylor series to dt^7
            double x = 1.0 + dt * (1.0 / 7.0);
            x = 1.0 + dt * (1.0 / 6.0) * x;
            x = 1.0 + dt * (1.0 / 5.0) * x;
            x = 1.0 + dt * (1.0 / 4.0) * x;
            x = 1.0 + dt * (1.0 / 3.0) * x;
            x = 1.0 + dt * 0.5 * x;
            x = 1.0 + dt * x;
            const double eT = row[FX_BOYS_NCOL - 1] * x, T2 = 2.0 * T;
#pragma unroll
            for (int m = M - 1; m >= 0; --m) F[m] = (T2 * F[m + 1] + eT) * (1.0 / (2 * m + 1));
        }
    } else {
        // e^{-T} < 1e-26 is below FP64 resolution of every F_m (m <= 8) here
        const double oT = 1.0 / T;
        F[0] = 0.88622692545275801365 * sqrt(oT);   // sqrt(pi)/2 / sqrt(T)
#pragma unroll
        for (int m = 0; m < M; ++m) F[m + 1] = (2 * m + 1) * F[m] * (0.5 * oT);
    }
}

// ---------------------------------------------------------------------------
// wave-level helpers (wave64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int fx_lane() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ void fx_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int fx_wave_max(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        int o = __shfl_xor(v, off, 64);
        v = v > o ? v : o;
    }
    return v;
}

// all-reduce sum; every lane obtains bitwise the same value (each butterfly
// step adds the same two operands on both partner lanes)
__device__ __forceinline__ double fx_wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int fx_mbcnt(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

constexpr int fx_ncart(int l) { return (l + 1) * (l + 2) / 2; }

// 8 x uint16 VRR descriptor: dst, a0, a1, b0 | b1, c1, k, e
__device__ __forceinline__ uint4 fx_unpack_lo(const uint16_t* p) {
    const ushort4 v = *(const ushort4*)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint4 fx_unpack_hi(const uint16_t* p) {
    const ushort4 v = *(const ushort4*)(p + 4);
    return make_uint4(v.x, v.y, v.z, v.w);
}

// Per-component normalisation factors sqrt((2l-1)!!/((2i-1)!!(2j-1)!!(2k-1)!!)),
// lexicographic Cartesian order; only d has factors other than 1.
__device__ __forceinline__ double fx_comp_factor(int l, int k) {
    if (l < 2) return 1.0;
    return (k == 1 || k == 2 || k == 4) ? 1.7320508075688772935 : 1.0;
}

// ---------------------------------------------------------------------------
// Work-unit loop of one class kernel.
//
// A unit is a K block (a, d) inside a surviving leaf item (A, D) of the
// hextree traversal; its candidate quartets are (a, b, c, d) with (B, C) in
// the item's surviving list, b in B and c in C of the class's angular
// momenta.  The shell-level metric query of Eq. (8) decides each candidate;
// survivors are compacted by wave ballot into an LDS queue in a fixed order
// and evaluated 64 at a time, one per lane.  Each lane accumulates its
// quartets' contributions to K_ad in FP64 registers; the 64 partial blocks
// are reduced by a fixed butterfly, so the block is a deterministic function
// of the unit, whatever order units are scheduled in.  The block is added
// once into the system's K accumulator: no atomics.
// ---------------------------------------------------------------------------
//
// DUAL (mixed precision in one pass): each candidate is screened once and
// queued for the FP64 routine `fn` (beta >= thr) or the FP32 routine `fn2`
// (beta < thr); both accumulate into the same FP64 K block.
// Candidate queue of one wave in LDS: a fill step screens up to G groups of
// 64 entries (G per kernel, from the generator's table; more groups overlap
// more gathers but cost registers) and adds their survivors to a queue
// holding at most 63; a batch takes 64 from its front.
constexpr int FX_FILL_GROUPS = 3;   // default G
template <int G>
constexpr int fx_qcap() { return 64 * (G + 1); }

template <int LA, int LB, int LC, int LD, bool COOP, int WAVES, int NDENS, bool DUAL, int G, typename Fn, typename Fn2>
__device__ __forceinline__ void fx_class_unit(const FxClassArgs& A, Fn fn, Fn2 fn2, long slot_unit, int wave,
                                              int2 (*queue)[fx_qcap<G>()], int2 (*queue2)[fx_qcap<G>()],
                                              double* b32s) {
    static_assert(!COOP || NDENS == 1, "the one-quartet-per-wave form contracts one density");
    static_assert(!COOP || !DUAL, "the one-quartet-per-wave form runs one precision");
    constexpr int NA = fx_ncart(LA), ND = fx_ncart(LD);
    constexpr int NK = COOP ? 1 : NA * ND;   // K elements held per lane and density
    const int lane = fx_lane();
    const long ulo = A.ulh[0];
    const int ur = __builtin_amdgcn_readfirstlane(A.order ? A.order[slot_unit] : (int)slot_unit);
    const long u = ulo + ur;
    const int sid = A.unit_sys ? __builtin_amdgcn_readfirstlane(A.unit_sys[u]) : -1;
    const FxSys Sy = sid >= 0 ? A.sys[sid] : A.one;
    const int sym = __builtin_amdgcn_readfirstlane(Sy.cnt->sym);
    const uint64_t t_start = A.times ? wall_clock64() : 0;
    const int item = __builtin_amdgcn_readfirstlane(A.units[3 * u]);
    const int a = __builtin_amdgcn_readfirstlane(A.units[3 * u + 1]);
    const int d = __builtin_amdgcn_readfirstlane(A.units[3 * u + 2]);
    const FxDevBasis& Bs = Sy.basis;
    const int S = Bs.nshell;
    const FxShellRef ra = fx_shell(Bs, a), rd = fx_shell(Bs, d);
    const double* __restrict__ Qa = Bs.Qn + (long)a * S;
    const double* __restrict__ Qd = Bs.Qn + (long)d * S;
    const double* __restrict__ Sa = Bs.Sm + (long)a * S;
    const double* __restrict__ Sd = Bs.Sm + (long)d * S;
    const double tau = A.tau, thr = A.thr, tau_ovlp = A.tau_ovlp;
    const bool ovlp = tau_ovlp > 0.0 && !A.block;
    const int mode = A.mode;
    double kacc[NDENS * NK];
#pragma unroll
    for (int i = 0; i < NDENS * NK; ++i) kacc[i] = 0.0;

    const long e0 = Sy.bc_off[item], e1 = Sy.bc_off[item + 1];
    int qn = 0, qn2 = 0;                  // queued candidates (FP64 or only queue; FP32 queue)
    long nq = 0, npq = 0, nq2 = 0, npq2 = 0;
    auto evaluate = [&](int2 q, auto& f, long& np) {
        const FxShellRef rb = fx_shell(Bs, q.x), rc = fx_shell(Bs, q.y);
        if (!COOP || lane == 0) np += (long)(ra.nprim * rb.nprim) * (rc.nprim * rd.nprim);
        const long pofs = (long)Bs.f0[q.x] * Sy.n + Bs.f0[q.y];
        const double* Pq[NDENS];
#pragma unroll
        for (int i = 0; i < NDENS; ++i) Pq[i] = Sy.P[i] + pofs;
        f(ra, rb, rc, rd, Bs, A.boys, Pq, Sy.n, kacc, wave);
    };
    // 0: culled; 1: first queue; 2: second queue (DUAL, beta < thr)
    // statistics calls: sum of beta over the FP32 quartets (a-priori error bound),
    // gathered in the wave's LDS slot so that it holds no register
    if (A.beta32 && lane == 0) b32s[wave] = 0.0;
    auto test = [&](int b, int c) -> int {
        const double beta = (Qa[b] * Qd[c]) * Sy.Pn[(long)b * S + c];
        // leaf_screen BLOCK: every quartet of a surviving leaf task is computed
        if (!(beta > tau) && !A.block) return 0;
        // overlap criterion of Eqs. (3)-(4): a pair of shells whose functions
        // all overlap less than tau_ovlp contributes nothing
        if (ovlp && !(Sa[b] >= tau_ovlp && Sd[c] >= tau_ovlp)) return 0;
        if (DUAL || mode == FX_MODE_MIXED_LO) {
            if (beta < thr) {
                if (A.beta32) atomicAdd(&b32s[wave], beta);
                return DUAL ? 2 : 1;
            }
            return DUAL ? 1 : 0;
        }
        if (mode == FX_MODE_MIXED_HI) return beta < thr ? 0 : 1;
        return 1;
    };
    // a stored screen outcome (0 culled, 1 beta >= thr, 2 beta < thr) as `test` returns it
    auto category = [&](int cat) -> int {
        if (cat == 0) return 0;
        if (DUAL) return cat;
        if (mode == FX_MODE_MIXED_HI) return cat == 1 ? 1 : 0;
        if (mode == FX_MODE_MIXED_LO) return cat == 2 ? 1 : 0;
        return 1;
    };
    auto push = [&](int cat, int b, int c) {
        const uint64_t m = __ballot(cat == 1);
        if (cat == 1) queue[wave][qn + fx_mbcnt(m)] = make_int2(b, c);
        qn += __popcll(m);
        if (DUAL) {
            const uint64_t m2 = __ballot(cat == 2);
            if (cat == 2) queue2[wave][qn2 + fx_mbcnt(m2)] = make_int2(b, c);
            qn2 += __popcll(m2);
        }
    };
    // Candidate cursor: single-shell leaves read the item's (lb, lc) segment
    // (leaf index == shell index); leaves with at most one shell per l map
    // (B, C) straight to (b, c), one candidate per entry; other leaves
    // enumerate b in B, c in C.
    const bool seg = Sy.cls_off != nullptr;
    const int* __restrict__ one = Bs.leaf_one;
    long cur = seg ? Sy.cls_off[(long)item * 10 + LB * 3 + LC] : e0;
    const long cend = seg ? Sy.cls_off[(long)item * 10 + LB * 3 + LC + 1] : e1;
    int kc = 0, maxc = 0, nb = 0, nc = 0, ob = 0, oc = 0, jb = 0, jc = 0;
    while (true) {
        // fill: screen candidates until a full batch is queued or none are left
        while (qn < 64 && qn2 < 64) {
            if (seg) {
                if (cur >= cend) break;
                const long e = cur + lane;
                int ok = 0;
                int b = 0, c = 0;
                if (e < cend) {
                    const int2 bc = Sy.bc[e];
                    b = bc.x;
                    c = bc.y;
                    ok = test(b, c);
                }
                push(ok, b, c);
                cur += 64;
            } else if (one) {
                // G groups of 64 entries per step: their gathers
                // overlap; pushed in entry order
                if (cur >= cend) break;
                int2 bcg[G];
                int bg[G], cg[G], okg[G];
                uint32_t mw[G];
                const uint32_t* __restrict__ msk = Sy.mask;
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    bcg[g] = make_int2(0, 0);
                    mw[g] = 0;
                    if (cur + 64 * g + lane < cend) {
                        bcg[g] = Sy.bc[cur + 64 * g + lane];
                        if (msk) mw[g] = msk[cur + 64 * g + lane];
                    }
                }
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    bg[g] = cg[g] = -1;
                    if (cur + 64 * g + lane < cend) {
                        bg[g] = one[bcg[g].x * 3 + LB];
                        cg[g] = one[bcg[g].y * 3 + LC];
                    }
                }
                if (msk) {
                    // the group's screen (same test, taken once for the nine (l_b, l_c))
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const int cat = (int)((mw[g] >> (2 * (3 * LB + LC))) & 3u);
                        okg[g] = (bg[g] >= 0 && cg[g] >= 0) ? category(cat) : 0;
                    }
                } else {
#pragma unroll
                    for (int g = 0; g < G; ++g) okg[g] = (bg[g] >= 0 && cg[g] >= 0) ? test(bg[g], cg[g]) : 0;
                }
#pragma unroll
                for (int g = 0; g < G; ++g) push(okg[g], bg[g], cg[g]);
                cur += 64 * G;
            } else {
                if (kc >= maxc) {
                    if (cur >= cend) break;
                    const long e = cur + lane;
                    nb = nc = ob = oc = 0;
                    if (e < cend) {
                        const int2 bc = Sy.bc[e];
                        ob = Bs.leaf_lofs[bc.x * 4 + LB];
                        nb = Bs.leaf_lofs[bc.x * 4 + LB + 1] - ob;
                        oc = Bs.leaf_lofs[bc.y * 4 + LC];
                        nc = Bs.leaf_lofs[bc.y * 4 + LC + 1] - oc;
                    }
                    maxc = fx_wave_max(nb * nc);
                    kc = jb = jc = 0;
                    cur += 64;
                    continue;
                }
                int ok = 0;
                int b = 0, c = 0;
                if (kc < nb * nc) {
                    // candidate kc = jb * nc + jc of this lane's (B, C) entry
                    b = Bs.leaf_lsh[ob + jb];
                    c = Bs.leaf_lsh[oc + jc];
                    ok = test(b, c);
                }
                push(ok, b, c);
                ++kc;
                if (++jc == nc) {
                    jc = 0;
                    ++jb;
                }
            }
        }
        fx_wave_sync();
        if (qn == 0 && qn2 == 0) break;
        // neither queue full: the candidates are exhausted, drain both
        const bool drain = qn < 64 && qn2 < 64;
        // evaluate one batch of a queue (the only call sites of the routines)
        auto batch = [&](int2 (*qq)[fx_qcap<G>()], int& n, auto& f, long& cnt, long& np) {
            const int nbatch = n < 64 ? n : 64;
            if (COOP) {
                // the whole wave evaluates the queued quartets one after another
                for (int i = 0; i < nbatch; ++i) evaluate(qq[wave][i], f, np);
            } else {
                const int2 q = qq[wave][lane];
                if (lane < nbatch) evaluate(q, f, np);
            }
            cnt += nbatch;
            fx_wave_sync();
            // move the rest (at most 64 G - 1) to the front; lane i reads
            // slots 64 (k + 1) + i and writes slots 64 k + i, so no lane
            // overwrites a slot another lane still has to read
            int2 t[G];
#pragma unroll
            for (int k = 0; k < G; ++k) t[k] = qq[wave][64 * (k + 1) + lane];
#pragma unroll
            for (int k = 0; k < G; ++k) qq[wave][64 * k + lane] = t[k];
            n -= nbatch;
            fx_wave_sync();
        };
        if (qn >= 64 || (drain && qn > 0)) batch(queue, qn, fn, nq, npq);
        if (DUAL && (qn2 >= 64 || (drain && qn2 > 0))) batch(queue2, qn2, fn2, nq2, npq2);
    }
    // deterministic reduction of the 64 lane partials, then one write per element
    const long rowbase = (long)Bs.f0[a] * Sy.n + Bs.f0[d];
    double outv[NDENS];
#pragma unroll
    for (int j = 0; j < NDENS; ++j) outv[j] = 0.0;
    if (COOP) {
        // lane t already owns element t of the block
        outv[0] = kacc[0] * (fx_comp_factor(LA, lane / ND) * fx_comp_factor(LD, lane % ND));
    } else {
#pragma unroll
        for (int j = 0; j < NDENS; ++j)
#pragma unroll
            for (int i = 0; i < NK; ++i) {
                const double s = fx_wave_sum(kacc[j * NK + i]);
                if (lane == i) outv[j] = s * (fx_comp_factor(LA, i / ND) * fx_comp_factor(LD, i % ND));
            }
    }
#pragma unroll
    for (int j = 0; j < NDENS; ++j) {
        // K_ad += this class's block.  Class launches of one system run one
        // after another on one stream and a launch has one unit per block, so
        // each element has one writer at a time and the additions follow the
        // launch order: no atomics, the same K for any schedule.
        double* kout = Sy.acc[j];
        if (lane < NA * ND) kout[rowbase + (long)(lane / ND) * Sy.n + (lane % ND)] += outv[j];
        // symmetric densities: K_da = K_ad^T, and unit (d, a) does not exist
        if (sym && a != d && lane < NA * ND)
            kout[(long)(Bs.f0[d] + lane % ND) * Sy.n + Bs.f0[a] + lane / ND] += outv[j];
    }
    if (A.times && lane == 0) A.times[ur] = (float)(wall_clock64() - t_start);
    auto count = [&](unsigned long long* ctr, long q, long npl) {
        long np = npl;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) np += __shfl_xor(np, off, 64);
        if (lane == 0) {
            atomicAdd(ctr, (unsigned long long)q);
            atomicAdd(ctr + 1, (unsigned long long)np);
            if (sym && a != d) atomicAdd(ctr + 2, (unsigned long long)q);
        }
    };
    if (A.counters) count(A.counters, nq, npq);
    if (DUAL && A.counters2) count(A.counters2, nq2, npq2);
    if (A.beta32 && (DUAL || mode == FX_MODE_MIXED_LO)) {
        fx_wave_sync();
        if (lane == 0 && b32s[wave] != 0.0) atomicAdd(A.beta32, b32s[wave]);
    }
}

// Kernel-level unit loop: one unit per wave, with an optional XCD-aware remap
// of workgroups (fx_xcd_remap) so that neighbouring units -- which share
// density and pair data -- run on one XCD and its L2.  K does not depend on
// the mapping.
template <int LA, int LB, int LC, int LD, bool COOP, int WAVES, int NDENS, bool DUAL = false,
          int G = FX_FILL_GROUPS, typename Fn, typename Fn2>
__device__ __forceinline__ void fx_class_body(const FxClassArgs& A, Fn fn, Fn2 fn2) {
    __shared__ int2 queue[WAVES][fx_qcap<G>()];
    __shared__ int2 queue2[DUAL ? WAVES : 1][fx_qcap<G>()];
    __shared__ double b32s[WAVES];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    long blk = blockIdx.x;
    if (A.flags & FX_LAUNCH_XCD) blk = fx_xcd_remap(blk, gridDim.x);
    const long slot_unit = blk * WAVES + wave;
    if (slot_unit >= __builtin_amdgcn_readfirstlane((int)(A.ulh[1] - A.ulh[0]))) return;
    fx_class_unit<LA, LB, LC, LD, COOP, WAVES, NDENS, DUAL, G>(A, fn, fn2, slot_unit, wave, queue, queue2, b32s);
}

// Thread variant: one quartet per lane.
// FX_THREAD_MIN_WAVES_f64 / _f32 (set per class by the generator): the least
// number of waves per SIMD the register allocation must allow.  Above 1 it
// trades register spills for latency hiding in kernels that spill anyway.
#ifndef FX_THREAD_MIN_WAVES_f64
#define FX_THREAD_MIN_WAVES_f64 1
#endif
#ifndef FX_THREAD_MIN_WAVES_f32
#define FX_THREAD_MIN_WAVES_f32 1
#endif
// FX_FILL_GROUPS_f64 / _f32 / _mix (set per class by the generator): entry
// groups per fill step of the candidate scan.
#ifndef FX_FILL_GROUPS_f64
#define FX_FILL_GROUPS_f64 FX_FILL_GROUPS
#endif
#ifndef FX_FILL_GROUPS_f32
#define FX_FILL_GROUPS_f32 FX_FILL_GROUPS
#endif
#ifndef FX_FILL_GROUPS_mix
#define FX_FILL_GROUPS_mix FX_FILL_GROUPS
#endif
// Instantiated for one and for two densities (FxClassArgs::ndens).
#define FX_THREAD_KERNEL(la, lb, lc, ld, cls, prec)                                                     \
    template <int NDENS>                                                                                 \
    __global__ __launch_bounds__(64 * FX_CLASS_WAVES, FX_THREAD_MIN_WAVES_##prec) void                  \
        fx_k_##cls##_##prec(FxClassArgs A) {                                                            \
        auto f = [](const FxShellRef& ra, const FxShellRef& rb, const FxShellRef& rc, const FxShellRef& rd, \
                    const FxDevBasis& B, const double* bt, const double* const* P, long n, double* k, int) { \
            eri_##cls##_##prec<NDENS>(ra, rb, rc, rd, B, bt, P, n, k);                                   \
        };                                                                                               \
        fx_class_body<la, lb, lc, ld, false, FX_CLASS_WAVES, NDENS, false, FX_FILL_GROUPS_##prec>(A, f, f); \
    }

// Mixed precision in one pass: each candidate screened once, evaluated by the
// FP64 or the FP32 routine by its bound (one density).
#ifndef FX_THREAD_MIN_WAVES_mix
#define FX_THREAD_MIN_WAVES_mix 1
#endif
#define FX_DUAL_KERNEL(la, lb, lc, ld, cls)                                                             \
    __global__ __launch_bounds__(64 * FX_CLASS_WAVES, FX_THREAD_MIN_WAVES_mix) void                     \
        fx_k_##cls##_mix(FxClassArgs A) {                                                               \
        auto f64 = [](const FxShellRef& ra, const FxShellRef& rb, const FxShellRef& rc, const FxShellRef& rd, \
                      const FxDevBasis& B, const double* bt, const double* const* P, long n, double* k, int) { \
            eri_##cls##_f64<1>(ra, rb, rc, rd, B, bt, P, n, k);                                          \
        };                                                                                               \
        auto f32 = [](const FxShellRef& ra, const FxShellRef& rb, const FxShellRef& rc, const FxShellRef& rd, \
                      const FxDevBasis& B, const double* bt, const double* const* P, long n, double* k, int) { \
            eri_##cls##_f32<1>(ra, rb, rc, rd, B, bt, P, n, k);                                          \
        };                                                                                               \
        fx_class_body<la, lb, lc, ld, false, FX_CLASS_WAVES, 1, true, FX_FILL_GROUPS_mix>(A, f64, f32);  \
    }
#define FX_LAUNCH_DUAL(cls)                                                                             \
    hipLaunchKernelGGL(fx_k_##cls##_mix, dim3((A.nbound + FX_CLASS_WAVES - 1) / FX_CLASS_WAVES),         \
                       dim3(64 * FX_CLASS_WAVES), 0, st, A)

// Cooperative variant: one quartet per wave, intermediates in LDS.
#define FX_COOP_KERNEL(la, lb, lc, ld, cls, prec, real)                                                 \
    __global__ __launch_bounds__(64 * FX_COOP_WAVES) void fx_kc_##cls##_##prec(FxClassArgs A) {        \
        __shared__ real lds[FX_COOP_WAVES * coop_##cls##_##prec::NSLOT];                                 \
        auto f = [&](const FxShellRef& ra, const FxShellRef& rb, const FxShellRef& rc, const FxShellRef& rd, \
                     const FxDevBasis& B, const double* bt, const double* const* P, long n, double* k, int w) { \
            eri_##cls##_##prec##_coop(ra, rb, rc, rd, B, bt, P[0], n, lds + w * coop_##cls##_##prec::NSLOT,  \
                                      k[0]);                                                             \
        };                                                                                               \
        fx_class_body<la, lb, lc, ld, true, FX_COOP_WAVES, 1>(A, f, f);                                  \
    }

#define FX_LAUNCH_THREAD(cls, prec)                                                                     \
    do {                                                                                                 \
        const dim3 g((A.nbound + FX_CLASS_WAVES - 1) / FX_CLASS_WAVES), b(64 * FX_CLASS_WAVES);          \
        if (A.ndens == 2)                                                                                \
            hipLaunchKernelGGL(fx_k_##cls##_##prec<2>, g, b, 0, st, A);                                  \
        else                                                                                             \
            hipLaunchKernelGGL(fx_k_##cls##_##prec<1>, g, b, 0, st, A);                                  \
    } while (0)
#define FX_LAUNCH_COOP(cls, prec)                                                                       \
    hipLaunchKernelGGL(fx_kc_##cls##_##prec,                                                            \
                       dim3((A.nbound + FX_COOP_WAVES - 1) / FX_COOP_WAVES),           \
                       dim3(64 * FX_COOP_WAVES), 0, st, A)

// Both variants; `variant` 0 = thread, 1 = cooperative.
#define FX_DEFINE_CLASS_KERNELS_BOTH(la, lb, lc, ld, cls)                                               \
    FX_THREAD_KERNEL(la, lb, lc, ld, cls, f64)                                                          \
    FX_THREAD_KERNEL(la, lb, lc, ld, cls, f32)                                                          \
    FX_DUAL_KERNEL(la, lb, lc, ld, cls)                                                                 \
    FX_COOP_KERNEL(la, lb, lc, ld, cls, f64, double)                                                    \
    FX_COOP_KERNEL(la, lb, lc, ld, cls, f32, float)                                                     \
    int fx_launch_##cls(int prec32, int variant, FxClassArgs A, hipStream_t st) {                        \
        if (A.mode == FX_MODE_DUAL) {                                                                    \
            FX_LAUNCH_DUAL(cls);                                                                         \
            return 2;                                                                                    \
        }                                                                                                \
        if (variant == 1 && A.ndens == 1) {                                                              \
            if (prec32) FX_LAUNCH_COOP(cls, f32); else FX_LAUNCH_COOP(cls, f64);                         \
            return 1;                                                                                    \
        }                                                                                                \
        if (prec32) FX_LAUNCH_THREAD(cls, f32); else FX_LAUNCH_THREAD(cls, f64);                         \
        return 0;                                                                                        \
    }

#define FX_DEFINE_CLASS_KERNELS_THREAD(la, lb, lc, ld, cls)                                             \
    FX_THREAD_KERNEL(la, lb, lc, ld, cls, f64)                                                          \
    FX_THREAD_KERNEL(la, lb, lc, ld, cls, f32)                                                          \
    FX_DUAL_KERNEL(la, lb, lc, ld, cls)                                                                 \
    int fx_launch_##cls(int prec32, int, FxClassArgs A, hipStream_t st) {                                \
        if (A.mode == FX_MODE_DUAL) {                                                                    \
            FX_LAUNCH_DUAL(cls);                                                                         \
            return 2;                                                                                    \
        }                                                                                                \
        if (prec32) FX_LAUNCH_THREAD(cls, f32); else FX_LAUNCH_THREAD(cls, f64);                         \
        return 0;                                                                                        \
    }

#define FX_DEFINE_CLASS_KERNELS_COOP(la, lb, lc, ld, cls)                                               \
    FX_COOP_KERNEL(la, lb, lc, ld, cls, f64, double)                                                    \
    FX_COOP_KERNEL(la, lb, lc, ld, cls, f32, float)                                                     \
    int fx_launch_##cls(int prec32, int, FxClassArgs A, hipStream_t st) {                                \
        if (prec32) FX_LAUNCH_COOP(cls, f32); else FX_LAUNCH_COOP(cls, f64);                             \
        return 1;                                                                                        \
    }

// Schwarz factors: one thread per unordered shell pair (a <= b) of the pair
// type (la, lb); Qn[a][b] = Qn[b][a] = sqrt(sum max(0, (mu nu|mu nu))).
#define FX_SCHWARZ_CASE(la, lb, cls)                                                                    \
    case (la * 3 + lb): s2 = eri_diag_##cls##_f64(r0, r1, B, boys); break;

#define FX_DEFINE_SCHWARZ_KERNEL()                                                                      \
    __global__ __launch_bounds__(256) void fx_k_schwarz(FxDevBasis B, const double* boys, const int2* pairs, \
                                                        long npairs, double* Qn) {                       \
        const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;                                     \
        if (i >= npairs) return;                                                                         \
        const int a = pairs[i].x, b = pairs[i].y;                                                        \
        const FxShellRef r0 = fx_shell(B, a), r1 = fx_shell(B, b);                                       \
        double s2 = 0.0;                                                                                 \
        switch (B.l[a] * 3 + B.l[b]) {                                                                   \
            FX_SCHWARZ_CASE(0, 0, ssss) FX_SCHWARZ_CASE(0, 1, spsp) FX_SCHWARZ_CASE(0, 2, sdsd)          \
            FX_SCHWARZ_CASE(1, 0, psps) FX_SCHWARZ_CASE(1, 1, pppp) FX_SCHWARZ_CASE(1, 2, pdpd)          \
            FX_SCHWARZ_CASE(2, 0, dsds) FX_SCHWARZ_CASE(2, 1, dpdp) FX_SCHWARZ_CASE(2, 2, dddd)          \
        }                                                                                                \
        const double v = sqrt(s2);                                                                       \
        Qn[(long)a * B.nshell + b] = v;                                                                  \
        Qn[(long)b * B.nshell + a] = v;                                                                  \
    }                                                                                                    \
    void fx_launch_schwarz(FxDevBasis B, const double* boys, const int2* pairs, long npairs, double* Qn, \
                           hipStream_t st) {                                                             \
        if (npairs > 0)                                                                                  \
            hipLaunchKernelGGL(fx_k_schwarz, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, st, B, \
                               boys, pairs, npairs, Qn);                                                 \
    }
