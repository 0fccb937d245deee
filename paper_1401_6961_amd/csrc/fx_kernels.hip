// Support kernels of the exchange build: density norms, block-norm
// quadtrees, the level-synchronous hextree traversal with deterministic
// scan-based compaction, K-block work units, and the final reduction.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fx_internal.h"
#include "fx_kernels.h"

// ---------------------------------------------------------------------------
// Shell-level density norms (Eq. 8): Pn[b][c] = max(||P_bc||_F, ||P_cb||_F)
// with each Frobenius norm summed row-major over its block, every product
// and sum rounded separately (no fused multiply-add), so the value is a
// fixed function of P.  b, c are tree-order shells; P is in caller order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double fx_block_frob(const double* __restrict__ P, long n, int r0, int nr, int c0,
                                                int nc) {
    double s = 0.0;
    for (int i = 0; i < nr; ++i) {
        const double* row = P + (long)(r0 + i) * n + c0;
        for (int j = 0; j < nc; ++j) s = __dadd_rn(s, __dmul_rn(row[j], row[j]));
    }
    return __dsqrt_rn(s);
}

__global__ void fx_k_pnorm(const double* __restrict__ P, long n, const int* __restrict__ l,
                           const int* __restrict__ f0, int S, double* __restrict__ Pn) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (c >= S || c < b) return;
    const int nb = (l[b] + 1) * (l[b] + 2) / 2, nc = (l[c] + 1) * (l[c] + 2) / 2;
    const double x = fx_block_frob(P, n, f0[b], nb, f0[c], nc);
    const double y = fx_block_frob(P, n, f0[c], nc, f0[b], nb);
    const double v = x > y ? x : y;
    Pn[(long)b * S + c] = v;
    Pn[(long)c * S + b] = v;
}

void fx_launch_pnorm(const double* P, long n, const int* l, const int* f0, int S, double* Pn, hipStream_t st) {
    dim3 grid((S + 255) / 256, S);
    hipLaunchKernelGGL(fx_k_pnorm, grid, dim3(256), 0, st, P, n, l, f0, S, Pn);
}

// ---------------------------------------------------------------------------
// Primitive-pair records for every ordered pair of primitives (global
// indices i, j): p = a_i + a_j, 1/p, P = (a_i X + a_j Y)/p and
// K = c_i c_j exp(-a_i a_j / p |X - Y|^2).
// ---------------------------------------------------------------------------
__global__ void fx_k_prim_pairs(const double* __restrict__ exps, const double* __restrict__ coefs,
                                const int* __restrict__ prim_shell, const double* __restrict__ xyz, long Nt,
                                FxPrimPair* __restrict__ out) {
    const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long i = blockIdx.y;
    if (j >= Nt) return;
    const int x = prim_shell[i], y = prim_shell[j];
    const double ai = exps[i], aj = exps[j];
    const double p = ai + aj, op = 1.0 / p;
    const double X0 = xyz[3 * x], X1 = xyz[3 * x + 1], X2 = xyz[3 * x + 2];
    const double Y0 = xyz[3 * y], Y1 = xyz[3 * y + 1], Y2 = xyz[3 * y + 2];
    const double d0 = X0 - Y0, d1 = X1 - Y1, d2 = X2 - Y2;
    FxPrimPair r;
    r.p = p;
    r.op = op;
    r.Px = (ai * X0 + aj * Y0) * op;
    r.Py = (ai * X1 + aj * Y1) * op;
    r.Pz = (ai * X2 + aj * Y2) * op;
    r.K = coefs[i] * coefs[j] * exp(-ai * aj * op * (d0 * d0 + d1 * d1 + d2 * d2));
    out[i * Nt + j] = r;
}

void fx_launch_prim_pairs(const double* exps, const double* coefs, const int* prim_shell, const double* xyz, long Nt,
                          FxPrimPair* out, hipStream_t st) {
    dim3 grid((unsigned)((Nt + 255) / 256), (unsigned)Nt);
    hipLaunchKernelGGL(fx_k_prim_pairs, grid, dim3(256), 0, st, exps, coefs, prim_shell, xyz, Nt, out);
}

// ---------------------------------------------------------------------------
// Squared block norms at the leaf level: X[A][B] = sum_{a in A, b in B} x_ab^2
// (shell ranges of leaf nodes are contiguous in tree order).
// ---------------------------------------------------------------------------
__global__ void fx_k_leaf_sq(const double* __restrict__ x, int S, const int* __restrict__ sL,
                             const int* __restrict__ sR, int nleaf, double* __restrict__ out) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    const int A = blockIdx.y;
    if (B >= nleaf) return;
    double s = 0.0;
    for (int a = sL[A]; a < sR[A]; ++a)
        for (int b = sL[B]; b < sR[B]; ++b) {
            const double v = x[(long)a * S + b];
            s += v * v;
        }
    out[(long)A * nleaf + B] = s;
}

void fx_launch_leaf_sq(const double* x, int S, const int* sL, const int* sR, int nleaf, double* out,
                       hipStream_t st) {
    dim3 grid((nleaf + 255) / 256, nleaf);
    hipLaunchKernelGGL(fx_k_leaf_sq, grid, dim3(256), 0, st, x, S, sL, sR, nleaf, out);
}

// Parent level from child level: X_k[A][B] = sum over children pairs.
__global__ void fx_k_level_up(const double* __restrict__ child, int nchild_nodes, const int* __restrict__ ch0,
                              const int* __restrict__ nch, int nk, double* __restrict__ out) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    const int A = blockIdx.y;
    if (B >= nk) return;
    double s = 0.0;
    for (int i = 0; i < nch[A]; ++i)
        for (int j = 0; j < nch[B]; ++j) s += child[(long)(ch0[A] + i) * nchild_nodes + (ch0[B] + j)];
    out[(long)A * nk + B] = s;
}

void fx_launch_level_up(const double* child, int nchild_nodes, const int* ch0, const int* nch, int nk, double* out,
                        hipStream_t st) {
    dim3 grid((nk + 255) / 256, nk);
    hipLaunchKernelGGL(fx_k_level_up, grid, dim3(256), 0, st, child, nchild_nodes, ch0, nch, nk, out);
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan (deterministic, three phases).
// in[i] (uint8 counts or uint32) -> out[i] = sum_{j<i}, out[n] = total.
// ---------------------------------------------------------------------------
#define SCAN_BLOCK 256
#define SCAN_ITEMS 16
#define SCAN_TILE (SCAN_BLOCK * SCAN_ITEMS)

__device__ __forceinline__ long fx_block_exclusive(long v, long* total) {
    // wave inclusive scan
    __shared__ long wsum[SCAN_BLOCK / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    long x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        long y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    long base = 0, tot = 0;
    for (int i = 0; i < SCAN_BLOCK / 64; ++i) {
        if (i < w) base += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

template <typename T, bool POPC>
__device__ __forceinline__ long fx_scan_load(const T* in, long i, long n) {
    if (i >= n) return 0;
    if (POPC) return __popc((unsigned)in[i]);
    return (long)in[i];
}

template <typename T, bool POPC>
__global__ void fx_k_scan_reduce(const T* __restrict__ in, long n, long* __restrict__ partial) {
    const long base = (long)blockIdx.x * SCAN_TILE;
    long s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) s += fx_scan_load<T, POPC>(in, base + (long)k * SCAN_BLOCK + threadIdx.x, n);
    long tot;
    fx_block_exclusive(s, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ void fx_k_scan_partials(long* __restrict__ partial, long nblk, long* __restrict__ total_out,
                                   long* __restrict__ out_end) {
    // single workgroup: exclusive scan of the per-tile sums in place
    long carry = 0;
    for (long base = 0; base < nblk; base += SCAN_BLOCK) {
        const long i = base + threadIdx.x;
        const long v = i < nblk ? partial[i] : 0;
        long tot;
        const long ex = fx_block_exclusive(v, &tot);
        if (i < nblk) partial[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *total_out = carry;
        *out_end = carry;
    }
}

template <typename T, bool POPC, typename O>
__global__ void fx_k_scan_write(const T* __restrict__ in, long n, const long* __restrict__ partial,
                                O* __restrict__ out) {
    const long base = (long)blockIdx.x * SCAN_TILE;
    // each thread owns SCAN_ITEMS consecutive elements
    const long my = base + (long)threadIdx.x * SCAN_ITEMS;
    long vals[SCAN_ITEMS];
    long s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        vals[k] = fx_scan_load<T, POPC>(in, my + k, n);
        s += vals[k];
    }
    long tot;
    long ex = fx_block_exclusive(s, &tot) + partial[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (my + k < n) out[my + k] = (O)ex;
        ex += vals[k];
    }
}

// out must hold n + 1 values; out[n] receives the total.
template <typename T, bool POPC, typename O>
static void fx_scan_impl(const T* in, long n, O* out, long* partial, long* total_dev, hipStream_t st) {
    const long nblk = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nblk > 0) hipLaunchKernelGGL((fx_k_scan_reduce<T, POPC>), dim3(nblk), dim3(SCAN_BLOCK), 0, st, in, n, partial);
    hipLaunchKernelGGL(fx_k_scan_partials, dim3(1), dim3(SCAN_BLOCK), 0, st, partial, nblk, total_dev, out + n);
    if (nblk > 0)
        hipLaunchKernelGGL((fx_k_scan_write<T, POPC, O>), dim3(nblk), dim3(SCAN_BLOCK), 0, st, in, n, partial, out);
}

long fx_scan_tiles(long n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

void fx_scan_popc_u8(const uint8_t* in, long n, long* out, long* partial, long* total_dev, hipStream_t st) {
    fx_scan_impl<uint8_t, true, long>(in, n, out, partial, total_dev, st);
}
void fx_scan_i32(const int* in, long n, long* out, long* partial, long* total_dev, hipStream_t st) {
    fx_scan_impl<int, false, long>(in, n, out, partial, total_dev, st);
}

// ---------------------------------------------------------------------------
// Hextree traversal, one level (Eqs. 7a-d with the metric query of Eq. 8).
//
// The frontier at level k is a list of K-side node pairs (A, D) ("ADs"),
// each owning a contiguous list of density-side pairs (B, C).  A task
// (A,B,C,D) has children (A_i, B_j, C_k, D_l), one child per non-leaf index
// choice (leaf nodes are carried unchanged, so 1..16 children).  A child
// survives iff  (Qsq_{A_i B_j} Qsq_{C_k D_l}) Psq_{B_j C_k} (1 + 1e-12) > tau^2
// with squared Frobenius block norms at level k+1.  Each norm bounds every
// contained shell-level norm, so no quartet with beta > tau is lost; the
// margin absorbs rounding.  Output order: child AD (parent AD, i, l) major,
// then (parent entry, j, k), which is deterministic.  With a symmetric
// density (L.sym) only children with A_i <= D_l are kept: nodes of a level
// are ordered by their shell ranges, so this keeps exactly the K blocks on
// and above the diagonal (in tree order), and K_DA is the transpose of K_AD.
// ---------------------------------------------------------------------------

__device__ __forceinline__ long fx_seg_index(const FxLevelArgs& L, int p, int il, long e) {
    const long o0 = L.bc_off[p] - L.e_begin, len = L.bc_off[p + 1] - L.bc_off[p];
    return 4 * o0 + il * len + (e - L.bc_off[p]);
}

__global__ void fx_k_expand_mask(FxLevelArgs L, uint8_t* __restrict__ mask) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= L.e_count * 4) return;
    const long e = L.e_begin + (t >> 2);
    const int il = (int)(t & 3);
    const int p = L.bc_parent[e] - L.p_base;
    const int2 ad = L.ad[p];
    const int2 bc = L.bc[e];
    const int i = il >> 1, l = il & 1;
    uint8_t m = 0;
    if (i < L.nch[ad.x] && l < L.nch[ad.y] && (!L.sym || L.ch0[ad.x] + i <= L.ch0[ad.y] + l)) {
        const int Ai = L.ch0[ad.x] + i, Dl = L.ch0[ad.y] + l;
        const int nB = L.nch[bc.x], nC = L.nch[bc.y];
        for (int j = 0; j < nB; ++j) {
            const int Bj = L.ch0[bc.x] + j;
            const double qab = L.Qsq[(long)Ai * L.nk1 + Bj];
            for (int k = 0; k < nC; ++k) {
                const int Ck = L.ch0[bc.y] + k;
                const double b2 = (qab * L.Qsq[(long)Ck * L.nk1 + Dl]) * L.Psq[(long)Bj * L.nk1 + Ck];
                if (b2 * (1.0 + 1e-12) > L.tau2) m |= (uint8_t)(1u << (j * 2 + k));
            }
        }
    }
    mask[fx_seg_index(L, p, il, e)] = m;
}

void fx_launch_expand_mask(const FxLevelArgs& L, uint8_t* mask, hipStream_t st) {
    const long n = L.e_count * 4;
    if (n > 0) hipLaunchKernelGGL(fx_k_expand_mask, dim3((n + 255) / 256), dim3(256), 0, st, L, mask);
}

// One thread per (parent AD, child il): does the child own any entries?
__global__ void fx_k_expand_adflag(FxLevelArgs L, const long* __restrict__ pos, int* __restrict__ flag) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (long)L.nad * 4) return;
    const int p = (int)(t >> 2), il = (int)(t & 3);
    const long len = L.bc_off[p + 1] - L.bc_off[p];
    const long s = 4 * (L.bc_off[p] - L.e_begin) + il * len;
    flag[t] = (len > 0 && pos[s + len] - pos[s] > 0) ? 1 : 0;
}

void fx_launch_expand_adflag(const FxLevelArgs& L, const long* pos, int* flag, hipStream_t st) {
    const long n = (long)L.nad * 4;
    if (n > 0) hipLaunchKernelGGL(fx_k_expand_adflag, dim3((n + 255) / 256), dim3(256), 0, st, L, pos, flag);
}

__global__ void fx_k_expand_adwrite(FxLevelArgs L, const long* __restrict__ pos, const int* __restrict__ flag,
                                    const long* __restrict__ adpos, int2* __restrict__ ad_next,
                                    long* __restrict__ bc_off_next, long total_entries, long total_ads) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) bc_off_next[total_ads] = total_entries;
    if (t >= (long)L.nad * 4 || !flag[t]) return;
    const int p = (int)(t >> 2), il = (int)(t & 3);
    const long len = L.bc_off[p + 1] - L.bc_off[p];
    const long s = 4 * (L.bc_off[p] - L.e_begin) + il * len;
    const int2 ad = L.ad[p];
    const long q = adpos[t];
    ad_next[q] = make_int2(L.ch0[ad.x] + (il >> 1), L.ch0[ad.y] + (il & 1));
    bc_off_next[q] = pos[s];
}

void fx_launch_expand_adwrite(const FxLevelArgs& L, const long* pos, const int* flag, const long* adpos, int2* ad_next,
                              long* bc_off_next, long total_entries, long total_ads, hipStream_t st) {
    const long n = (long)L.nad * 4;
    hipLaunchKernelGGL(fx_k_expand_adwrite, dim3(n > 0 ? (n + 255) / 256 : 1), dim3(256), 0, st, L, pos, flag, adpos,
                       ad_next, bc_off_next, total_entries, total_ads);
}

__global__ void fx_k_expand_write(FxLevelArgs L, const uint8_t* __restrict__ mask, const long* __restrict__ pos,
                                  const long* __restrict__ adpos, int2* __restrict__ bc_next,
                                  int* __restrict__ parent_next) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= L.e_count * 4) return;
    const long e = L.e_begin + (t >> 2);
    const int il = (int)(t & 3);
    const int p = L.bc_parent[e] - L.p_base;
    const long idx = fx_seg_index(L, p, il, e);
    unsigned m = mask[idx];
    if (!m) return;
    const int2 bc = L.bc[e];
    long o = pos[idx];
    const int child = (int)adpos[(long)p * 4 + il];
    for (int jk = 0; jk < 4; ++jk)
        if (m & (1u << jk)) {
            bc_next[o] = make_int2(L.ch0[bc.x] + (jk >> 1), L.ch0[bc.y] + (jk & 1));
            if (parent_next) parent_next[o] = child;
            ++o;
        }
}

void fx_launch_expand_write(const FxLevelArgs& L, const uint8_t* mask, const long* pos, const long* adpos,
                            int2* bc_next, int* parent_next, hipStream_t st) {
    const long n = L.e_count * 4;
    if (n > 0)
        hipLaunchKernelGGL(fx_k_expand_write, dim3((n + 255) / 256), dim3(256), 0, st, L, mask, pos, adpos, bc_next,
                           parent_next);
}

// ---------------------------------------------------------------------------
// K-block work units.  For every leaf item (A, D) and every (la, ld): the
// shells a in A with l = la and d in D with l = ld.  Units are laid out per
// (la, ld) list in item order, then a, then d.
// ---------------------------------------------------------------------------
// On a diagonal item (A == A) of a symmetric build only the pairs a <= d.
__device__ __forceinline__ int fx_unit_pairs(const int* __restrict__ leaf_lsh, int oa, int na, int od, int nd,
                                             bool diag) {
    if (!diag) return na * nd;
    int c = 0;
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nd; ++j) c += leaf_lsh[oa + i] <= leaf_lsh[od + j];
    return c;
}

__global__ void fx_k_unit_count(const int2* __restrict__ items, long nitems, const int* __restrict__ leaf_lofs,
                                const int* __restrict__ leaf_lsh, int sym, int* __restrict__ cnt) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nitems) return;
    const int2 ad = items[p];
    const bool diag = sym && ad.x == ad.y;
    for (int la = 0; la < 3; ++la)
        for (int ld = 0; ld < 3; ++ld) {
            const int oa = leaf_lofs[ad.x * 4 + la], na = leaf_lofs[ad.x * 4 + la + 1] - oa;
            const int od = leaf_lofs[ad.y * 4 + ld], nd = leaf_lofs[ad.y * 4 + ld + 1] - od;
            cnt[(long)(la * 3 + ld) * nitems + p] = fx_unit_pairs(leaf_lsh, oa, na, od, nd, diag);
        }
}

void fx_launch_unit_count(const int2* items, long nitems, const int* leaf_lofs, const int* leaf_lsh, int sym, int* cnt,
                          hipStream_t st) {
    if (nitems > 0)
        hipLaunchKernelGGL(fx_k_unit_count, dim3((nitems + 255) / 256), dim3(256), 0, st, items, nitems, leaf_lofs,
                           leaf_lsh, sym, cnt);
}

__global__ void fx_k_unit_write(const int2* __restrict__ items, long nitems, long item_base,
                                const int* __restrict__ leaf_lofs, const int* __restrict__ leaf_lsh, int sym,
                                const long* __restrict__ upos, int* __restrict__ units) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nitems * 9) return;
    const int cls = (int)(t / nitems);
    const long p = t - (long)cls * nitems;
    const int la = cls / 3, ld = cls % 3;
    const int2 ad = items[p];
    const bool diag = sym && ad.x == ad.y;
    const int oa = leaf_lofs[ad.x * 4 + la], na = leaf_lofs[ad.x * 4 + la + 1] - oa;
    const int od = leaf_lofs[ad.y * 4 + ld], nd = leaf_lofs[ad.y * 4 + ld + 1] - od;
    long o = upos[t];
    for (int i = 0; i < na; ++i)
        for (int j = 0; j < nd; ++j) {
            if (diag && leaf_lsh[oa + i] > leaf_lsh[od + j]) continue;
            units[3 * o] = (int)(item_base + p);
            units[3 * o + 1] = leaf_lsh[oa + i];
            units[3 * o + 2] = leaf_lsh[od + j];
            ++o;
        }
}

void fx_launch_unit_write(const int2* items, long nitems, long item_base, const int* leaf_lofs, const int* leaf_lsh,
                          int sym, const long* upos, int* units, hipStream_t st) {
    const long n = nitems * 9;
    if (n > 0)
        hipLaunchKernelGGL(fx_k_unit_write, dim3((n + 255) / 256), dim3(256), 0, st, items, nitems, item_base, leaf_lofs,
                           leaf_lsh, sym, upos, units);
}

// a[i] = max(a[i], b[i])
__global__ void fx_k_max_inplace(double* __restrict__ a, const double* __restrict__ b, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = fmax(a[i], b[i]);
}

void fx_launch_max_inplace(double* a, const double* b, long n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(fx_k_max_inplace, dim3((n + 255) / 256), dim3(256), 0, st, a, b, n);
}

// ---------------------------------------------------------------------------
// Bitwise symmetry test of P: 32x32 tiles (bi <= bj) and their mirror tiles
// staged through LDS, so both reads are coalesced.  Any mismatch (NaN
// included) sets *flag = 1; every writer stores the same value.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void fx_k_psym(const double* __restrict__ P, long n, int* __restrict__ flag) {
    __shared__ double t1[32][33], t2[32][33];
    const long bi = blockIdx.y, bj = blockIdx.x;
    if (bi > bj) return;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const long i = bi * 32 + r, j = bj * 32 + tx;
        t1[r][tx] = (i < n && j < n) ? P[i * n + j] : 0.0;
        const long i2 = bj * 32 + r, j2 = bi * 32 + tx;
        t2[r][tx] = (i2 < n && j2 < n) ? P[i2 * n + j2] : 0.0;
    }
    __syncthreads();
    bool bad = false;
    for (int r = ty; r < 32; r += 8) bad |= !(t1[r][tx] == t2[tx][r]);
    if (bad) *flag = 1;
}

void fx_launch_psym(const double* P, long n, int* flag, hipStream_t st) {
    const long nb = (n + 31) / 32;
    if (nb > 0) hipLaunchKernelGGL(fx_k_psym, dim3(nb, nb), dim3(256), 0, st, P, n, flag);
}

// ---------------------------------------------------------------------------
// Leaves that are single shells: group every K-block item's (B, C) entries by
// density-side class (l_b, l_c), stably, one wave per item; cls_off[p*10+k]
// is the first entry of class k = l_b*3 + l_c, cls_off[p*10+9] the end.
// ---------------------------------------------------------------------------
__global__ void fx_k_class_sort(const long* __restrict__ bc_off, const int2* __restrict__ bc, long nitems,
                                const int* __restrict__ l, int2* __restrict__ out, long* __restrict__ cls_off) {
    const long p = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= nitems) return;
    const long e0 = bc_off[p], e1 = bc_off[p + 1];
    long base[9];
    for (int c = 0; c < 9; ++c) base[c] = 0;
    for (long e = e0; e < e1; e += 64) {
        const long i = e + lane;
        int k = -1;
        if (i < e1) {
            const int2 x = bc[i];
            k = l[x.x] * 3 + l[x.y];
        }
        for (int c = 0; c < 9; ++c) base[c] += __popcll(__ballot(k == c));
    }
    long run = e0;
    for (int c = 0; c < 9; ++c) {
        const long n = base[c];
        if (lane == 0) cls_off[p * 10 + c] = run;
        base[c] = run;
        run += n;
    }
    if (lane == 0) cls_off[p * 10 + 9] = e1;
    for (long e = e0; e < e1; e += 64) {
        const long i = e + lane;
        int k = -1;
        int2 x = make_int2(0, 0);
        if (i < e1) {
            x = bc[i];
            k = l[x.x] * 3 + l[x.y];
        }
        for (int c = 0; c < 9; ++c) {
            const uint64_t m = __ballot(k == c);
            if (k == c) {
                const int r = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                out[base[c] + r] = x;
            }
            base[c] += __popcll(m);
        }
    }
}

void fx_launch_class_sort(const long* bc_off, const int2* bc, long nitems, const int* l, int2* out, long* cls_off,
                          hipStream_t st) {
    if (nitems > 0)
        hipLaunchKernelGGL(fx_k_class_sort, dim3((nitems + 3) / 4), dim3(256), 0, st, bc_off, bc, nitems, l, out,
                           cls_off);
}

// ---------------------------------------------------------------------------
// Fill and final reduction: K = alpha * sum_s slot_s + beta * K, slots summed
// in index order (deterministic).
// ---------------------------------------------------------------------------
__global__ void fx_k_fill(double* __restrict__ x, long n, double v) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long k = i; k < n; k += stride) x[k] = v;
}

template <typename T>
__global__ void fx_k_fill_t(T* __restrict__ x, long n, T v) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long k = i; k < n; k += stride) x[k] = v;
}

void fx_launch_fill_i32(int* x, long n, int v, hipStream_t st) {
    if (n <= 0) return;
    long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fx_k_fill_t<int>, dim3(blocks), dim3(256), 0, st, x, n, v);
}

void fx_launch_fill_u32(unsigned int* x, long n, unsigned int v, hipStream_t st) {
    if (n <= 0) return;
    long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fx_k_fill_t<unsigned int>, dim3(blocks), dim3(256), 0, st, x, n, v);
}

void fx_launch_fill(double* x, long n, double v, hipStream_t st) {
    if (n <= 0) return;
    long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fx_k_fill, dim3(blocks), dim3(256), 0, st, x, n, v);
}

__global__ void fx_k_finalize(const double* __restrict__ slots, int nslot, long nn, double alpha, double beta,
                              double* __restrict__ K) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long k = i; k < nn; k += stride) {
        double s = 0.0;
        for (int q = 0; q < nslot; ++q) s += slots[(long)q * nn + k];
        K[k] = beta == 0.0 ? alpha * s : alpha * s + beta * K[k];
    }
}

void fx_launch_finalize(const double* slots, int nslot, long nn, double alpha, double beta, double* K,
                        hipStream_t st) {
    long blocks = (nn + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(fx_k_finalize, dim3(blocks), dim3(256), 0, st, slots, nslot, nn, alpha, beta, K);
}
