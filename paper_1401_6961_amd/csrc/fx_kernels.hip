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
    if (c >= S) return;
    for (int b = blockIdx.y; b <= c; b += gridDim.y) {
        const int nb = (l[b] + 1) * (l[b] + 2) / 2, nc = (l[c] + 1) * (l[c] + 2) / 2;
        const double x = fx_block_frob(P, n, f0[b], nb, f0[c], nc);
        const double y = fx_block_frob(P, n, f0[c], nc, f0[b], nb);
        const double v = x > y ? x : y;
        Pn[(long)b * S + c] = v;
        Pn[(long)c * S + b] = v;
    }
}

// gridDim.y is at most 65535: kernels with a row index in y loop over rows
static unsigned fx_grid_y(long rows) { return (unsigned)(rows < 1 ? 1 : (rows > 65535 ? 65535 : rows)); }

void fx_launch_pnorm(const double* P, long n, const int* l, const int* f0, int S, double* Pn, hipStream_t st) {
    dim3 grid((S + 255) / 256, fx_grid_y(S));
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
    if (j >= Nt) return;
    for (long i = blockIdx.y; i < Nt; i += gridDim.y) {
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
}

void fx_launch_prim_pairs(const double* exps, const double* coefs, const int* prim_shell, const double* xyz, long Nt,
                          FxPrimPair* out, hipStream_t st) {
    dim3 grid((unsigned)((Nt + 255) / 256), fx_grid_y(Nt));
    hipLaunchKernelGGL(fx_k_prim_pairs, grid, dim3(256), 0, st, exps, coefs, prim_shell, xyz, Nt, out);
}

// ---------------------------------------------------------------------------
// Squared block norms at the leaf level: X[A][B] = sum_{a in A, b in B} x_ab^2
// (shell ranges of leaf nodes are contiguous in tree order).
// ---------------------------------------------------------------------------
__global__ void fx_k_leaf_sq(const double* __restrict__ x, int S, const int* __restrict__ sL,
                             const int* __restrict__ sR, int nleaf, double* __restrict__ out) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= nleaf) return;
    for (int A = blockIdx.y; A < nleaf; A += gridDim.y) {
        double s = 0.0;
        for (int a = sL[A]; a < sR[A]; ++a)
            for (int b = sL[B]; b < sR[B]; ++b) {
                const double v = x[(long)a * S + b];
                s += v * v;
            }
        out[(long)A * nleaf + B] = s;
    }
}

void fx_launch_leaf_sq(const double* x, int S, const int* sL, const int* sR, int nleaf, double* out,
                       hipStream_t st) {
    dim3 grid((nleaf + 255) / 256, fx_grid_y(nleaf));
    hipLaunchKernelGGL(fx_k_leaf_sq, grid, dim3(256), 0, st, x, S, sL, sR, nleaf, out);
}

// Block maxima (overlap criterion): X[A][B] = max_{a in A, b in B} x_ab.
__global__ void fx_k_leaf_max(const double* __restrict__ x, int S, const int* __restrict__ sL,
                              const int* __restrict__ sR, int nleaf, double* __restrict__ out) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= nleaf) return;
    for (int A = blockIdx.y; A < nleaf; A += gridDim.y) {
        double m = 0.0;
        for (int a = sL[A]; a < sR[A]; ++a)
            for (int b = sL[B]; b < sR[B]; ++b) m = fmax(m, x[(long)a * S + b]);
        out[(long)A * nleaf + B] = m;
    }
}

void fx_launch_leaf_max(const double* x, int S, const int* sL, const int* sR, int nleaf, double* out,
                        hipStream_t st) {
    dim3 grid((nleaf + 255) / 256, fx_grid_y(nleaf));
    hipLaunchKernelGGL(fx_k_leaf_max, grid, dim3(256), 0, st, x, S, sL, sR, nleaf, out);
}

__global__ void fx_k_level_max(const double* __restrict__ child, int nchild_nodes, const int* __restrict__ ch0,
                               const int* __restrict__ nch, int nk, double* __restrict__ out) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= nk) return;
    for (int A = blockIdx.y; A < nk; A += gridDim.y) {
        double m = 0.0;
        for (int i = 0; i < nch[A]; ++i)
            for (int j = 0; j < nch[B]; ++j) m = fmax(m, child[(long)(ch0[A] + i) * nchild_nodes + (ch0[B] + j)]);
        out[(long)A * nk + B] = m;
    }
}

void fx_launch_level_max(const double* child, int nchild_nodes, const int* ch0, const int* nch, int nk, double* out,
                         hipStream_t st) {
    dim3 grid((nk + 255) / 256, fx_grid_y(nk));
    hipLaunchKernelGGL(fx_k_level_max, grid, dim3(256), 0, st, child, nchild_nodes, ch0, nch, nk, out);
}

// Overlaps of shell pairs (Obara-Saika): for a primitive pair with record
// (p, P, K = c_i c_j exp(-a_i a_j / p |AB|^2)), the one-dimensional
// overlaps s_{i,j} of (x - A)^i (x - B)^j e^{-p (x - P)^2}, relative to
// sqrt(pi/p), satisfy s_00 = 1, s_{i+1,j} = PA s_{i,j} + (i s_{i-1,j} +
// j s_{i,j-1}) / 2p and s_{0,j+1} = PB s_{0,j} + j s_{0,j-1} / 2p; a
// component pair adds K (pi/p)^{3/2} s^x s^y s^z.  Components carry the
// normalisation factors of the Cartesian d components.  One thread per
// shell pair a <= b; Sm is mirrored.
__device__ __forceinline__ void fx_os_overlap_1d(double PA, double PB, double o2p, int la, int lb, double s[3][3]) {
    s[0][0] = 1.0;
    for (int j = 1; j <= lb; ++j) s[0][j] = PB * s[0][j - 1] + (j > 1 ? (j - 1) * o2p * s[0][j - 2] : 0.0);
    for (int i = 1; i <= la; ++i)
        for (int j = 0; j <= lb; ++j)
            s[i][j] = PA * s[i - 1][j] + o2p * ((i > 1 ? (i - 1) * s[i - 2][j] : 0.0) + (j > 0 ? j * s[i - 1][j - 1] : 0.0));
}

__device__ __forceinline__ void fx_cart_exp(int l, int k, int* e) {
    // lexicographic: x^l first (p: x, y, z; d: xx, xy, xz, yy, yz, zz)
    int n = 0;
    for (int i = l; i >= 0; --i)
        for (int j = l - i; j >= 0; --j) {
            if (n == k) {
                e[0] = i;
                e[1] = j;
                e[2] = l - i - j;
                return;
            }
            ++n;
        }
}

__device__ __forceinline__ double fx_comp_norm(int l, int k) {
    if (l < 2) return 1.0;
    return (k == 1 || k == 2 || k == 4) ? 1.7320508075688772935 : 1.0;   // sqrt(3) for xy, xz, yz
}

__global__ __launch_bounds__(256) void fx_k_overlap_max(FxDevBasis B, const int2* __restrict__ pairs, long npairs,
                                                        double* __restrict__ Sm) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npairs) return;
    const int a = pairs[t].x, b = pairs[t].y;
    const int la = B.l[a], lb = B.l[b];
    const int na = (la + 1) * (la + 2) / 2, nb = (lb + 1) * (lb + 2) / 2;
    double blk[36];
    for (int k = 0; k < 36; ++k) blk[k] = 0.0;
    const double Ax = B.xyz[3 * a], Ay = B.xyz[3 * a + 1], Az = B.xyz[3 * a + 2];
    const double Bx = B.xyz[3 * b], By = B.xyz[3 * b + 1], Bz = B.xyz[3 * b + 2];
    for (int i = 0; i < B.nprim[a]; ++i)
        for (int j = 0; j < B.nprim[b]; ++j) {
            const FxPrimPair r = B.pp[(long)(B.pofs[a] + i) * B.ntprim + B.pofs[b] + j];
            double sx[3][3], sy[3][3], sz[3][3];
            const double o2p = 0.5 * r.op;
            fx_os_overlap_1d(r.Px - Ax, r.Px - Bx, o2p, la, lb, sx);
            fx_os_overlap_1d(r.Py - Ay, r.Py - By, o2p, la, lb, sy);
            fx_os_overlap_1d(r.Pz - Az, r.Pz - Bz, o2p, la, lb, sz);
            const double pre = r.K * 5.568327996831707845 * r.op * sqrt(r.op);   // K (pi/p)^{3/2}
            for (int u = 0; u < na; ++u) {
                int eu[3];
                fx_cart_exp(la, u, eu);
                for (int v = 0; v < nb; ++v) {
                    int ev[3];
                    fx_cart_exp(lb, v, ev);
                    blk[u * nb + v] += pre * sx[eu[0]][ev[0]] * sy[eu[1]][ev[1]] * sz[eu[2]][ev[2]];
                }
            }
        }
    double m = 0.0;
    for (int u = 0; u < na; ++u)
        for (int v = 0; v < nb; ++v) m = fmax(m, fabs(blk[u * nb + v]) * (fx_comp_norm(la, u) * fx_comp_norm(lb, v)));
    Sm[(long)a * B.nshell + b] = m;
    Sm[(long)b * B.nshell + a] = m;
}

void fx_launch_overlap_max(FxDevBasis B, const int2* pairs, long npairs, double* Sm, hipStream_t st) {
    if (npairs > 0)
        hipLaunchKernelGGL(fx_k_overlap_max, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, st, B, pairs,
                           npairs, Sm);
}

// Parent level from child level: X_k[A][B] = sum over children pairs.
__global__ void fx_k_level_up(const double* __restrict__ child, int nchild_nodes, const int* __restrict__ ch0,
                              const int* __restrict__ nch, int nk, double* __restrict__ out) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    if (B >= nk) return;
    for (int A = blockIdx.y; A < nk; A += gridDim.y) {
        double s = 0.0;
        for (int i = 0; i < nch[A]; ++i)
            for (int j = 0; j < nch[B]; ++j) s += child[(long)(ch0[A] + i) * nchild_nodes + (ch0[B] + j)];
        out[(long)A * nk + B] = s;
    }
}

void fx_launch_level_up(const double* child, int nchild_nodes, const int* ch0, const int* nch, int nk, double* out,
                        hipStream_t st) {
    dim3 grid((nk + 255) / 256, fx_grid_y(nk));
    hipLaunchKernelGGL(fx_k_level_up, grid, dim3(256), 0, st, child, nchild_nodes, ch0, nch, nk, out);
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan (deterministic, three phases), with the element
// count read from device memory: n = mult * (*n_dev), or the host count when
// n_dev is null.  out[i] = sum_{j<i} in[j], out[n] = total, *total = total.
// The reduce and write phases loop over tiles with a fixed grid, so the
// launch shape never depends on device data.
// ---------------------------------------------------------------------------
#define SCAN_BLOCK 256
#define SCAN_ITEMS 16
#define SCAN_TILE (SCAN_BLOCK * SCAN_ITEMS)
#define FX_GRID_MAX 8192

__device__ __forceinline__ long fx_block_exclusive(long v, long* total) {
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

__device__ __forceinline__ long fx_dev_n(const long* n_dev, int mult, long n_host) {
    return n_dev ? (long)mult * *n_dev : n_host;
}

template <typename T, bool POPC>
__global__ __launch_bounds__(SCAN_BLOCK) void fx_k_scan_reduce(const T* __restrict__ in, const long* n_dev, int mult,
                                                               long n_host, long* __restrict__ partial) {
    const long n = fx_dev_n(n_dev, mult, n_host);
    const long ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long base = tile * SCAN_TILE;
        long s = 0;
        for (int k = 0; k < SCAN_ITEMS; ++k)
            s += fx_scan_load<T, POPC>(in, base + (long)k * SCAN_BLOCK + threadIdx.x, n);
        long tot;
        fx_block_exclusive(s, &tot);
        if (threadIdx.x == 0) partial[tile] = tot;
    }
}

template <typename O>
__global__ __launch_bounds__(SCAN_BLOCK) void fx_k_scan_partials(long* __restrict__ partial, const long* n_dev,
                                                                 int mult, long n_host, long* __restrict__ total_out,
                                                                 O* __restrict__ out) {
    // single workgroup: exclusive scan of the per-tile sums in place
    const long n = fx_dev_n(n_dev, mult, n_host);
    const long nblk = (n + SCAN_TILE - 1) / SCAN_TILE;
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
        if (total_out) *total_out = carry;
        out[n] = (O)carry;
    }
}

template <typename T, bool POPC, typename O>
__global__ __launch_bounds__(SCAN_BLOCK) void fx_k_scan_write(const T* __restrict__ in, const long* n_dev, int mult,
                                                              long n_host, const long* __restrict__ partial,
                                                              O* __restrict__ out) {
    const long n = fx_dev_n(n_dev, mult, n_host);
    const long ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long base = tile * SCAN_TILE;
        const long my = base + (long)threadIdx.x * SCAN_ITEMS;
        long vals[SCAN_ITEMS];
        long s = 0;
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            vals[k] = fx_scan_load<T, POPC>(in, my + k, n);
            s += vals[k];
        }
        long tot;
        long ex = fx_block_exclusive(s, &tot) + partial[tile];
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            if (my + k < n) out[my + k] = (O)ex;
            ex += vals[k];
        }
    }
}

long fx_scan_tiles(long n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

template <typename T, bool POPC, typename O>
static void fx_scan_impl(const T* in, const long* n_dev, int mult, long n_max, O* out, long* partial, long* total,
                         hipStream_t st) {
    // n_max: the host count (n_dev null) or an upper bound of the device count
    long grid = (n_max + SCAN_TILE - 1) / SCAN_TILE;
    if (grid > FX_GRID_MAX) grid = FX_GRID_MAX;
    if (grid > 0)
        hipLaunchKernelGGL((fx_k_scan_reduce<T, POPC>), dim3(grid), dim3(SCAN_BLOCK), 0, st, in, n_dev, mult, n_max,
                           partial);
    hipLaunchKernelGGL(fx_k_scan_partials<O>, dim3(1), dim3(SCAN_BLOCK), 0, st, partial, n_dev, mult, n_max, total,
                       out);
    if (grid > 0)
        hipLaunchKernelGGL((fx_k_scan_write<T, POPC, O>), dim3(grid), dim3(SCAN_BLOCK), 0, st, in, n_dev, mult, n_max,
                           partial, out);
}

void fx_scan_popc_u8_dev(const uint8_t* in, const long* n_dev, int mult, long n_max, uint32_t* out, long* partial,
                         long* total, hipStream_t st) {
    fx_scan_impl<uint8_t, true, uint32_t>(in, n_dev, mult, n_max, out, partial, total, st);
}
void fx_scan_i32_dev(const int* in, const long* n_dev, int mult, long n_max, long* out, long* partial, long* total,
                     hipStream_t st) {
    fx_scan_impl<int, false, long>(in, n_dev, mult, n_max, out, partial, total, st);
}
void fx_scan_i32(const int* in, long n, long* out, long* partial, long* total_dev, hipStream_t st) {
    fx_scan_impl<int, false, long>(in, nullptr, 1, n, out, partial, total_dev, st);
}

static long fx_grid_for(long n, int block) {
    long g = (n + block - 1) / block;
    if (g > FX_GRID_MAX) g = FX_GRID_MAX;
    return g < 1 ? 1 : g;
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
// density only children with A_i <= D_l are kept: nodes of a level are
// ordered by their shell ranges, so this keeps exactly the K blocks on and
// above the diagonal (in tree order), and K_DA is the transpose of K_AD.
// A traversal chunk keeps only children A_i whose shells meet its row range
// [a_lo, a_hi) of K; chunks partition the K blocks.
//
// Every size is read from FxDevCounts on the device; a level whose entries
// exceed the capacity sets the overflow flag and empties every later level,
// so no kernel ever writes past its buffers.
// ---------------------------------------------------------------------------

__device__ __forceinline__ long fx_seg_index(const FxLevelArgs& L, int p, int il, long e) {
    const long o0 = L.bc_off[p], len = L.bc_off[p + 1] - L.bc_off[p];
    return 4 * o0 + il * len + (e - L.bc_off[p]);
}

__device__ __forceinline__ bool fx_in_chunk(const FxLevelArgs& L, int Ai) {
    return L.sR1[Ai] > L.a_lo && L.sL1[Ai] < L.a_hi;
}

// the chunk that owns a node for the partition sums: the one holding its first shell
__device__ __forceinline__ bool fx_owned(const FxLevelArgs& L, int Ai) {
    return L.sL1[Ai] >= L.a_lo && L.sL1[Ai] < L.a_hi;
}

// Root task (level 0): kept iff its block bound exceeds tau.  The root's
// partition sum (culled, or a leaf when the tree has one level) is counted
// by the chunk that owns shell 0.
__global__ void fx_k_root(FxDevCounts* cnt, const double* Qsq0, const double* Psq0, double tau2, int2* ad, long* bc_off,
                          int2* bc, int* parent, unsigned long long* part, unsigned long long n4, int one_level,
                          int count_root) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double q = Qsq0[0];
    const bool keep = (q * q) * Psq0[0] * (1.0 + 1e-12) > tau2;
    cnt->overflow = 0;
    cnt->need = 0;
    cnt->need_level = 0;
    cnt->nad[0] = keep ? 1 : 0;
    cnt->ne[0] = keep ? 1 : 0;
    ad[0] = make_int2(0, 0);
    bc_off[0] = 0;
    bc_off[1] = keep ? 1 : 0;
    bc[0] = make_int2(0, 0);
    if (parent) parent[0] = 0;
    if (count_root && part) {
        if (!keep) atomicAdd(part + FX_PART_SLOTS, n4);
        else if (one_level) atomicAdd(part, n4);
    }
}

void fx_launch_root(FxDevCounts* cnt, const double* Qsq0, const double* Psq0, double tau2, int2* ad, long* bc_off,
                    int2* bc, int* parent, unsigned long long* part, unsigned long long n4, int one_level,
                    int count_root, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_root, dim3(1), dim3(64), 0, st, cnt, Qsq0, Psq0, tau2, ad, bc_off, bc, parent, part, n4,
                       one_level, count_root);
}

__global__ __launch_bounds__(256) void fx_k_expand_mask(FxLevelArgs L, uint8_t* __restrict__ mask) {
    const long n = 4 * L.cnt->ne[L.k];
    const int sym = L.cnt->sym;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const long e = t >> 2;
        const int il = (int)(t & 3);
        const int p = L.bc_parent[e];
        const int2 ad = L.ad[p];
        const int2 bc = L.bc[e];
        const int i = il >> 1, l = il & 1;
        uint8_t m = 0;
        if (i < L.nch[ad.x] && l < L.nch[ad.y]) {
            const int Ai = L.ch0[ad.x] + i, Dl = L.ch0[ad.y] + l;
            if ((!sym || Ai <= Dl) && fx_in_chunk(L, Ai)) {
                const int nB = L.nch[bc.x], nC = L.nch[bc.y];
                for (int j = 0; j < nB; ++j) {
                    const int Bj = L.ch0[bc.x] + j;
                    const double qab = L.Qsq[(long)Ai * L.nk1 + Bj];
                    // overlap criterion of Eqs. (3)-(4) on the pair blocks (block maxima are exact)
                    const bool bra_ok = L.tau_ovlp <= 0.0 || L.Smx[(long)Ai * L.nk1 + Bj] >= L.tau_ovlp;
                    for (int k = 0; k < nC; ++k) {
                        const int Ck = L.ch0[bc.y] + k;
                        const double b2 = (qab * L.Qsq[(long)Ck * L.nk1 + Dl]) * L.Psq[(long)Bj * L.nk1 + Ck];
                        const bool ket_ok = L.tau_ovlp <= 0.0 || L.Smx[(long)Ck * L.nk1 + Dl] >= L.tau_ovlp;
                        if (b2 * (1.0 + 1e-12) > L.tau2 && bra_ok && ket_ok) m |= (uint8_t)(1u << (j * 2 + k));
                    }
                }
            }
        }
        mask[fx_seg_index(L, p, il, e)] = m;
    }
}

void fx_launch_expand_mask(const FxLevelArgs& L, long n_max, uint8_t* mask, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_expand_mask, dim3(fx_grid_for(4 * n_max, 256)), dim3(256), 0, st, L, mask);
}

// Entries of level k+1: the scan total, unless it exceeds the capacity
// (then the overflow flag is set and this and every later level is empty).
__global__ void fx_k_commit_entries(FxDevCounts* cnt, int k, const long* total, long cap) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const long t = *total;
    if (!cnt->overflow && t > cap) {
        cnt->overflow = 1;
        cnt->need = t;
        cnt->need_level = k + 1;
    }
    cnt->ne[k + 1] = cnt->overflow ? 0 : t;
}

// End of a chunk's traversal: keep its partition sums and level sizes if no
// level overflowed, and record the sizes for the next call's capacities.
__global__ void fx_k_chunk_done(const FxDevCounts* cnt, int nl, const unsigned long long* __restrict__ cpart,
                                unsigned long long* __restrict__ part, FxDevRun* run) {
    const bool ok = !cnt->overflow;
    if (ok && part)
        for (int i = threadIdx.x; i < 3 * FX_PART_SLOTS; i += blockDim.x) part[i] += cpart[i];
    if (threadIdx.x == 0) {
        long ein = 0;
        for (int k = 0; k + 1 < nl; ++k) ein = cnt->ne[k] > ein ? cnt->ne[k] : ein;
        if (ein > run->e_in) run->e_in = ein;
        if (cnt->ne[nl - 1] > run->e_leaf) run->e_leaf = cnt->ne[nl - 1];
        if (!ok) {
            run->overflow = 1;
            run->incomplete = 1;
            long* w = cnt->need_level == nl - 1 ? &run->need_leaf : &run->need_in;
            if (cnt->need > *w) *w = cnt->need;
        } else {
            for (int k = 0; k < nl; ++k) run->frontier[k] += cnt->ne[k];
            run->items += cnt->nad[nl - 1];
        }
    }
}

void fx_launch_chunk_done(const FxDevCounts* cnt, int nl, const unsigned long long* cpart, unsigned long long* part,
                          FxDevRun* run, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_chunk_done, dim3(1), dim3(256), 0, st, cnt, nl, cpart, part, run);
}

__global__ void fx_k_units_done(const FxDevCounts* cnt, FxDevRun* run) {
    if (threadIdx.x == 0 && blockIdx.x == 0) run->units += cnt->ubase[9];
}

void fx_launch_units_done(const FxDevCounts* cnt, FxDevRun* run, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_units_done, dim3(1), dim3(64), 0, st, cnt, run);
}

__global__ void fx_k_commit_ads(FxDevCounts* cnt, int k, const long* total) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    cnt->nad[k + 1] = cnt->overflow ? 0 : *total;
}

void fx_launch_commit_entries(FxDevCounts* cnt, int k, const long* total, long cap, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_commit_entries, dim3(1), dim3(64), 0, st, cnt, k, total, cap);
}
void fx_launch_commit_ads(FxDevCounts* cnt, int k, const long* total, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_commit_ads, dim3(1), dim3(64), 0, st, cnt, k, total);
}

// One thread per (parent AD, child il): does the child own any entries?
__global__ __launch_bounds__(256) void fx_k_expand_adflag(FxLevelArgs L, const uint32_t* __restrict__ pos,
                                                          int* __restrict__ flag) {
    const long n = 4 * L.cnt->nad[L.k];
    const bool dead = L.cnt->overflow != 0;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const int p = (int)(t >> 2), il = (int)(t & 3);
        const long len = L.bc_off[p + 1] - L.bc_off[p];
        const long s = 4 * L.bc_off[p] + il * len;
        flag[t] = (!dead && len > 0 && pos[s + len] - pos[s] > 0) ? 1 : 0;
    }
}

void fx_launch_expand_adflag(const FxLevelArgs& L, long nad_max, const uint32_t* pos, int* flag, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_expand_adflag, dim3(fx_grid_for(4 * nad_max, 256)), dim3(256), 0, st, L, pos, flag);
}

__global__ __launch_bounds__(256) void fx_k_expand_adwrite(FxLevelArgs L, const uint32_t* __restrict__ pos,
                                                           const int* __restrict__ flag,
                                                           const long* __restrict__ adpos, int2* __restrict__ ad_next,
                                                           long* __restrict__ bc_off_next) {
    const long nads = L.cnt->nad[L.k + 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) bc_off_next[nads] = L.cnt->ne[L.k + 1];
    if (L.cnt->overflow) return;
    const long n = 4 * L.cnt->nad[L.k];
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        if (!flag[t]) continue;
        const int p = (int)(t >> 2), il = (int)(t & 3);
        const long len = L.bc_off[p + 1] - L.bc_off[p];
        const long s = 4 * L.bc_off[p] + il * len;
        const int2 ad = L.ad[p];
        const long q = adpos[t];
        ad_next[q] = make_int2(L.ch0[ad.x] + (il >> 1), L.ch0[ad.y] + (il & 1));
        bc_off_next[q] = (long)pos[s];
    }
}

void fx_launch_expand_adwrite(const FxLevelArgs& L, long nad_max, const uint32_t* pos, const int* flag,
                              const long* adpos, int2* ad_next, long* bc_off_next, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_expand_adwrite, dim3(fx_grid_for(4 * nad_max, 256)), dim3(256), 0, st, L, pos, flag, adpos,
                       ad_next, bc_off_next);
}

// Traversal partition: every task (A,B,C,D) of the product of the four
// trees ends in exactly one of three sets -- a surviving leaf task, a culled
// task, or (symmetric form) a task whose mirror (D,C,B,A) is traversed -- so
// the three sums of |A||B||C||D| (function counts) add up to n^4.  One
// thread per (parent entry, child AD) sums the children (i, j, k, l) it owns;
// a workgroup adds its sums into one of FX_PART_SLOTS counter slots (integer
// sums: the totals do not depend on the order of the additions).
__device__ __forceinline__ void fx_partition_sums(const FxLevelArgs& L, int sym, int p, int il, long e, unsigned m,
                                                  unsigned long long* s3) {
    const int2 ad = L.ad[p];
    const int2 bc = L.bc[e];
    const int i = il >> 1, l = il & 1;
    if (i >= L.nch[ad.x] || l >= L.nch[ad.y]) return;
    const int Ai = L.ch0[ad.x] + i, Dl = L.ch0[ad.y] + l;
    if (!fx_owned(L, Ai)) return;
    const unsigned long long fad = (unsigned long long)L.nf1[Ai] * (unsigned long long)L.nf1[Dl];
    const bool mirrored = sym && Ai > Dl;
    for (int j = 0; j < L.nch[bc.x]; ++j)
        for (int k = 0; k < L.nch[bc.y]; ++k) {
            const unsigned long long t =
                fad * ((unsigned long long)L.nf1[L.ch0[bc.x] + j] * (unsigned long long)L.nf1[L.ch0[bc.y] + k]);
            if (mirrored) s3[2] += t;
            else if (m & (1u << (j * 2 + k))) s3[0] += L.leaf_next ? t : 0ull;
            else s3[1] += t;
        }
}

__device__ __forceinline__ void fx_partition_flush(const FxLevelArgs& L, unsigned long long* s3) {
    __shared__ unsigned long long red[3][256 / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        unsigned long long v = s3[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[q][w] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        unsigned long long v = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) v += red[threadIdx.x][k];
        if (v) atomicAdd(L.part + (long)threadIdx.x * FX_PART_SLOTS + (blockIdx.x % FX_PART_SLOTS), v);
    }
}

__global__ __launch_bounds__(256) void fx_k_expand_write(FxLevelArgs L, const uint8_t* __restrict__ mask,
                                                         const uint32_t* __restrict__ pos,
                                                         const long* __restrict__ adpos, int2* __restrict__ bc_next,
                                                         int* __restrict__ parent_next) {
    if (L.cnt->overflow) return;   // uniform: the whole grid returns
    const long n = 4 * L.cnt->ne[L.k];
    const int sym = L.cnt->sym;
    unsigned long long s3[3] = {0ull, 0ull, 0ull};
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
        const long e = t >> 2;
        const int il = (int)(t & 3);
        const int p = L.bc_parent[e];
        const long idx = fx_seg_index(L, p, il, e);
        const unsigned m = mask[idx];
        if (L.part) fx_partition_sums(L, sym, p, il, e, m, s3);
        if (!m) continue;
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
    if (L.part) fx_partition_flush(L, s3);
}

void fx_launch_expand_write(const FxLevelArgs& L, long n_max, const uint8_t* mask, const uint32_t* pos,
                            const long* adpos, int2* bc_next, int* parent_next, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_expand_write, dim3(fx_grid_for(4 * n_max, 256)), dim3(256), 0, st, L, mask, pos, adpos,
                       bc_next, parent_next);
}

// ---------------------------------------------------------------------------
// K-block work units.  For every leaf item (A, D) and every (la, ld): the
// shells a in A with l = la and d in D with l = ld.  Units are laid out per
// (la, ld) list in item order, then a, then d.  Counts are laid out
// [la*3+ld][item] with the item capacity as stride (zero past the items).
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

__global__ __launch_bounds__(256) void fx_k_unit_count(const int2* __restrict__ items, const FxDevCounts* cnt, int lv,
                                                       long cap, const int* __restrict__ leaf_lofs,
                                                       const int* __restrict__ leaf_lsh, int* __restrict__ out) {
    const long nitems = cnt->nad[lv];
    const int sym = cnt->sym;
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < cap; p += (long)gridDim.x * blockDim.x) {
        if (p >= nitems) {
            for (int k = 0; k < 9; ++k) out[(long)k * cap + p] = 0;
            continue;
        }
        const int2 ad = items[p];
        const bool diag = sym && ad.x == ad.y;
        for (int la = 0; la < 3; ++la)
            for (int ld = 0; ld < 3; ++ld) {
                const int oa = leaf_lofs[ad.x * 4 + la], na = leaf_lofs[ad.x * 4 + la + 1] - oa;
                const int od = leaf_lofs[ad.y * 4 + ld], nd = leaf_lofs[ad.y * 4 + ld + 1] - od;
                out[(long)(la * 3 + ld) * cap + p] = fx_unit_pairs(leaf_lsh, oa, na, od, nd, diag);
            }
    }
}

void fx_launch_unit_count(const int2* items, const FxDevCounts* cnt, int lv, long cap, const int* leaf_lofs,
                          const int* leaf_lsh, int* out, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_unit_count, dim3(fx_grid_for(cap, 256)), dim3(256), 0, st, items, cnt, lv, cap, leaf_lofs,
                       leaf_lsh, out);
}

// Screen of one (l_a, l_d) group, for leaves that hold at most one shell of
// each angular momentum: a leaf item (A, D) then has one K-block unit (a, d)
// in the group and each of its (B, C) entries one candidate (b, c) per
// (l_b, l_c).  The nine candidates of an entry are tested here once with the
// shell-level metric query of Eq. (8) (and the overlap criterion of
// Eqs. (3)-(4) when on), in exactly the arithmetic the class kernels use, and
// the outcomes are stored as 2 bits per (l_b, l_c); the group's nine class
// kernels read them instead of gathering the norms again.  The 3x3 block of
// ||P_bc|| an entry needs lies in three rows of the norm table, so this pass
// reads each row segment once for the group.  One wave per leaf item.
__global__ __launch_bounds__(256) void fx_k_screen_group(const int2* __restrict__ items,
                                                         const long* __restrict__ item_off,
                                                         const int2* __restrict__ bc, const FxDevCounts* cnt, int lv,
                                                         long cap, FxDevBasis B, const double* __restrict__ Pn, int la,
                                                         int ld, double tau, double thr, double tau_ovlp,
                                                         uint32_t* __restrict__ mask) {
    const long nitems = cnt->nad[lv] < cap ? cnt->nad[lv] : cap;
    const int lane = threadIdx.x & 63;
    const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long nwaves = ((long)gridDim.x * blockDim.x) >> 6;
    const int S = B.nshell;
    const int* __restrict__ one = B.leaf_one;
    const bool ovlp = tau_ovlp > 0.0;
    for (long it = wave; it < nitems; it += nwaves) {
        const int2 ad = items[it];
        const int a = one[ad.x * 3 + la], d = one[ad.y * 3 + ld];
        if (a < 0 || d < 0) continue;
        const double* __restrict__ Qa = B.Qn + (long)a * S;
        const double* __restrict__ Qd = B.Qn + (long)d * S;
        const double* __restrict__ Sa = B.Sm + (long)a * S;
        const double* __restrict__ Sd = B.Sm + (long)d * S;
        const long e1 = item_off[it + 1];
        for (long e = item_off[it] + lane; e < e1; e += 64) {
            const int2 x = bc[e];
            uint32_t m = 0;
#pragma unroll
            for (int lb = 0; lb < 3; ++lb) {
                const int b = one[x.x * 3 + lb];
                if (b < 0) continue;
#pragma unroll
                for (int lc = 0; lc < 3; ++lc) {
                    const int c = one[x.y * 3 + lc];
                    if (c < 0) continue;
                    const double beta = (Qa[b] * Qd[c]) * Pn[(long)b * S + c];
                    uint32_t cat = 0;
                    if (beta > tau && !(ovlp && !(Sa[b] >= tau_ovlp && Sd[c] >= tau_ovlp))) cat = beta < thr ? 2u : 1u;
                    m |= cat << (2 * (3 * lb + lc));
                }
            }
            mask[e] = m;
        }
    }
}

void fx_launch_screen_group(const int2* items, const long* item_off, const int2* bc, const FxDevCounts* cnt, int lv,
                            long cap, const FxDevBasis& B, const double* Pn, int la, int ld, double tau, double thr,
                            double tau_ovlp, uint32_t* mask, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_screen_group, dim3(fx_grid_for(64 * cap, 256)), dim3(256), 0, st, items, item_off, bc,
                       cnt, lv, cap, B, Pn, la, ld, tau, thr, tau_ovlp, mask);
}

// Leaf entries per leaf row: for every leaf item (A, D), its entry count is
// added to row A.  Used to cut K into row ranges of similar size.
__global__ __launch_bounds__(256) void fx_k_leaf_rows(const int2* __restrict__ items, const long* __restrict__ off,
                                                      const FxDevCounts* cnt, int lv, long cap,
                                                      unsigned long long* __restrict__ rows) {
    const long nitems = cnt->nad[lv];
    for (long p = (long)blockIdx.x * blockDim.x + threadIdx.x; p < cap && p < nitems; p += (long)gridDim.x * blockDim.x)
        atomicAdd(rows + items[p].x, (unsigned long long)(off[p + 1] - off[p]));
}

void fx_launch_leaf_rows(const int2* items, const long* off, const FxDevCounts* cnt, int lv, long cap,
                         unsigned long long* rows, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_leaf_rows, dim3(fx_grid_for(cap, 256)), dim3(256), 0, st, items, off, cnt, lv, cap, rows);
}

// unit list bounds per (la, ld) from the scanned counts
// Unit list bounds per (la, ld) from the scanned counts.  Counts above the
// chunk's unit capacities (taken from earlier calls) mark the chunk as
// overflowed and leave every list empty, so no kernel writes past the unit
// buffer; the counts are recorded for the next call's capacities.
__global__ void fx_k_unit_bounds(const long* __restrict__ upos, long cap, FxDevCounts* cnt, FxDevRun* run,
                                 FxUnitCaps uc) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    long b[10];
    for (int k = 0; k < 10; ++k) b[k] = upos[(long)k * cap];
    bool over = b[9] > uc.total;
    for (int k = 0; k < 9; ++k) {
        const long n = b[k + 1] - b[k];
        if (n > uc.cap[k]) over = true;
        if (n > run->ucls[k]) run->ucls[k] = n;
    }
    if (over && !cnt->overflow) {
        cnt->overflow = 1;
        run->overflow = 1;
        run->incomplete = 1;
    }
    for (int k = 0; k < 10; ++k) cnt->ubase[k] = cnt->overflow ? 0 : b[k];
}

void fx_launch_unit_bounds(const long* upos, long cap, FxDevCounts* cnt, FxDevRun* run, const FxUnitCaps& uc,
                           hipStream_t st) {
    hipLaunchKernelGGL(fx_k_unit_bounds, dim3(1), dim3(64), 0, st, upos, cap, cnt, run, uc);
}

__global__ __launch_bounds__(256) void fx_k_unit_write(const int2* __restrict__ items, const FxDevCounts* cnt, int lv,
                                                       long cap, const int* __restrict__ leaf_lofs,
                                                       const int* __restrict__ leaf_lsh, const long* __restrict__ upos,
                                                       int* __restrict__ units) {
    const long nitems = cnt->overflow ? 0 : cnt->nad[lv];
    const int sym = cnt->sym;
    for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < 9 * cap; t += (long)gridDim.x * blockDim.x) {
        const int cls = (int)(t / cap);
        const long p = t - (long)cls * cap;
        if (p >= nitems) continue;
        const int la = cls / 3, ld = cls % 3;
        const int2 ad = items[p];
        const bool diag = sym && ad.x == ad.y;
        const int oa = leaf_lofs[ad.x * 4 + la], na = leaf_lofs[ad.x * 4 + la + 1] - oa;
        const int od = leaf_lofs[ad.y * 4 + ld], nd = leaf_lofs[ad.y * 4 + ld + 1] - od;
        long o = upos[t];
        for (int i = 0; i < na; ++i)
            for (int j = 0; j < nd; ++j) {
                if (diag && leaf_lsh[oa + i] > leaf_lsh[od + j]) continue;
                units[3 * o] = (int)p;
                units[3 * o + 1] = leaf_lsh[oa + i];
                units[3 * o + 2] = leaf_lsh[od + j];
                ++o;
            }
    }
}

void fx_launch_unit_write(const int2* items, const FxDevCounts* cnt, int lv, long cap, const int* leaf_lofs,
                          const int* leaf_lsh, const long* upos, int* units, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_unit_write, dim3(fx_grid_for(9 * cap, 256)), dim3(256), 0, st, items, cnt, lv, cap,
                       leaf_lofs, leaf_lsh, upos, units);
}

// Batched launches: the (la, ld) unit lists of several systems concatenated.
// merge_bounds (one workgroup): per system its offset in the merged list,
// and the merged bounds {0, total}.  merge_copy: one system's list.
__global__ void fx_k_merge_bounds(const FxDevCounts* __restrict__ cnts, int nsys, int k2, long* __restrict__ moff,
                                  long* __restrict__ mb) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    long o = 0;
    for (int i = 0; i < nsys; ++i) {
        moff[i] = o;
        o += cnts[i].ubase[k2 + 1] - cnts[i].ubase[k2];
    }
    mb[0] = 0;
    mb[1] = o;
}

void fx_launch_merge_bounds(const FxDevCounts* cnts, int nsys, int k2, long* moff, long* mb, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_merge_bounds, dim3(1), dim3(64), 0, st, cnts, nsys, k2, moff, mb);
}

__global__ __launch_bounds__(256) void fx_k_merge_copy(const int* __restrict__ units, const FxDevCounts* cnt, int k2,
                                                       const long* __restrict__ moff, int sys, int* __restrict__ munits,
                                                       int* __restrict__ msys) {
    const long lo = cnt->ubase[k2], n = cnt->ubase[k2 + 1] - lo, o = moff[sys];
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (long)gridDim.x * blockDim.x) {
        munits[3 * (o + j)] = units[3 * (lo + j)];
        munits[3 * (o + j) + 1] = units[3 * (lo + j) + 1];
        munits[3 * (o + j) + 2] = units[3 * (lo + j) + 2];
        msys[o + j] = sys;
    }
}

void fx_launch_merge_copy(const int* units, const FxDevCounts* cnt, int k2, long n_max, const long* moff, int sys,
                          int* munits, int* msys, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_merge_copy, dim3(fx_grid_for(n_max, 256)), dim3(256), 0, st, units, cnt, k2, moff, sys,
                       munits, msys);
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
    const long nb = (n + 31) / 32, bj = blockIdx.x;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (long bi = blockIdx.y; bi <= bj && bi < nb; bi += gridDim.y) {
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
        __syncthreads();
    }
}

void fx_launch_psym(const double* P, long n, int* flag, hipStream_t st) {
    const long nb = (n + 31) / 32;
    if (nb > 0) hipLaunchKernelGGL(fx_k_psym, dim3(nb, fx_grid_y(nb)), dim3(256), 0, st, P, n, flag);
}

// ---------------------------------------------------------------------------
// Leaves that are single shells: group every K-block item's (B, C) entries by
// density-side class (l_b, l_c), stably, one wave per item; cls_off[p*10+k]
// is the first entry of class k = l_b*3 + l_c, cls_off[p*10+9] the end.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void fx_k_class_sort(const long* __restrict__ bc_off, const int2* __restrict__ bc,
                                                       const FxDevCounts* cnt, int lv, const int* __restrict__ l,
                                                       int2* __restrict__ out, long* __restrict__ cls_off) {
    const long nitems = cnt->nad[lv];
    const int lane = threadIdx.x & 63;
    const long nw = (long)gridDim.x * (blockDim.x >> 6);
    for (long p = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); p < nitems; p += nw) {
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
}

void fx_launch_class_sort(const long* bc_off, const int2* bc, const FxDevCounts* cnt, int lv, long items_max,
                          const int* l, int2* out, long* cls_off, hipStream_t st) {
    long g = (items_max + 3) / 4;
    if (g > FX_GRID_MAX) g = FX_GRID_MAX;
    if (g < 1) g = 1;
    hipLaunchKernelGGL(fx_k_class_sort, dim3(g), dim3(256), 0, st, bc_off, bc, cnt, lv, l, out, cls_off);
}

// ---------------------------------------------------------------------------
// Fill, and the final scaling K = alpha * acc + beta * K (acc may be K).
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

void fx_launch_fill_u64(unsigned long long* x, long n, unsigned long long v, hipStream_t st) {
    if (n <= 0) return;
    long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(fx_k_fill_t<unsigned long long>, dim3(blocks), dim3(256), 0, st, x, n, v);
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

__global__ void fx_k_finalize(const double* acc, long nn, double alpha, double beta, double* K,
                              const int* overflow) {
    const bool bad = overflow && *overflow;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long k = i; k < nn; k += stride) {
        if (bad) K[k] = __builtin_nan("");
        else K[k] = beta == 0.0 ? alpha * acc[k] : alpha * acc[k] + beta * K[k];
    }
}

void fx_launch_finalize(const double* acc, long nn, double alpha, double beta, double* K, const int* overflow,
                        hipStream_t st) {
    long blocks = (nn + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(fx_k_finalize, dim3(blocks), dim3(256), 0, st, acc, nn, alpha, beta, K, overflow);
}

// Density symmetry flag of a chunk: sym = (no mismatch found) && allowed.
__global__ void fx_k_set_sym(FxDevCounts* cnt, const int* mismatch, int allowed) {
    if (threadIdx.x == 0 && blockIdx.x == 0) cnt->sym = (allowed && *mismatch == 0) ? 1 : 0;
}

void fx_launch_set_sym(FxDevCounts* cnt, const int* mismatch, int allowed, hipStream_t st) {
    hipLaunchKernelGGL(fx_k_set_sym, dim3(1), dim3(64), 0, st, cnt, mismatch, allowed);
}
