// Launchers of the support kernels (fx_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fx_internal.h"

// counter slots of each traversal-partition sum (spread to avoid contention)
#define FX_PART_SLOTS 256

// One level of the hextree traversal (see fx_kernels.hip); level k -> k+1.
struct FxLevelArgs {
    const int2* ad;        // level-k ADs
    const long* bc_off;    // [nad+1] offsets into bc
    const int2* bc;        // level-k entries
    const int* bc_parent;  // AD index of each entry
    FxDevCounts* cnt;      // device sizes (nad[k], ne[k] in; level k+1 out)
    int k;
    const int* ch0;        // level-k node -> first child at level k+1
    const int* nch;        // 1 or 2
    const double* Qsq;     // level k+1 tables
    const double* Psq;
    int nk1;
    double tau2;
    const double* Smx;     // level k+1 block maxima of the shell-pair overlaps (nullable)
    double tau_ovlp;       // > 0: a child needs Smx_{A_i B_j} >= tau_ovlp and Smx_{C_k D_l} >= tau_ovlp
    const int* sL1;        // level k+1 node shell ranges (chunk filter)
    const int* sR1;
    int a_lo, a_hi;        // this chunk's K rows: shells [a_lo, a_hi) in tree order
    // traversal partition (nullable): function counts of the level k+1 nodes
    // and three sums of |A||B||C||D| over tasks: [0] surviving leaf tasks
    // (when level k+1 is the leaf level), [1] culled children, [2] children
    // dropped by the symmetric form (their mirrors are traversed)
    const int* nf1;
    int leaf_next;
    unsigned long long* part;
};

struct FxPrimPair;
void fx_launch_prim_pairs(const double* exps, const double* coefs, const int* prim_shell, const double* xyz, long Nt,
                          FxPrimPair* out, hipStream_t st);
void fx_launch_pnorm(const double* P, long n, const int* l, const int* f0, int S, double* Pn, hipStream_t st);
void fx_launch_leaf_sq(const double* x, int S, const int* sL, const int* sR, int nleaf, double* out, hipStream_t st);
// block maxima of an S x S table: leaf level, then parents from children
void fx_launch_leaf_max(const double* x, int S, const int* sL, const int* sR, int nleaf, double* out, hipStream_t st);
void fx_launch_level_max(const double* child, int nchild_nodes, const int* ch0, const int* nch, int nk, double* out,
                         hipStream_t st);
// largest |overlap| of every shell pair (normalised Cartesian components)
void fx_launch_overlap_max(FxDevBasis B, const int2* pairs, long npairs, double* Sm, hipStream_t st);
void fx_launch_level_up(const double* child, int nchild_nodes, const int* ch0, const int* nch, int nk, double* out,
                        hipStream_t st);
long fx_scan_tiles(long n);
// exclusive scans; *_dev: element count mult * (*n_dev) read on the device,
// n_max an upper bound of it; out[n] and *total receive the total
void fx_scan_popc_u8_dev(const uint8_t* in, const long* n_dev, int mult, long n_max, uint32_t* out, long* partial,
                         long* total, hipStream_t st);
void fx_scan_i32_dev(const int* in, const long* n_dev, int mult, long n_max, long* out, long* partial, long* total,
                     hipStream_t st);
void fx_scan_i32(const int* in, long n, long* out, long* partial, long* total_dev, hipStream_t st);
void fx_launch_root(FxDevCounts* cnt, const double* Qsq0, const double* Psq0, double tau2, int2* ad, long* bc_off,
                    int2* bc, int* parent, unsigned long long* part, unsigned long long n4, int one_level,
                    int count_root, hipStream_t st);
void fx_launch_expand_mask(const FxLevelArgs& L, long n_max, uint8_t* mask, hipStream_t st);
void fx_launch_commit_entries(FxDevCounts* cnt, int k, const long* total, long cap, hipStream_t st);
void fx_launch_commit_ads(FxDevCounts* cnt, int k, const long* total, hipStream_t st);
void fx_launch_expand_adflag(const FxLevelArgs& L, long nad_max, const uint32_t* pos, int* flag, hipStream_t st);
void fx_launch_expand_adwrite(const FxLevelArgs& L, long nad_max, const uint32_t* pos, const int* flag,
                              const long* adpos, int2* ad_next, long* bc_off_next, hipStream_t st);
void fx_launch_expand_write(const FxLevelArgs& L, long n_max, const uint8_t* mask, const uint32_t* pos,
                            const long* adpos, int2* bc_next, int* parent_next, hipStream_t st);
void fx_launch_unit_count(const int2* items, const FxDevCounts* cnt, int lv, long cap, const int* leaf_lofs,
                          const int* leaf_lsh, int* out, hipStream_t st);
void fx_launch_screen_group(const int2* items, const long* item_off, const int2* bc, const FxDevCounts* cnt, int lv,
                            long cap, const FxDevBasis& B, const double* Pn, int la, int ld, double tau, double thr,
                            double tau_ovlp, uint32_t* mask, hipStream_t st);
void fx_launch_leaf_rows(const int2* items, const long* off, const FxDevCounts* cnt, int lv, long cap,
                         unsigned long long* rows, hipStream_t st);
void fx_launch_unit_bounds(const long* upos, long cap, FxDevCounts* cnt, FxDevRun* run, const FxUnitCaps& uc,
                           hipStream_t st);
void fx_launch_unit_write(const int2* items, const FxDevCounts* cnt, int lv, long cap, const int* leaf_lofs,
                          const int* leaf_lsh, const long* upos, int* units, hipStream_t st);
void fx_launch_merge_bounds(const FxDevCounts* cnts, int nsys, int k2, long* moff, long* mb, hipStream_t st);
void fx_launch_merge_copy(const int* units, const FxDevCounts* cnt, int k2, long n_max, const long* moff, int sys,
                          int* munits, int* msys, hipStream_t st);
void fx_launch_set_sym(FxDevCounts* cnt, const int* mismatch, int allowed, hipStream_t st);
void fx_launch_chunk_done(const FxDevCounts* cnt, int nl, const unsigned long long* cpart, unsigned long long* part,
                          FxDevRun* run, hipStream_t st);
void fx_launch_units_done(const FxDevCounts* cnt, FxDevRun* run, hipStream_t st);
void fx_launch_max_inplace(double* a, const double* b, long n, hipStream_t st);
// flag <- 1 if P (n x n) is not bitwise symmetric; flag must be 0 on entry
void fx_launch_psym(const double* P, long n, int* flag, hipStream_t st);
void fx_launch_class_sort(const long* bc_off, const int2* bc, const FxDevCounts* cnt, int lv, long items_max,
                          const int* l, int2* out, long* cls_off, hipStream_t st);
void fx_launch_fill(double* x, long n, double v, hipStream_t st);
void fx_launch_fill_i32(int* x, long n, int v, hipStream_t st);
void fx_launch_fill_u32(unsigned int* x, long n, unsigned int v, hipStream_t st);
void fx_launch_fill_u64(unsigned long long* x, long n, unsigned long long v, hipStream_t st);
// K <- alpha * acc + beta * K elementwise (acc may equal K); NaN when *overflow
void fx_launch_finalize(const double* acc, long nn, double alpha, double beta, double* K, const int* overflow,
                        hipStream_t st);
