// Launchers of the support kernels (fx_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// One level of the hextree traversal (see fx_kernels.hip).
struct FxLevelArgs {
    const int2* ad;        // parent ADs (this chunk)
    const long* bc_off;    // [nad+1] absolute offsets into bc
    const int2* bc;        // entries
    const int* bc_parent;  // AD index of each entry (relative to chunk when p_base applied)
    long e_begin, e_count; // entry range of this chunk
    int p_base;            // subtract from bc_parent to get chunk-relative AD index
    int nad;
    const int* ch0;        // level-k node -> first child at level k+1
    const int* nch;        // 1 or 2
    const double* Qsq;     // level k+1 tables
    const double* Psq;
    int nk1;
    double tau2;
    int sym;               // keep only children with A_i <= D_l (symmetric density)
};

struct FxPrimPair;
void fx_launch_prim_pairs(const double* exps, const double* coefs, const int* prim_shell, const double* xyz, long Nt,
                          FxPrimPair* out, hipStream_t st);
void fx_launch_pnorm(const double* P, long n, const int* l, const int* f0, int S, double* Pn, hipStream_t st);
void fx_launch_leaf_sq(const double* x, int S, const int* sL, const int* sR, int nleaf, double* out, hipStream_t st);
void fx_launch_level_up(const double* child, int nchild_nodes, const int* ch0, const int* nch, int nk, double* out,
                        hipStream_t st);
long fx_scan_tiles(long n);
void fx_scan_popc_u8(const uint8_t* in, long n, long* out, long* partial, long* total_dev, hipStream_t st);
void fx_scan_i32(const int* in, long n, long* out, long* partial, long* total_dev, hipStream_t st);
void fx_launch_expand_mask(const FxLevelArgs& L, uint8_t* mask, hipStream_t st);
void fx_launch_expand_adflag(const FxLevelArgs& L, const long* pos, int* flag, hipStream_t st);
void fx_launch_expand_adwrite(const FxLevelArgs& L, const long* pos, const int* flag, const long* adpos, int2* ad_next,
                              long* bc_off_next, long total_entries, long total_ads, hipStream_t st);
void fx_launch_expand_write(const FxLevelArgs& L, const uint8_t* mask, const long* pos, const long* adpos,
                            int2* bc_next, int* parent_next, hipStream_t st);
void fx_launch_unit_count(const int2* items, long nitems, const int* leaf_lofs, const int* leaf_lsh, int sym, int* cnt,
                          hipStream_t st);
void fx_launch_unit_write(const int2* items, long nitems, long item_base, const int* leaf_lofs, const int* leaf_lsh,
                          int sym, const long* upos, int* units, hipStream_t st);
void fx_launch_max_inplace(double* a, const double* b, long n, hipStream_t st);
// flag <- 1 if P (n x n) is not bitwise symmetric; flag must be 0 on entry
void fx_launch_psym(const double* P, long n, int* flag, hipStream_t st);
void fx_launch_class_sort(const long* bc_off, const int2* bc, long nitems, const int* l, int2* out, long* cls_off,
                          hipStream_t st);
void fx_launch_fill(double* x, long n, double v, hipStream_t st);
void fx_launch_fill_i32(int* x, long n, int v, hipStream_t st);
void fx_launch_fill_u32(unsigned int* x, long n, unsigned int v, hipStream_t st);
void fx_launch_finalize(const double* slots, int nslot, long nn, double alpha, double beta, double* K, hipStream_t st);
