// Internal structures shared by the host planner and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// One wave (one K-block unit) per workgroup: units differ widely in work, and
// a workgroup of several waves holds its slot until its slowest wave ends
// (4 waves per workgroup: 20.7 s; 1: 17.0 s on the 1000-atom cluster).
#define FX_CLASS_WAVES 1          // waves (work units) per thread-variant workgroup
#define FX_COOP_WAVES 2           // waves per cooperative-variant workgroup
#define FX_MAX_DENS 2             // densities contracted with the same integrals

// Boys table: row i holds F_j(T_i), j = 0..14 (highest m 8 + 6 Taylor terms),
// then e^{-T_i} in column 15; T_i = i / 32, i = 0..FX_BOYS_NROW-1.
#define FX_BOYS_DT (1.0 / 32.0)
#define FX_BOYS_INV_DT 32.0
#define FX_BOYS_TMAX 60.0
#define FX_BOYS_NF 15
#define FX_BOYS_NCOL 16
#define FX_BOYS_NROW 1922

// Primitive-pair data, one record per ordered pair of primitives (i of shell
// x, j of shell y): exponent sum p, 1/p, centre P, and
// K = c_i c_j exp(-a_i a_j / p |XY|^2) with normalised weights.
struct FxPrimPair {
    double p, op, Px, Py, Pz, K;
};

// ALL: every surviving quartet in the kernel's precision; MIXED_HI / _LO: the
// quartets with beta >= / < the FP32 threshold; DUAL: both, in one kernel.
enum { FX_MODE_ALL = 0, FX_MODE_MIXED_HI = 1, FX_MODE_MIXED_LO = 2, FX_MODE_DUAL = 3 };

// Basis in the tree's shell order (device pointers).
struct FxDevBasis {
    int nshell, nbf;
    const int* l;         // [S]
    const int* nprim;     // [S]
    const int* pofs;      // [S] first primitive
    const int* f0;        // [S] first function, CALLER order (rows/cols of P and K)
    const double* xyz;    // [S*3] bohr
    const double* exps;   // [sum nprim]
    const double* coefs;  // [sum nprim] normalised radial weights
    const double* Qn;     // [S*S] ||Q_ab||_F
    const double* Sm;     // [S*S] largest |overlap| of the functions of shells a and b (Eqs. 3-4)
    const int* leaf_lofs; // [nleaf*4] per leaf: offsets of its l=0,1,2 shell lists, then end
    const int* leaf_lsh;  // shell indices grouped per leaf and l
    const int* leaf_one;  // [nleaf*3] per leaf and l: its one shell of that l (-1: none);
                          // null when some leaf holds two shells of one l
    long ntprim;          // total primitives Nt
    const FxPrimPair* pp; // [Nt*Nt] primitive-pair records, (global prim i, global prim j)
};

#define FX_MAX_LEVELS 32

// Sizes of one traversal chunk of one system, produced and read on the
// device (the host never needs them to launch the next step).
struct FxDevCounts {
    long nad[FX_MAX_LEVELS];          // (A, D) pairs at each level
    long ne[FX_MAX_LEVELS];           // (B, C) entries at each level
    long tot[2];                      // scan totals (entries, ADs) of the level being expanded
    long ubase[10];                   // unit list bounds per (la, ld): units of la*3+ld in [ubase[k], ubase[k+1])
    long need;                        // entries requested by a level that exceeded its capacity
    int need_level;                   // that level
    int overflow;                     // a level exceeded its capacity: this chunk's K blocks are incomplete
    int sym;                          // 1: symmetric density, only K blocks a <= d are built
};

// Totals of one call over its systems and traversal chunks (device).
struct FxDevRun {
    long e_in, e_leaf;                // largest inner / leaf entry counts of a chunk (next call's capacities)
    long need_in, need_leaf;          // largest requests of an inner / the leaf level that exceeded its capacity
    int overflow;                     // some chunk exceeded a capacity
    int incomplete;                   // some chunk that exceeded a capacity was not run again: K is NaN
    long frontier[FX_MAX_LEVELS];     // entries per level, summed over the completed chunks
    long items, units;                // leaf (A, D) items and K-block units, summed
    long ucls[9];                     // largest unit count per (la, ld) of a chunk (next call's capacities)
};

// Unit capacities of one chunk per (la, ld), and of its whole unit list.
struct FxUnitCaps {
    long cap[9];
    long total;
};

// One system (or traversal chunk) as seen by the class kernels.
struct FxSys {
    FxDevBasis basis;
    const double* P[FX_MAX_DENS];     // densities (n x n, caller order); the first FxClassArgs::ndens are used
    long n;
    const double* Pn;                 // [S*S] shell-level ||P_bc||_F (largest over the densities)
    const long* bc_off;               // per leaf item: offsets into bc
    const int2* bc;                   // (B, C) leaf nodes
    const long* cls_off;              // single-shell leaves: per item 10 class offsets, else null
    const uint32_t* mask;             // leaves with at most one shell of each l: per leaf entry, the screen of
                                      // the (l_a, l_d) group being launched, 2 bits per (l_b, l_c) at bit
                                      // 2 (3 l_b + l_c): 0 culled, 1 beta >= thr, 2 beta < thr; or null
    double* acc[FX_MAX_DENS];         // K accumulator of each density (n x n, caller order)
    const FxDevCounts* cnt;           // sizes; cnt->sym = 1: only units a <= d (tree order) exist and each
                                      // writes K_ad and K_da
};

// launch options (autotuned per class and precision)
#define FX_LAUNCH_XCD 1               // XCD-aware workgroup remap

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8).  This bijection of [0, nb) gives XCD x the logical blocks
// [x*q + min(x, r), ...) of a contiguous range (q = nb / 8, r = nb % 8), so
// consecutive logical blocks share an XCD and its L2.
__host__ __device__ inline long fx_xcd_remap(long b, long nb) {
    const long q = nb / 8, r = nb % 8, x = b % 8, i = b / 8;
    return x * q + (x < r ? x : r) + i;
}

// Arguments of one class kernel launch.
struct FxClassArgs {
    FxSys one;                        // the system when sys == null
    const FxSys* sys;                 // batched launches: per-unit system descriptors
    const int* unit_sys;              // batched launches: system of every unit
    const double* boys;
    const int* units;                 // unit list (item, a, d), 3 ints per unit
    const long* ulh;                  // device {lo, hi}: this launch's units are units[lo..hi)
    long nbound;                      // host bound of hi - lo (the grid size)
    const int* order;                 // schedule permutation of units (relative to lo), or null
    double tau, thr;
    double tau_ovlp;                  // > 0: a quartet needs Sm_ab >= tau_ovlp and Sm_cd >= tau_ovlp
    int block;                        // 1: leaf_screen BLOCK, every quartet of a surviving leaf task
    int mode;                         // FX_MODE_*
    int flags;                        // FX_LAUNCH_*
    int ndens;                        // densities per system (1 or 2)
    unsigned long long* counters;     // [3]: quartets, primitive quartets, quartets that also stand
                                      // for their mirror (symmetric system, a != d) (nullable)
    unsigned long long* counters2;    // DUAL: the same for the FP32 quartets (nullable)
    float* times;                     // per-unit wall-clock ticks (nullable; timing probes)
    double* beta32;                   // sum of the bounds beta of the quartets evaluated in FP32 (nullable)
};

// launches one wave per unit; returns the variant launched (0 one quartet
// per lane, 1 one quartet per wave, 2 one quartet per lane in both precisions)
#define FX_DECLARE_LAUNCH(cls) int fx_launch_##cls(int prec32, int variant, FxClassArgs A, hipStream_t st);
typedef int (*fx_class_launcher)(int, int, FxClassArgs, hipStream_t);
void fx_launch_schwarz(FxDevBasis B, const double* boys, const int2* pairs, long npairs, double* Qn,
                       hipStream_t st);
