// Device-side data layout, per-precision traits and the small helpers shared
// by the kernels and the host engine of libmdx.
//
// HBM layout (one particle arena of P slots, structure of arrays, every
// per-particle record a multiple of 16 bytes so that loads are dwordx4):
//   state word k  : uint4 st[k][P]   (k < NW; precision-dependent packing)
//   snapshot      : uint4 snap[2][NS][P]  ping-pong, read by neighbours
//   reference pos : uint4 xref[NS][P]     positions at the last list build
//   meta          : int4 meta[P]          (image x, image y, image z, id)
//   list count    : int nbr_cnt[P];  list: int4 rows in tiles of 64 slots
//                   (row q of slot i at list_row_index(i, q, cap); the rows
//                   of a tile are contiguous, and row q of its 64 slots is
//                   1 KB contiguous); an entry is the neighbour's slot times
//                   16, the byte offset of its 16-byte snapshot record
//   observation   : double obs[P][8]      (fx, fy, fz, e_i, w_i, vx, vy, vz)
// plus a scratch copy of st/snap/meta used by the cell sort.
//
// The snapshot is what neighbours gather every step.  For the FP32, DS and
// MIXED64 paths it is a 32-bit fixed-point copy of the position,
// X = round(x * 2^32 / L) mod 2^32, so that the minimum image is the int32
// wrap-around of X_i - X_j and a pair separation is exact before it is
// converted to float.  Its w word holds species << 31 | slot << 4 (the
// species in the sign bit, so one compare tests it).  The FP64
// path keeps double positions (two words: x,y | z,w) and the textbook
// minimum image.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "ds.hpp"

enum { PREC_FP32 = 0, PREC_DS = 1, PREC_MIX = 2, PREC_FP64 = 3 };

template <int P> struct Traits;
template <> struct Traits<PREC_FP32> { static constexpr int NW = 2, NS = 1; };
template <> struct Traits<PREC_DS> { static constexpr int NW = 3, NS = 1; };
template <> struct Traits<PREC_MIX> { static constexpr int NW = 3, NS = 1; };
template <> struct Traits<PREC_FP64> { static constexpr int NW = 3, NS = 2; };

// Replica (slot) geometry, one entry per slot in device memory.
struct RepDev {
    int n;        // particles
    int off;      // first particle slot in the arena
    int nd;       // cells per box edge (1 = single-cell mode)
    int coff;     // first cell in the cell arena (planes * nd^3 + 1 entries reserved)
    int planes;   // species planes of the sort key (1, or 2 for a binary mixture)
    int curve;    // 1: cells are ranked along a space-filling curve (rank table at coff)
    double L;     // box edge
    double invL;  // 1 / L
    double fxs;   // 2^32 / L   (double -> fixed point)
    float sc;     // L / 2^32   (fixed point unit in length units)
    float L_hi, L_lo; // L as double-single
    int items3, items4; // work items of the sort and list-build kernels
    int bparts;   // list-build work items per row segment (its members split evenly)
    int blanes;   // lanes building one member's list; 0 = chosen per work item
    // pair constants in fixed-point units u = L / 2^32, per species pair
    // [si*2+sj]: rc^2/u^2, sigma^2/u^2, 24 eps/u; smoothing: rc/u, u/(h sigma),
    // 1/(h sigma); and (skin/2)^2/u^2 for the displacement test
    float rc2s[4], sig2s[4], e24s[4], rcs[4], xsc[4], ihs[4];
    float hs2s;
    float hs2s_early; // (rebuild_early * skin/2)^2 / u^2 (aligned rebuilds)
    int items4b;      // list-build work items of a bulk build (unsplit segments)
};

// Control word of a slot: x = completed steps, y = 1 if velocities are at a
// full step, z = 1 if attached.  Double-buffered by step parity.
typedef int4 Ctl;

// Pair table in float and double, indexed [si*2+sj].
struct PairDev {
    float rl2[4];    // list radius^2 = (rc + skin)^2
    float rc2[4];
    float sig2[4];
    float eps24[4];  // 24 eps
    float eps4[4];   // 4 eps
    float shift[4];  // V_LJ(rc)
    double rl2d[4], rc2d[4], sig2d[4], eps24d[4], eps4d[4], shiftd[4];
    float hs2;       // (skin/2)^2
    double hs2d;
    double hs2d_early; // (rebuild_early * skin/2)^2
    int align_every;   // rebuild_every (0 = off)
    int nsp;
    int uniform;     // 1 if rc_ab / sigma_ab is the same for every pair
    float s2cut;     // then (sigma_ab / rc_ab)^2: a pair is inside iff sigma^2/r^2 > s2cut
    int smooth;      // 1: potential times g(x) = x^4/(1+x^4), x = (r - rc)/(h sigma) (Sec. 4)
    double hsd[4];   // h sigma_ab
    double rcd[4];   // rc_ab
};

// Integration constants (dt and dt/2m) in every representation.
struct IntegDev {
    double dt, h;       // h = dt / (2 m)
    float dtf, hf;
    float dt_hi, dt_lo, h_hi, h_lo;
    double m;
};

// FP64 snapshots carry the meta word as the raw bits of their fourth double.
__host__ __device__ __forceinline__ uint32_t meta_of_bits(double w)
{
#ifdef __HIP_DEVICE_COMPILE__
    return (uint32_t)(unsigned long long)__double_as_longlong(w);
#else
    unsigned long long b;
    __builtin_memcpy(&b, &w, 8);
    return (uint32_t)b;
#endif
}
__host__ __device__ __forceinline__ double bits_of_meta(uint32_t m)
{
    unsigned long long b = 0xFFFFFFFF00000000ull | m;
#ifdef __HIP_DEVICE_COMPILE__
    return __longlong_as_double((long long)b);
#else
    double w;
    __builtin_memcpy(&w, &b, 8);
    return w;
#endif
}

// Per-replica status bits written by the kernels (the MD_ST_* values of the
// C ABI): list overflow, non-finite position, lost particles, unpaddable
// list.  Any of them stops the replica.
#define ST_HALT (1 | 2 | 4 | 8)

#define SLOT_SHIFT 4
#define MAX_ARENA_SLOTS (1 << 28) // list entries are 32-bit byte offsets (slot x 16)

// List entry of slot j: the byte offset of its snapshot record.
__host__ __device__ __forceinline__ int list_entry(int j) { return (int)((uint32_t)j << 4); }
__host__ __device__ __forceinline__ int list_slot(int e) { return (int)((uint32_t)e >> 4); }

// int4 row q of the list of slot i: tiles of LIST_TILE slots, each holding
// its cap/4 rows one after another.  P is a multiple of the tile, so the
// P * cap / 4 rows fill the list array exactly.
#define LIST_TILE 64
__host__ __device__ __forceinline__ size_t list_row_index(int i, int q, int cap)
{
    return ((size_t)(i / LIST_TILE) * (size_t)(cap >> 2) + (size_t)q) * LIST_TILE + (size_t)(i % LIST_TILE);
}

// The L lanes of a particle (L = 1, 2 or 4, lg = log2 L) read its list in
// rows of four entries, lane l taking rows l, l + L, l + 2L, ...  Entries
// are dealt to the lanes in turn, so that the lanes of a particle gather
// neighbouring entries (often one cache line) in the same instruction:
// entry k sits in row L (k / 4L) + k % L, column (k / L) % 4.  A list is
// padded to a multiple of 4L entries (the capacity is a multiple of 16) and
// fills L ceil(n / 4L) rows.
__host__ __device__ __forceinline__ int list_entry_row(int k, int lg)
{
    return ((k >> (lg + 2)) << lg) | (k & ((1 << lg) - 1));
}
__host__ __device__ __forceinline__ int list_entry_col(int k, int lg) { return (k >> lg) & 3; }
__host__ __device__ __forceinline__ int list_rows(int n, int lg)
{
    return ((n + (4 << lg) - 1) >> (lg + 2)) << lg;
}
#define NO_SLOT 0xFFFFFFFFu

// Species (0 = A, 1 = B) of a meta word.
__host__ __device__ __forceinline__ int species_of(uint32_t w) { return (int)(w >> 31); }

// ---------------------------------------------------------------- fixed point
__host__ __device__ __forceinline__ uint32_t to_fixed(double x, double fxs)
{
    double t = x * fxs;
#ifdef __HIP_DEVICE_COMPILE__
    long long k = __double2ll_rn(t);
#else
    long long k = llrint(t);
#endif
    return (uint32_t)(unsigned long long)k;
}

__host__ __device__ __forceinline__ uint32_t fixed_cell1(uint32_t X, uint32_t nd)
{
    return (uint32_t)(((unsigned long long)X * nd) >> 32);
}

__host__ __device__ __forceinline__ int fixed_cell(uint32_t X, uint32_t Y, uint32_t Z, int nd)
{
    return (int)(fixed_cell1(X, nd) + (uint32_t)nd * (fixed_cell1(Y, nd) + (uint32_t)nd * fixed_cell1(Z, nd)));
}

// FP64 path: cell of a double position (wrapped into [0, L) first).
__host__ __device__ __forceinline__ int dbl_cell1(double x, double L, double invL, int nd)
{
    double w = x - L * floor(x * invL);
    int c = (int)(w * invL * (double)nd);
    if (c < 0) c = 0;
    if (c >= nd) c = nd - 1;
    return c;
}

// Sort key of a particle (its index in the replica's cell arrays): the rank
// of its cell in the replica's cell order, within the plane of its species.
// With two planes every species is sorted by cell on its own (all A, then
// all B), so a wave of the force kernel holds particles of one species,
// whose lists are of similar length.
__host__ __device__ __forceinline__ int sort_key(int rank, uint32_t meta, int planes, int nd)
{
    return planes > 1 ? species_of(meta) * nd * nd * nd + rank : rank;
}

__host__ __device__ __forceinline__ int dbl_cell(double x, double y, double z, double L, double invL, int nd)
{
    return dbl_cell1(x, L, invL, nd) + nd * (dbl_cell1(y, L, invL, nd) + nd * dbl_cell1(z, L, invL, nd));
}

// The 13 half-space cell offsets; a neighbour search visits the own cell and
// then each offset o followed by -o (opposite cells summed together, Sec. 4.1).
__host__ __device__ __forceinline__ void half_offset(int k, int &dx, int &dy, int &dz)
{
    // k in [0,13): enumerate (dz, dy, dx) lexicographically, keep the half
    // space dz > 0 or (dz == 0 and (dy > 0 or (dy == 0 and dx > 0))).
    int cnt = 0;
    for (int z = -1; z <= 1; ++z)
        for (int y = -1; y <= 1; ++y)
            for (int x = -1; x <= 1; ++x) {
                bool pos = z > 0 || (z == 0 && (y > 0 || (y == 0 && x > 0)));
                if (!pos) continue;
                if (cnt == k) { dx = x; dy = y; dz = z; return; }
                ++cnt;
            }
    dx = dy = dz = 0;
}
