#pragma once
// Device code shared by the HIP kernels of libmdx for gfx950 (wave64):
// work-item walkers, word conversions and the per-precision particle state.
//
// Overview of the kernels (step.hip, rebuild.hip, aux_kernels.hip):
//
// One MD step (Sec. 2.2, velocity Verlet with Verlet lists) is one fused
// launch of k_step plus three rebuild kernels that exit at once unless the
// replica's maximum displacement since its last list build exceeded skin/2:
//
//   k_step<P>    per particle: force over its Verlet list (FP32 pair term,
//                sum in the precision P), second half-kick of step n (full-
//                step velocity), first half-kick of step n+1, drift,
//                fixed-point snapshot of the new position, displacement test
//                against the list's reference position, and the count of the
//                particle's new cell (for the sort, Sec. 2.2 cell binning).
//                The sort key is the cell within the particle's species
//                plane: a binary mixture is stored as all A particles by
//                cell, then all B particles by cell.
//   k_scan       per replica: exclusive scan of the cell counts -> cell starts.
//   k_permute<P> per cell of a plane (one wave): stable counting-sort
//                scatter.  Members of a new cell come from the 27
//                surrounding old cells of the same plane (a
//                particle moves less than one cell between builds); a ballot
//                over them in old slot order gives each its new slot.  The
//                whole particle record is gathered into the scratch arena,
//                positions folded back into the box.
//   k_build<P>   per row segment of cells (one workgroup): the segment's
//                27-cell neighbourhood is staged in LDS, every member scans
//                its own cell and then the 13 opposite cell pairs (Sec. 4.1)
//                and writes its list column-major; the sorted record is
//                copied back from scratch.
//
// Bitwise determinism: lists are in a canonical order (own cell, then +o/-o
// pairs; inside a cell the A members, then the B members, in slot order), the sort is stable, each particle sums
// its own list sequentially, and no floating-point atomics are used.  The
// result for a replica therefore does not depend on launch shapes or on
// other replicas in the pool.
#include "md_dev.hpp"
#include "kernels.hpp"

#define LAUNCH_CHECK() return hipGetLastError()

// --------------------------------------------------------------- utilities
__device__ __forceinline__ int remap_block(int b, int nblk, int on)
{
    // Consecutive tiles to one XCD: workgroups are dealt round-robin over
    // the 8 XCDs, so block b runs on XCD b % 8.
    if (!on) return b;
    int per = nblk >> 3;
    if (b < (per << 3)) return (b & 7) * per + (b >> 3);
    return b;
}

__device__ __forceinline__ int slot_of_meta(uint32_t w) { return (int)((w & 0x7FFFFFFFu) >> SLOT_SHIFT); }

// Rank of cell c (= x + nd (y + nd z)) in the replica's cell order: itself
// in row-major order, else from the replica's rank table (a space-filling
// curve through the cells).
__device__ __forceinline__ int cell_rank(int c, const RepDev &r, const int *corder)
{
    return r.curve ? corder[r.coff + c] : c;
}

__device__ __forceinline__ int find_item_slot(const int *pref, int nslots, int item)
{
    // pref[0..nslots] non-decreasing; find s with pref[s] <= item < pref[s+1]
    int lo = 0, hi = nslots;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (pref[mid] <= item) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool slot_selected(int s, int force_slot, const int *need, const Ctl *ctl)
{
    if (force_slot == -1) return need && need[s] != 0;
    if (force_slot == -2) return ctl[s].z != 0;
    return s == force_slot;
}

// Work-item walk of the rebuild kernels.  A step's rebuild (force_slot -1)
// visits the items of the slots on the rebuild list written by k_step; a
// host-forced rebuild visits those of the selected slots (items_pref holds
// the host's per-slot item counts as a prefix).  `which` names the item
// count of a listed slot: 3 the sort's, 4 the list build's, 5 the bulk list
// build's.  `unit` is this worker's index among `nunits` workers;
// visit(slot, item) is called for each item assigned to it.  Consecutive
// slots start on different workers so that small replicas spread over the
// grid.  The slots and their item counts are read 64 at a time, one per lane
// (a few round trips to memory however many replicas rebuild), then walked
// from registers; visit is called from one place only, so that its code is
// emitted once.
template <class F>
__device__ __forceinline__ void for_items(const int *rlist, const int *items_pref, const RepDev *rep,
                                          int max_slots, int force_slot, const Ctl *ctl, int which,
                                          int unit, int nunits, F visit)
{
    const bool listed = force_slot == -1;
    const int cnt = listed ? rlist[0] : max_slots;
    const int lane = __lane_id();
    int cum = 0;
    for (int base = 0; base < cnt; base += 64) {
        const int li = base + lane;
        int sl = 0, its = 0;
        if (li < cnt) {
            if (listed) {
                sl = rlist[1 + li];
                its = which == 3 ? rep[sl].items3 : which == 4 ? rep[sl].items4 : rep[sl].items4b;
            } else {
                sl = li;
                if (slot_selected(sl, force_slot, nullptr, ctl)) its = items_pref[sl + 1] - items_pref[sl];
            }
        }
        const int m = min(64, cnt - base);
        for (int k = 0; k < m; ++k) {
            const int items = __builtin_amdgcn_readlane(its, k);
            if (items == 0) continue;
            const int s = __builtin_amdgcn_readlane(sl, k);
            int first = unit - cum % nunits;
            first += first < 0 ? nunits : 0;
            for (int it = first; it < items; it += nunits) visit(s, it);
            cum += items;
        }
    }
}

__device__ __forceinline__ uint4 dbl2_to_u4(double a, double b)
{
    uint4 u;
    unsigned long long x = __double_as_longlong(a), y = __double_as_longlong(b);
    u.x = (uint32_t)x; u.y = (uint32_t)(x >> 32); u.z = (uint32_t)y; u.w = (uint32_t)(y >> 32);
    return u;
}
__device__ __forceinline__ void u4_to_dbl2(uint4 u, double &a, double &b)
{
    a = __longlong_as_double(((unsigned long long)u.y << 32) | u.x);
    b = __longlong_as_double(((unsigned long long)u.w << 32) | u.z);
}

// ------------------------------------------------------- per-precision state
template <int P> struct State;

template <> struct State<PREC_FP32> {
    float x, y, z, vx, vy, vz;
    __device__ void load(const KArena &A, int i)
    {
        float4 a = ((const float4 *)A.st[0])[i], b = ((const float4 *)A.st[1])[i];
        x = a.x; y = a.y; z = a.z; vx = b.x; vy = b.y; vz = b.z;
    }
    __device__ void store(const KArena &A, int i) const
    {
        ((float4 *)A.st[0])[i] = make_float4(x, y, z, 0.0f);
        ((float4 *)A.st[1])[i] = make_float4(vx, vy, vz, 0.0f);
    }
};

template <> struct State<PREC_DS> {
    dsf x, y, z, vx, vy, vz;
    __device__ void load(const KArena &A, int i)
    {
        float4 a = ((const float4 *)A.st[0])[i], b = ((const float4 *)A.st[1])[i],
               c = ((const float4 *)A.st[2])[i];
        x = {a.x, a.w}; y = {a.y, b.x}; z = {a.z, b.y};
        vx = {b.z, c.y}; vy = {b.w, c.z}; vz = {c.x, c.w};
    }
    __device__ void store(const KArena &A, int i) const
    {
        ((float4 *)A.st[0])[i] = make_float4(x.hi, y.hi, z.hi, x.lo);
        ((float4 *)A.st[1])[i] = make_float4(y.lo, z.lo, vx.hi, vy.hi);
        ((float4 *)A.st[2])[i] = make_float4(vz.hi, vx.lo, vy.lo, vz.lo);
    }
};

struct StateD {
    double x, y, z, vx, vy, vz;
    __device__ void load(const KArena &A, int i)
    {
        double2 a = ((const double2 *)A.st[0])[i], b = ((const double2 *)A.st[1])[i],
                c = ((const double2 *)A.st[2])[i];
        x = a.x; y = a.y; z = b.x; vx = b.y; vy = c.x; vz = c.y;
    }
    __device__ void store(const KArena &A, int i) const
    {
        ((double2 *)A.st[0])[i] = make_double2(x, y);
        ((double2 *)A.st[1])[i] = make_double2(z, vx);
        ((double2 *)A.st[2])[i] = make_double2(vy, vz);
    }
};
template <> struct State<PREC_MIX> : StateD {};
template <> struct State<PREC_FP64> : StateD {};
