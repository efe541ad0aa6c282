// HIP kernels of libmdx for gfx950 (wave64).
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
//   k_scan       per replica: exclusive scan of the cell counts -> cell starts.
//   k_permute<P> per cell (one wave): stable counting-sort scatter.  Members
//                of a new cell come from the 27 surrounding old cells (a
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
// pairs, slot order inside a cell), the sort is stable, each particle sums
// its own list sequentially, and no floating-point atomics are used.  The
// result for a replica therefore does not depend on launch shapes or on
// other replicas in the pool.
#include "md_dev.hpp"
#include "kernels.hpp"

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

__device__ __forceinline__ int slot_of_meta(uint32_t w) { return (int)(w >> SLOT_SHIFT); }

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

// Work-item walk of the rebuild kernels.  A step's rebuild (force_slot -1)
// visits only the items of the slots on the rebuild list written by k_step;
// a host-forced rebuild visits every item and filters by slot.  `unit` is
// this worker's index among `nunits` workers; visit(slot, item) is called for
// each item assigned to it.  Consecutive slots start on different workers so
// that small replicas spread over the grid.
template <class F>
__device__ __forceinline__ void for_items(const int *rlist, const int *items_pref, const RepDev *rep,
                                          int max_slots, int force_slot, const Ctl *ctl, int which,
                                          int unit, int nunits, F visit);

__device__ __forceinline__ bool slot_selected(int s, int force_slot, const int *need, const Ctl *ctl)
{
    if (force_slot == -1) return need && need[s] != 0;
    if (force_slot == -2) return ctl[s].z != 0;
    return s == force_slot;
}

template <class F>
__device__ __forceinline__ void for_items(const int *rlist, const int *items_pref, const RepDev *rep,
                                          int max_slots, int force_slot, const Ctl *ctl, int which,
                                          int unit, int nunits, F visit)
{
    if (force_slot == -1) {
        const int cnt = rlist[0];
        int cum = 0;
        for (int li = 0; li < cnt; ++li) {
            const int s = rlist[1 + li];
            const int items = which == 3 ? rep[s].items3 : rep[s].items4;
            int first = unit - cum % nunits;
            first += first < 0 ? nunits : 0;
            for (int it = first; it < items; it += nunits) visit(s, it);
            cum += items;
        }
        return;
    }
    const int total = items_pref[max_slots];
    for (int it = unit; it < total; it += nunits) {
        const int s = find_item_slot(items_pref, max_slots, it);
        if (!slot_selected(s, force_slot, nullptr, ctl)) continue;
        visit(s, it - items_pref[s]);
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

// ---------------------------------------------------- force accumulators
template <int P> struct FAcc;

template <> struct FAcc<PREC_FP32> {
    float x, y, z;
    __device__ void init() { x = y = z = 0.0f; }
    __device__ void add(float fs, float dx, float dy, float dz, int, int, int)
    {
        x = __builtin_fmaf(fs, dx, x);
        y = __builtin_fmaf(fs, dy, y);
        z = __builtin_fmaf(fs, dz, z);
    }
    __device__ void get(double &fx, double &fy, double &fz) const { fx = x; fy = y; fz = z; }
};

template <> struct FAcc<PREC_DS> {
    sum2f x, y, z;
    __device__ void init() { x.init(); y.init(); z.init(); }
    __device__ void add(float fs, float dx, float dy, float dz, int, int, int)
    {
        x.add(fs * dx);
        y.add(fs * dy);
        z.add(fs * dz);
    }
    __device__ void get(double &fx, double &fy, double &fz) const
    {
        fx = ds_to_double(x.result()); fy = ds_to_double(y.result()); fz = ds_to_double(z.result());
    }
};

template <> struct FAcc<PREC_MIX> {
    double x, y, z;
    __device__ void init() { x = y = z = 0.0; }
    __device__ void add(float fs, float, float, float, int ix, int iy, int iz)
    {
        double f = (double)fs;
        x = __builtin_fma(f, (double)ix, x);
        y = __builtin_fma(f, (double)iy, y);
        z = __builtin_fma(f, (double)iz, z);
    }
    __device__ void get(double &fx, double &fy, double &fz) const { fx = x; fy = y; fz = z; }
};

// Butterfly sum of the partial sums of the LPP lanes that share a particle
// (lanes 2^k apart exchange; every step is a commutative add, so all lanes
// of the group end with the same bits).
__device__ __forceinline__ void lane_sum(float &x, int m) { x += __shfl_xor(x, m, 64); }
__device__ __forceinline__ void lane_sum(double &x, int m) { x += __shfl_xor(x, m, 64); }
__device__ __forceinline__ void lane_sum(dsf &x, int m)
{
    dsf o = {__shfl_xor(x.hi, m, 64), __shfl_xor(x.lo, m, 64)};
    x = ds_add(x, o);
}

// ------------------------------------------------------------ integration
// Velocity-Verlet pieces: kick v += (dt/2m) F, drift r += dt v.
__device__ __forceinline__ void kick(State<PREC_FP32> &s, const FAcc<PREC_FP32> &f, const IntegDev &g)
{
    s.vx = __builtin_fmaf(g.hf, f.x, s.vx);
    s.vy = __builtin_fmaf(g.hf, f.y, s.vy);
    s.vz = __builtin_fmaf(g.hf, f.z, s.vz);
}
__device__ __forceinline__ void drift(State<PREC_FP32> &s, const IntegDev &g)
{
    s.x = __builtin_fmaf(g.dtf, s.vx, s.x);
    s.y = __builtin_fmaf(g.dtf, s.vy, s.y);
    s.z = __builtin_fmaf(g.dtf, s.vz, s.z);
}

struct DsForce { dsf x, y, z; };
__device__ __forceinline__ void kick(State<PREC_DS> &s, const DsForce &f, const IntegDev &g)
{
    dsf h = {g.h_hi, g.h_lo};
    s.vx = ds_add(s.vx, ds_mul(f.x, h));
    s.vy = ds_add(s.vy, ds_mul(f.y, h));
    s.vz = ds_add(s.vz, ds_mul(f.z, h));
}
__device__ __forceinline__ void drift(State<PREC_DS> &s, const IntegDev &g)
{
    dsf dt = {g.dt_hi, g.dt_lo};
    s.x = ds_add(s.x, ds_mul(s.vx, dt));
    s.y = ds_add(s.y, ds_mul(s.vy, dt));
    s.z = ds_add(s.z, ds_mul(s.vz, dt));
}

__device__ __forceinline__ void kickd(StateD &s, double fx, double fy, double fz, const IntegDev &g)
{
    s.vx = __builtin_fma(g.h, fx, s.vx);
    s.vy = __builtin_fma(g.h, fy, s.vy);
    s.vz = __builtin_fma(g.h, fz, s.vz);
}
__device__ __forceinline__ void driftd(StateD &s, const IntegDev &g)
{
    s.x = __builtin_fma(g.dt, s.vx, s.x);
    s.y = __builtin_fma(g.dt, s.vy, s.y);
    s.z = __builtin_fma(g.dt, s.vz, s.z);
}

// Fixed-point snapshot of a state's position.
__device__ __forceinline__ uint4 snap_of(const State<PREC_FP32> &s, const RepDev &r, uint32_t w)
{
    return make_uint4(to_fixed((double)s.x, r.fxs), to_fixed((double)s.y, r.fxs), to_fixed((double)s.z, r.fxs), w);
}
__device__ __forceinline__ uint4 snap_of(const State<PREC_DS> &s, const RepDev &r, uint32_t w)
{
    return make_uint4(to_fixed(ds_to_double(s.x), r.fxs), to_fixed(ds_to_double(s.y), r.fxs),
                      to_fixed(ds_to_double(s.z), r.fxs), w);
}
__device__ __forceinline__ uint4 snap_of(const StateD &s, const RepDev &r, uint32_t w)
{
    return make_uint4(to_fixed(s.x, r.fxs), to_fixed(s.y, r.fxs), to_fixed(s.z, r.fxs), w);
}

// ------------------------------------------------ pair constants per lane
// Scaled units: separations in fixed-point units u = L / 2^32.  With
// r2s = r^2 / u^2 the pair term needs rc^2/u^2, sigma^2/u^2 and 24 eps / u.
struct LaneConsts {
    float rc2s[2], sig2s[2], e24s[2];
};

__device__ __forceinline__ LaneConsts lane_consts(const PairDev &pp, int si, const RepDev &r)
{
    LaneConsts c;
    double u = (double)r.sc;
    double iu2 = 1.0 / (u * u);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        int t = si * 2 + b;
        c.rc2s[b] = (float)(pp.rc2d[t] * iu2);
        c.sig2s[b] = (float)(pp.sig2d[t] * iu2);
        c.e24s[b] = (float)(pp.eps24d[t] / u);
    }
    return c;
}

// The Verlet list of particle i is stored in blocks of four entries:
// entry k lives in int4 row k/4, lane k%4, of column i (nbr4[(k/4)*P + i]),
// so one dwordx4 load fetches four indices and a wave reads 1 KB contiguous.
typedef int v4i __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int4 list_row(const KArena &A, int i, int q)
{
    const v4i *p = (const v4i *)A.nbr + (size_t)q * A.P + i;
    v4i v = __builtin_nontemporal_load(p); // streamed once per step: keep it out of the caches
    return make_int4(v.x, v.y, v.z, v.w);
}

// One list entry, fixed-point snapshots, FP32 pair term.  With a uniform
// cutoff ratio (rc_ab = c sigma_ab for every pair) the cutoff test is
// sigma^2/r^2 > 1/c^2 and needs no per-pair cutoff.
template <int P, bool EN, bool UNI>
__device__ __forceinline__ void entry_fixed(uint4 xi, uint4 xj, const LaneConsts &c, const PairDev &pp,
                                            int si, FAcc<P> &acc, double &e_sum, double &w_sum)
{
    const int ix = (int)(xi.x - xj.x), iy = (int)(xi.y - xj.y), iz = (int)(xi.z - xj.z);
    const float dx = (float)ix, dy = (float)iy, dz = (float)iz;
    const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    const bool b = (xj.w & SPECIES_MASK) != 0;
    const float sig2 = b ? c.sig2s[1] : c.sig2s[0];
    const float e24 = b ? c.e24s[1] : c.e24s[0];
    const float ir2 = __builtin_amdgcn_rcpf(r2);
    const float s2 = sig2 * ir2;
    const float s6 = s2 * s2 * s2;
    const float t = __builtin_fmaf(2.0f, s6, -1.0f);
    float fs = e24 * ir2 * s6 * t;
    bool in;
    if (UNI) in = s2 > pp.s2cut;
    else in = r2 < (b ? c.rc2s[1] : c.rc2s[0]);
    fs = in ? fs : 0.0f;
    acc.add(fs, dx, dy, dz, ix, iy, iz);
    if (EN) {
        const int tt = si * 2 + (b ? 1 : 0);
        if (in) {
            e_sum += 0.5 * ((double)(pp.eps4[tt] * s6 * (s6 - 1.0f)) - (double)pp.shift[tt]);
            w_sum += 0.5 * (double)(pp.eps24[tt] * s6 * t);
        }
    }
}

// Snapshot gather with a 32-bit byte offset from a uniform base.
__device__ __forceinline__ uint4 ld_snap(const uint4 *__restrict__ snap, int j)
{
    return *(const uint4 *)((const char *)snap + (uint32_t)j * 16u);
}

// Force (and optionally energy/virial) on particle i from its list.  The
// loop is software-pipelined over blocks of four entries with two register
// buffers: while one block is computed, the snapshots of the next block and
// the indices of the block after it are in flight.  Lists are padded to a
// multiple of eight valid entries by the list build and row indices are clamped, so every
// prefetch is unconditional and no control-flow join forces the memory
// counters to drain inside the loop.
template <int P, bool EN, bool UNI>
__device__ __forceinline__ void force_fixed(const KArena &A, const uint4 *__restrict__ snap, int i,
                                            uint4 xi, const LaneConsts &c, const PairDev &pp, int si,
                                            FAcc<P> &acc, double &e_sum, double &w_sum, int sub, int lpp)
{
    const int cnt = A.nbr_cnt[i];
    const int nq = ((cnt + 7) >> 3) << 1; // blocks of four, padded to an even count
    acc.init();
    const int npair = nq >> 1;            // this lane takes pairs sub, sub + lpp, ...
    if (sub >= npair) return;
    const int last = nq - 1;
    int p = sub;
    // indices two blocks ahead, snapshots one block ahead
    int4 ja = list_row(A, i, 2 * p), jb = list_row(A, i, 2 * p + 1);
    uint4 a0 = ld_snap(snap, ja.x), a1 = ld_snap(snap, ja.y), a2 = ld_snap(snap, ja.z),
          a3 = ld_snap(snap, ja.w);
    ja = list_row(A, i, min(2 * (p + lpp), last));
    for (; p < npair; p += lpp) {
        // (the scheduling barriers keep each batch of loads ahead of the
        // block computed while it is in flight)
        const uint4 b0 = ld_snap(snap, jb.x), b1 = ld_snap(snap, jb.y), b2 = ld_snap(snap, jb.z),
                    b3 = ld_snap(snap, jb.w);
        jb = list_row(A, i, min(2 * (p + lpp) + 1, last));
        __builtin_amdgcn_sched_barrier(0);
        entry_fixed<P, EN, UNI>(xi, a0, c, pp, si, acc, e_sum, w_sum);
        entry_fixed<P, EN, UNI>(xi, a1, c, pp, si, acc, e_sum, w_sum);
        entry_fixed<P, EN, UNI>(xi, a2, c, pp, si, acc, e_sum, w_sum);
        entry_fixed<P, EN, UNI>(xi, a3, c, pp, si, acc, e_sum, w_sum);
        __builtin_amdgcn_sched_barrier(0);
        a0 = ld_snap(snap, ja.x);
        a1 = ld_snap(snap, ja.y);
        a2 = ld_snap(snap, ja.z);
        a3 = ld_snap(snap, ja.w);
        ja = list_row(A, i, min(2 * (p + 2 * lpp), last));
        __builtin_amdgcn_sched_barrier(0);
        entry_fixed<P, EN, UNI>(xi, b0, c, pp, si, acc, e_sum, w_sum);
        entry_fixed<P, EN, UNI>(xi, b1, c, pp, si, acc, e_sum, w_sum);
        entry_fixed<P, EN, UNI>(xi, b2, c, pp, si, acc, e_sum, w_sum);
        entry_fixed<P, EN, UNI>(xi, b3, c, pp, si, acc, e_sum, w_sum);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// FP64 path: double snapshots, textbook minimum image, FP64 pair term.
__device__ __forceinline__ void force_dbl(const KArena &A, const uint4 *__restrict__ snap, int i,
                                          double xi, double yi, double zi, int si, const RepDev &r,
                                          const PairDev &pp, double &fx, double &fy, double &fz,
                                          bool en, double &e_sum, double &w_sum, int sub, int lpp)
{
    const int cnt = A.nbr_cnt[i];
    const size_t P_ = (size_t)A.P;
    const uint4 *__restrict__ snap1 = snap + P_;
    fx = fy = fz = 0.0;
    double rc2[2], sig2[2], e24[2];
    rc2[0] = pp.rc2d[si * 2]; rc2[1] = pp.rc2d[si * 2 + 1];
    sig2[0] = pp.sig2d[si * 2]; sig2[1] = pp.sig2d[si * 2 + 1];
    e24[0] = pp.eps24d[si * 2]; e24[1] = pp.eps24d[si * 2 + 1];
    const int nq = ((cnt + 7) >> 3) << 1;
    for (int q = sub; q < nq; q += lpp) {
        const int4 jj = list_row(A, i, q);
        const int js[4] = {jj.x, jj.y, jj.z, jj.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = js[u]; // padding entries lie beyond the cutoff
            double xj, yj, zj, wj;
            u4_to_dbl2(snap[j], xj, yj);
            u4_to_dbl2(snap1[j], zj, wj);
            double dx = xi - xj, dy = yi - yj, dz = zi - zj;
            dx -= r.L * rint(dx * r.invL);
            dy -= r.L * rint(dy * r.invL);
            dz -= r.L * rint(dz * r.invL);
            double r2 = dx * dx + dy * dy + dz * dz;
            int b = meta_of_bits(wj) & 1;
            double ir2 = 1.0 / r2;
            double s2 = sig2[b] * ir2;
            double s6 = s2 * s2 * s2;
            double ff = e24[b] * ir2 * s6 * (2.0 * s6 - 1.0);
            bool in = r2 < rc2[b];
            ff = in ? ff : 0.0;
            fx += ff * dx;
            fy += ff * dy;
            fz += ff * dz;
            if (en && in) {
                int tt = si * 2 + b;
                e_sum += 0.5 * (pp.eps4d[tt] * s6 * (s6 - 1.0) - pp.shiftd[tt]);
                w_sum += 0.5 * ff * r2;
            }
        }
    }
}

// ------------------------------------------------------------ k_step
enum { M_ADV = 0, M_FIN = 1, M_IDLE = 2 };

template <int P, bool OBS, bool UNI, int LPP>
__global__ void __launch_bounds__(1024) k_step(const StepArgs a)
{
    const KArena &A = a.A;
    const int nblk = gridDim.x;
    const int blk = remap_block(blockIdx.x, nblk, a.xcd);
    const int gid = blk * blockDim.x + threadIdx.x;
    const int i = gid / LPP;   // LPP adjacent lanes share particle i
    const int sub = gid % LPP;
    constexpr int NS = Traits<P>::NS;

    if (!OBS) { // clear the other parity's cell counters and rebuild list (read
                // by the previous step's rebuild)
        const int gt = blockIdx.x * blockDim.x + threadIdx.x;
        for (int c = gt; c < a.cell_cap; c += nblk * blockDim.x) a.count_other[c] = 0;
        if (gt == 0) a.rlist_other[0] = 0;
    }
    if (i >= A.P) return;

    uint4 s0 = a.snap_cur[i];
    uint4 s1;
    uint32_t meta;
    if (NS == 2) {
        s1 = a.snap_cur[(size_t)A.P + i];
        double zz, ww;
        u4_to_dbl2(s1, zz, ww);
        meta = meta_of_bits(ww);
    } else {
        meta = s0.w;
    }
    if (meta == NO_SLOT) return;
    const int r = slot_of_meta(meta);
    if (r >= a.max_slots) return;
    const Ctl ctl = a.ctl_cur[r];
    if (!ctl.z) return;
    const RepDev rp = a.rep[r];
    int mode;
    if (OBS) {
        mode = M_FIN;
    } else {
        const int tgt = a.target[r];
        mode = ctl.x < tgt ? M_ADV : (ctl.y ? M_IDLE : M_FIN);
        if (i == rp.off && sub == 0) { // the replica's first particle owns its control words
            Ctl nx = ctl;
            if (mode == M_ADV) { nx.x = ctl.x + 1; nx.y = 0; }
            else nx.y = 1;
            a.ctl_next[r] = nx;
            a.need_other[r] = 0;
        }
        if (mode == M_IDLE) {
            if (sub == 0) {
                a.snap_next[i] = s0;
                if (NS == 2) a.snap_next[(size_t)A.P + i] = s1;
            }
            return;
        }
    }
    const int si = (int)(meta & SPECIES_MASK);
    double e_sum = 0.0, w_sum = 0.0;
    double fxd, fyd, fzd;

    State<P> st;
    st.load(A, i);

    if constexpr (P == PREC_FP64) {
        double xi, yi, zi, wi;
        u4_to_dbl2(s0, xi, yi);
        u4_to_dbl2(s1, zi, wi);
        force_dbl(A, a.snap_cur, i, xi, yi, zi, si, rp, a.pp, fxd, fyd, fzd, OBS, e_sum, w_sum, sub, LPP);
#pragma unroll
        for (int m = 1; m < LPP; m <<= 1) {
            lane_sum(fxd, m); lane_sum(fyd, m); lane_sum(fzd, m);
            if (OBS) { lane_sum(e_sum, m); lane_sum(w_sum, m); }
        }
        if (sub != 0) return;
        if (OBS) {
            double *o = a.obs + (size_t)i * 8;
            o[0] = fxd; o[1] = fyd; o[2] = fzd; o[3] = e_sum; o[4] = w_sum;
            o[5] = st.vx; o[6] = st.vy; o[7] = st.vz;
            return;
        }
        if (!ctl.y) kickd(st, fxd, fyd, fzd, a.ig);
        if (mode == M_ADV) {
            kickd(st, fxd, fyd, fzd, a.ig);
            driftd(st, a.ig);
        }
    } else {
        const LaneConsts c = lane_consts(a.pp, si, rp);
        FAcc<P> acc;
        force_fixed<P, OBS, UNI>(A, a.snap_cur, i, s0, c, a.pp, si, acc, e_sum, w_sum, sub, LPP);
        // combine the lanes' partial sums (a no-op for one lane per particle)
        DsForce F;
        if constexpr (P == PREC_DS) F = {acc.x.result(), acc.y.result(), acc.z.result()};
#pragma unroll
        for (int m = 1; m < LPP; m <<= 1) {
            if constexpr (P == PREC_DS) { lane_sum(F.x, m); lane_sum(F.y, m); lane_sum(F.z, m); }
            else { lane_sum(acc.x, m); lane_sum(acc.y, m); lane_sum(acc.z, m); }
            if (OBS) { lane_sum(e_sum, m); lane_sum(w_sum, m); }
        }
        if (sub != 0) return;
        if (OBS) {
            if constexpr (P == PREC_DS) { fxd = ds_to_double(F.x); fyd = ds_to_double(F.y); fzd = ds_to_double(F.z); }
            else acc.get(fxd, fyd, fzd);
            double *o = a.obs + (size_t)i * 8;
            o[0] = fxd; o[1] = fyd; o[2] = fzd; o[3] = e_sum; o[4] = w_sum;
            double vx, vy, vz;
            if constexpr (P == PREC_FP32) { vx = st.vx; vy = st.vy; vz = st.vz; }
            else if constexpr (P == PREC_DS) { vx = ds_to_double(st.vx); vy = ds_to_double(st.vy); vz = ds_to_double(st.vz); }
            else { vx = st.vx; vy = st.vy; vz = st.vz; }
            o[5] = vx; o[6] = vy; o[7] = vz;
            return;
        }
        if constexpr (P == PREC_FP32) {
            if (!ctl.y) kick(st, acc, a.ig);
            if (mode == M_ADV) { kick(st, acc, a.ig); drift(st, a.ig); }
        } else if constexpr (P == PREC_DS) {
            if (!ctl.y) kick(st, F, a.ig);
            if (mode == M_ADV) { kick(st, F, a.ig); drift(st, a.ig); }
        } else { // MIXED64: FP64 sum of FP32 pair terms
            fxd = acc.x; fyd = acc.y; fzd = acc.z;
            if (!ctl.y) kickd(st, fxd, fyd, fzd, a.ig);
            if (mode == M_ADV) { kickd(st, fxd, fyd, fzd, a.ig); driftd(st, a.ig); }
        }
    }
    st.store(A, i);
    if (mode != M_ADV) { // finalised: positions unchanged
        a.snap_next[i] = s0;
        if (NS == 2) a.snap_next[(size_t)A.P + i] = s1;
        return;
    }

    // new snapshot, displacement test, cell count
    int cell;
    bool far, bad;
    if constexpr (P == PREC_FP64) {
        double w = bits_of_meta(meta);
        a.snap_next[i] = dbl2_to_u4(st.x, st.y);
        a.snap_next[(size_t)A.P + i] = dbl2_to_u4(st.z, w);
        double rx, ry, rz, rw;
        u4_to_dbl2(A.xref[i], rx, ry);
        u4_to_dbl2(A.xref[(size_t)A.P + i], rz, rw);
        double dx = st.x - rx, dy = st.y - ry, dz = st.z - rz;
        dx -= rp.L * rint(dx * rp.invL);
        dy -= rp.L * rint(dy * rp.invL);
        dz -= rp.L * rint(dz * rp.invL);
        far = dx * dx + dy * dy + dz * dz > a.pp.hs2d;
        bad = !isfinite(st.x + st.y + st.z);
        cell = dbl_cell(st.x, st.y, st.z, rp.L, rp.invL, rp.nd);
    } else {
        uint4 X = snap_of(st, rp, meta);
        a.snap_next[i] = X;
        uint4 R = A.xref[i];
        float dx = (float)(int)(X.x - R.x), dy = (float)(int)(X.y - R.y), dz = (float)(int)(X.z - R.z);
        float d2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
        float thr = (float)(a.pp.hs2d / ((double)rp.sc * (double)rp.sc));
        far = d2 > thr;
        if constexpr (P == PREC_FP32) bad = !isfinite(st.x + st.y + st.z);
        else if constexpr (P == PREC_DS) bad = !isfinite(st.x.hi + st.y.hi + st.z.hi);
        else bad = !isfinite(st.x + st.y + st.z);
        cell = rp.nd == 1 ? 0 : fixed_cell(X.x, X.y, X.z, rp.nd);
    }
    atomicAdd(a.count_cur + rp.coff + cell, 1);
    if (far && atomicOr(a.need_cur + r, 1) == 0) { // first to flag: enlist the slot
        const int k = atomicAdd(a.rlist_cur, 1);
        a.rlist_cur[1 + k] = r;
    }
    if (bad) atomicOr(a.status + r, 2);
}

// ------------------------------------------------------------ k_count
// Cell counts for a rebuild forced from the host (md_rebuild_neighbours).
template <int P>
__global__ void k_count(const CountArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.P) return;
    constexpr int NS = Traits<P>::NS;
    uint4 s0 = a.snap[i];
    uint32_t meta;
    double x = 0, y = 0, z = 0, w = 0;
    if (NS == 2) {
        u4_to_dbl2(s0, x, y);
        u4_to_dbl2(a.snap[(size_t)a.P + i], z, w);
        meta = meta_of_bits(w);
    } else meta = s0.w;
    if (meta == NO_SLOT) return;
    int r = slot_of_meta(meta);
    if (r >= a.max_slots) return;
    if (!slot_selected(r, a.force_slot, nullptr, a.ctl)) return;
    RepDev rp = a.rep[r];
    int cell;
    if (NS == 2) cell = dbl_cell(x, y, z, rp.L, rp.invL, rp.nd);
    else cell = rp.nd == 1 ? 0 : fixed_cell(s0.x, s0.y, s0.z, rp.nd);
    atomicAdd(a.count + rp.coff + cell, 1);
}

// ------------------------------------------------------------ k_scan
// One workgroup (1024 threads) per slot: exclusive scan of the cell counts
// in tiles of 8 cells per thread, cell starts written as absolute slots.
__global__ void __launch_bounds__(1024) k_scan(const ScanArgs a)
{
    int s = blockIdx.x;
    if (a.force_slot == -1) {
        if (s >= a.rlist[0]) return;
        s = a.rlist[1 + s];
    } else {
        if (s >= a.max_slots) return;
        if (!slot_selected(s, a.force_slot, a.need, a.ctl)) return;
    }
    const RepDev rp = a.rep[s];
    const int ncell = rp.nd * rp.nd * rp.nd;
    const int B = blockDim.x, t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6, nw = (B + 63) >> 6;
    const int *cnt = a.count + rp.coff;
    int *out = a.cs_new + rp.coff;
    __shared__ int wsum[16];
    __shared__ int tile_total;
    int carry = 0;
    for (int base = 0; base < ncell; base += 8 * B) {
        int v[8];
        int local = 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int c = base + 8 * t + u;
            v[u] = c < ncell ? cnt[c] : 0;
            local += v[u];
        }
        int incl = local;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int w = __shfl_up(incl, o, 64);
            if (lane >= o) incl += w;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        if (t == 0) {
            int acc = 0;
            for (int k = 0; k < nw; ++k) { const int w = wsum[k]; wsum[k] = acc; acc += w; }
            tile_total = acc;
        }
        __syncthreads();
        int run = rp.off + carry + wsum[wv] + incl - local;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int c = base + 8 * t + u;
            if (c < ncell) out[c] = run;
            run += v[u];
        }
        carry += tile_total;
        __syncthreads();
    }
    if (t == 0) {
        out[ncell] = rp.off + carry;
        if (carry != rp.n) atomicOr(a.status + s, 4 | 2);
        a.nreb[s] += 1;
    }
}

// ------------------------------------------------------------ k_permute
// One wave per new cell: stable scatter of its members into scratch.  Each
// pass first loads every member it moves, then folds and stores them: on
// this hardware one counter tracks loads and stores alike, so a load issued
// after a store would also wait for that store.
template <int P> struct Moved {
    uint4 st[Traits<P>::NW];
    int4 meta;
    uint4 snap; // the snapshot (fixed point), or its second word (double)
};

template <int P>
__device__ __forceinline__ void move_load(const PermArgs &a, int q, Moved<P> &mv)
{
    constexpr int NW = Traits<P>::NW, NS = Traits<P>::NS;
#pragma unroll
    for (int w = 0; w < NW; ++w) mv.st[w] = a.A.st[w][q];
    mv.meta = a.A.meta[q];
    mv.snap = NS == 1 ? a.snap[q] : a.snap[(size_t)a.A.P + q];
}

__device__ __forceinline__ float4 u4_as_f4(uint4 u)
{
    return make_float4(__uint_as_float(u.x), __uint_as_float(u.y), __uint_as_float(u.z), __uint_as_float(u.w));
}
__device__ __forceinline__ uint4 f4_as_u4(float4 f)
{
    return make_uint4(__float_as_uint(f.x), __float_as_uint(f.y), __float_as_uint(f.z), __float_as_uint(f.w));
}

// Fold the member's position into [0, L) (counting the image shift in its
// meta word) and store it at scratch slot dst.
template <int P>
__device__ __forceinline__ void move_store(const PermArgs &a, const RepDev &rp, const Moved<P> &mv, int dst)
{
    constexpr int NS = Traits<P>::NS;
    int4 m = mv.meta;
    int ix = 0, iy = 0, iz = 0;
    int *im[3] = {&ix, &iy, &iz};
    if constexpr (P == PREC_FP32) {
        float4 p = u4_as_f4(mv.st[0]);
        float *c[3] = {&p.x, &p.y, &p.z};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (*c[d] < 0.0f) { *c[d] += rp.Lf; *im[d] -= 1; }
            if (*c[d] >= rp.Lf) { *c[d] -= rp.Lf; *im[d] += 1; }
        }
        a.sc_st[0][dst] = f4_as_u4(p);
        a.sc_st[1][dst] = mv.st[1];
    } else if constexpr (P == PREC_DS) {
        const float4 w0 = u4_as_f4(mv.st[0]), w1 = u4_as_f4(mv.st[1]);
        dsf x = {w0.x, w0.w}, y = {w0.y, w1.x}, z = {w0.z, w1.y};
        const dsf L = {rp.L_hi, rp.L_lo};
        dsf *c[3] = {&x, &y, &z};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (c[d]->hi < 0.0f) { *c[d] = ds_add(*c[d], L); *im[d] -= 1; }
            const dsf t = ds_sub(*c[d], L);
            if (t.hi >= 0.0f) { *c[d] = t; *im[d] += 1; }
        }
        a.sc_st[0][dst] = f4_as_u4(make_float4(x.hi, y.hi, z.hi, x.lo));
        a.sc_st[1][dst] = f4_as_u4(make_float4(y.lo, z.lo, w1.z, w1.w));
        a.sc_st[2][dst] = mv.st[2];
    } else {
        double x, y, z, w;
        u4_to_dbl2(mv.st[0], x, y);
        u4_to_dbl2(mv.st[1], z, w);
        double *c[3] = {&x, &y, &z};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (*c[d] < 0.0) { *c[d] += rp.L; *im[d] -= 1; }
            if (*c[d] >= rp.L) { *c[d] -= rp.L; *im[d] += 1; }
        }
        a.sc_st[0][dst] = dbl2_to_u4(x, y);
        a.sc_st[1][dst] = dbl2_to_u4(z, w);
        a.sc_st[2][dst] = mv.st[2];
        if constexpr (NS == 2) { // the double snapshot, from the folded state
            double zz, ww;
            u4_to_dbl2(mv.snap, zz, ww);
            a.sc_snap[dst] = dbl2_to_u4(x, y);
            a.sc_snap[(size_t)a.A.P + dst] = dbl2_to_u4(z, ww);
        }
    }
    m.x += ix; m.y += iy; m.z += iz;
    a.sc_meta[dst] = m;
    if constexpr (NS == 1) a.sc_snap[dst] = mv.snap;
}

template <int P>
__device__ __forceinline__ bool in_cell(const PermArgs &a, const RepDev &rp, int q, int c)
{
    constexpr int NS = Traits<P>::NS;
    if (NS == 2) {
        double x, y, z, w;
        u4_to_dbl2(a.snap[q], x, y);
        u4_to_dbl2(a.snap[(size_t)a.A.P + q], z, w);
        return dbl_cell(x, y, z, rp.L, rp.invL, rp.nd) == c;
    }
    const uint4 X = a.snap[q];
    return fixed_cell(X.x, X.y, X.z, rp.nd) == c;
}

template <int P>
__global__ void __launch_bounds__(256) k_permute(const PermArgs a)
{
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int wv = threadIdx.x >> 6;
    __shared__ int pref[4][28], pst[4][27];
    for_items(a.rlist, a.items_pref, a.rep, a.max_slots, a.force_slot, a.ctl, 3,
              blockIdx.x * wpb + wv, gridDim.x * wpb, [&](int s, int c) {
        const RepDev rp = a.rep[s];
        const int nd = rp.nd;
        const int *cs = a.cs + rp.coff;
        const int dst0 = a.cs_new[rp.coff + c];
        const int want = a.cs_new[rp.coff + c + 1] - dst0;
        // the old cells that can hold members of new cell c, ascending (so
        // that the flattened candidates are in old slot order)
        int nold = 1;
        if (lane == 0) { pst[wv][0] = cs[0]; pref[wv][0] = 0; pref[wv][1] = cs[1] - cs[0]; }
        if (nd > 1) {
            nold = 27;
            const int cx = c % nd, cy = (c / nd) % nd, cz = c / (nd * nd);
            int v[3][3] = {{(cx + nd - 1) % nd, cx, (cx + 1) % nd},
                           {(cy + nd - 1) % nd, cy, (cy + 1) % nd},
                           {(cz + nd - 1) % nd, cz, (cz + 1) % nd}};
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                int *u = v[d];
                if (u[0] > u[1]) { int t = u[0]; u[0] = u[1]; u[1] = t; }
                if (u[1] > u[2]) { int t = u[1]; u[1] = u[2]; u[2] = t; }
                if (u[0] > u[1]) { int t = u[0]; u[0] = u[1]; u[1] = t; }
            }
            int len = 0, st0 = 0;
            if (lane < 27) {
                const int kx = lane % 3, ky = (lane / 3) % 3, kz = lane / 9;
                const int oc = v[0][kx] + nd * (v[1][ky] + nd * v[2][kz]);
                st0 = cs[oc];
                len = cs[oc + 1] - st0;
            }
            int incl = len;
#pragma unroll
            for (int o = 1; o < 32; o <<= 1) {
                const int u = __shfl_up(incl, o, 64);
                if (lane >= o) incl += u;
            }
            if (lane < 27) { pst[wv][lane] = st0; pref[wv][lane + 1] = incl; }
            if (lane == 0) pref[wv][0] = 0;
        }
        __builtin_amdgcn_wave_barrier();
        const int tot = pref[wv][nold];
        int run = 0;
        int r = 0; // old cell of the lane's current candidate (only moves forward)
        constexpr int U = 4; // candidates per lane per pass
        for (int b = 0; b < tot; b += 64 * U) {
            int q[U];
            bool m[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = b + 64 * u + lane;
                q[u] = -1;
                if (e < tot) {
                    while (r + 1 < nold && pref[wv][r + 1] <= e) ++r;
                    q[u] = pst[wv][r] + (e - pref[wv][r]);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) m[u] = q[u] >= 0 && (nd == 1 || in_cell<P>(a, rp, q[u], c));
            Moved<P> mv[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (m[u]) move_load<P>(a, q[u], mv[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const unsigned long long bal = __ballot(m[u]);
                if (m[u]) move_store<P>(a, rp, mv[u], dst0 + run + __popcll(bal & ((1ull << lane) - 1ull)));
                run += __popcll(bal);
            }
        }
        // every particle counted in this cell must have come from a
        // neighbouring old cell; a shortfall means a particle jumped further
        if (lane == 0 && run != want) atomicOr(a.status + s, 4);
        __builtin_amdgcn_wave_barrier();
    });
}

// ------------------------------------------------------------ k_build
// One workgroup per row segment of cells (cells x0..x1-1 of row (y, z)):
// the 9 neighbouring rows over x0-1..x1 are staged in LDS, then every member
// writes its list in the canonical order.
#define BUILD_LDS_CAP 3072 // staged candidates (x 16 B = 48 KB, fixed point)
#define BUILD_MAX_NX 18    // cells per staged row (width + 2 halo)
#define BUILD_TAB (9 * BUILD_MAX_NX)

struct BuildTabs {
    int start[BUILD_TAB]; // LDS start of staged cell (global start when not staged)
    int cnt[BUILD_TAB];
    int glob[BUILD_TAB];  // global start of the cell
    int4 pk[BUILD_TAB];   // (start, cnt, glob) of each staged cell, for the grouped scan
    int run_lds[19], run_glob[19];
    int nruns, total, fits, NX;
};

template <int P, bool FROM_LDS>
__device__ __forceinline__ void build_member(const BuildArgs &a, const RepDev &rp, int i, int lx_m,
                                             const BuildTabs &T, bool full, const uint4 *cand, int s,
                                             int nd)
{
    constexpr int NS = Traits<P>::NS;
    const KArena &A = a.A;
    const size_t P_ = (size_t)A.P;
    const int NX = T.NX;
    uint4 xi = a.src_x[i];
    double xd = 0, yd = 0, zd = 0, wd = 0;
    uint32_t meta;
    if (NS == 2) {
        u4_to_dbl2(xi, xd, yd);
        u4_to_dbl2(a.src_x[P_ + i], zd, wd);
        meta = meta_of_bits(wd);
    } else meta = xi.w;
    const int si = (int)(meta & SPECIES_MASK);
    float rl2s0, rl2s1;
    double rl2d0 = a.pp.rl2d[si * 2], rl2d1 = a.pp.rl2d[si * 2 + 1];
    {
        const double u = (double)rp.sc;
        rl2s0 = (float)(rl2d0 / (u * u));
        rl2s1 = (float)(rl2d1 / (u * u));
    }
    const int cap = A.cap;
    // entry k of slot i: int4 row k/4, lane k%4 (see list_row)
    int *col = A.nbr_w + 4 * (size_t)i;
    const size_t row_stride = 4 * P_;
    int cnt = 0;
    int *wp = col; // where entry cnt goes
    auto test = [&](int e, int st) -> bool {
        if (NS == 2) {
            double xj, yj, zj, wj;
            if (FROM_LDS) {
                u4_to_dbl2(cand[2 * (st + e)], xj, yj);
                u4_to_dbl2(cand[2 * (st + e) + 1], zj, wj);
            } else {
                u4_to_dbl2(a.src_x[st + e], xj, yj);
                u4_to_dbl2(a.src_x[P_ + st + e], zj, wj);
            }
            double dx = xd - xj, dy = yd - yj, dz = zd - zj;
            dx -= rp.L * rint(dx * rp.invL);
            dy -= rp.L * rint(dy * rp.invL);
            dz -= rp.L * rint(dz * rp.invL);
            const double r2 = dx * dx + dy * dy + dz * dz;
            return r2 < ((meta_of_bits(wj) & 1) ? rl2d1 : rl2d0);
        }
        const uint4 xj = FROM_LDS ? cand[st + e] : a.src_x[st + e];
        const float dx = (float)(int)(xi.x - xj.x), dy = (float)(int)(xi.y - xj.y),
                    dz = (float)(int)(xi.z - xj.z);
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
        return r2 < ((xj.w & SPECIES_MASK) ? rl2s1 : rl2s0);
    };
    // Candidates of one cell in slot order; accepted ones are stored at once
    // (a predicated 4-byte store).  `self` is the candidate index of i in
    // this cell, or -1.
    auto put = [&](bool acc, int j) {
        if (acc) {
            if (cnt < cap) *wp = j;
            ++cnt;
            wp += (cnt & 3) ? 1 : (ptrdiff_t)row_stride - 3;
        }
    };
    // four candidates per iteration: independent reads and tests in flight
    // (the scan is a dependent chain per member), stores in slot order
    auto scan_cell = [&](int k, int self) {
        const int st = T.start[k], n = T.cnt[k], g0 = T.glob[k];
        int e = 0;
        for (; e + 4 <= n; e += 4) {
            const bool c0 = test(e, st), c1 = test(e + 1, st), c2 = test(e + 2, st), c3 = test(e + 3, st);
            put(c0 && e != self, g0 + e);
            put(c1 && e + 1 != self, g0 + e + 1);
            put(c2 && e + 2 != self, g0 + e + 2);
            put(c3 && e + 3 != self, g0 + e + 3);
        }
        for (; e < n; ++e) put(test(e, st) && e != self, g0 + e);
    };
    int last_cell = 0;
    if (nd == 1) {
        scan_cell(0, i - T.glob[0]);
    } else {
        // own cell, then each half-space offset o followed by -o: in the
        // (dz, dy, dx) enumeration of the 27 offsets the positive half space
        // is indices 14..26
        auto cell_k = [&](int dx, int dy, int dz) {
            int lx = lx_m + dx;
            if (full) { lx += lx < 0 ? nd : 0; lx -= lx >= nd ? nd : 0; }
            return ((dz + 1) * 3 + (dy + 1)) * NX + lx;
        };
        const int own = cell_k(0, 0, 0);
        scan_cell(own, i - T.glob[own]);
        for (int q = 14; q < 27; ++q) {
            const int dz = q / 9 - 1, dy = (q / 3) % 3 - 1, dx = q % 3 - 1;
            scan_cell(cell_k(dx, dy, dz), -1);
            last_cell = cell_k(-dx, -dy, -dz);
            scan_cell(last_cell, -1);
        }
    }
    // Pad the list to a multiple of 8 with a particle that is outside the
    // list radius at this build: it stays beyond the force cutoff until the
    // next build (each particle moves at most skin/2), so the force loop
    // needs no per-entry validity test.  The pad is the first rejected
    // candidate of the last cell visited (a corner cell), else of any cell.
    if (cnt & 7) {
        int pad = -1;
        {
            const int st = T.start[last_cell], n = T.cnt[last_cell], g0 = T.glob[last_cell];
            for (int e = 0; e < n && pad < 0; ++e)
                if (!test(e, st) && g0 + e != i) pad = g0 + e;
        }
        for (int k = 0; k < (nd == 1 ? 1 : 9 * NX) && pad < 0; ++k) {
            const int st = T.start[k], n = T.cnt[k], g0 = T.glob[k];
            for (int e = 0; e < n && pad < 0; ++e)
                if (!test(e, st) && g0 + e != i) pad = g0 + e;
        }
        if (pad < 0) atomicOr(a.status + s, 8);
        for (int k = cnt; k < ((cnt + 7) & ~7) && k < cap; ++k)
            col[(size_t)(k >> 2) * row_stride + (k & 3)] = pad < 0 ? i : pad;
    }
    A.nbr_cnt_w[i] = cnt < A.cap ? cnt : A.cap;
    if (cnt > A.cap) atomicOr(a.status + s, 1);
}

// The same list, built by a group of G lanes (G a power of two <= 64, the
// group's lanes adjacent in one wave): the member's candidates, concatenated
// in the canonical cell order, are tested G at a time, one per lane, and the
// accepted ones are stored at the running count plus their rank among the
// group's accepted lanes (ballot + popcount), i.e. in exactly the order of
// the one-lane scan.  Splits one member's dependent candidate chain G ways,
// which is what bounds the build of small replicas.
template <int P, bool FROM_LDS>
__device__ __forceinline__ void build_member_grp(const BuildArgs &a, const RepDev &rp, int i, int lx_m,
                                                 const BuildTabs &T, bool full, const uint4 *cand, int s,
                                                 int nd, int G, int gl, unsigned long long gmask,
                                                 unsigned long long below)
{
    constexpr int NS = Traits<P>::NS;
    const KArena &A = a.A;
    const size_t P_ = (size_t)A.P;
    const int NX = T.NX;
    uint4 xi = a.src_x[i];
    double xd = 0, yd = 0, zd = 0, wd = 0;
    uint32_t meta;
    if (NS == 2) {
        u4_to_dbl2(xi, xd, yd);
        u4_to_dbl2(a.src_x[P_ + i], zd, wd);
        meta = meta_of_bits(wd);
    } else meta = xi.w;
    const int si = (int)(meta & SPECIES_MASK);
    float rl2s0, rl2s1;
    double rl2d0 = a.pp.rl2d[si * 2], rl2d1 = a.pp.rl2d[si * 2 + 1];
    {
        const double u = (double)rp.sc;
        rl2s0 = (float)(rl2d0 / (u * u));
        rl2s1 = (float)(rl2d1 / (u * u));
    }
    const int cap = A.cap;
    int *col = A.nbr_w + 4 * (size_t)i;
    const size_t row_stride = 4 * P_;
    auto test = [&](int e, int st) -> bool {
        if (NS == 2) {
            double xj, yj, zj, wj;
            if (FROM_LDS) {
                u4_to_dbl2(cand[2 * (st + e)], xj, yj);
                u4_to_dbl2(cand[2 * (st + e) + 1], zj, wj);
            } else {
                u4_to_dbl2(a.src_x[st + e], xj, yj);
                u4_to_dbl2(a.src_x[P_ + st + e], zj, wj);
            }
            double dx = xd - xj, dy = yd - yj, dz = zd - zj;
            dx -= rp.L * rint(dx * rp.invL);
            dy -= rp.L * rint(dy * rp.invL);
            dz -= rp.L * rint(dz * rp.invL);
            const double r2 = dx * dx + dy * dy + dz * dz;
            return r2 < ((meta_of_bits(wj) & 1) ? rl2d1 : rl2d0);
        }
        const uint4 xj = FROM_LDS ? cand[st + e] : a.src_x[st + e];
        const float dx = (float)(int)(xi.x - xj.x), dy = (float)(int)(xi.y - xj.y),
                    dz = (float)(int)(xi.z - xj.z);
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
        return r2 < ((xj.w & SPECIES_MASK) ? rl2s1 : rl2s0);
    };
    // one cell's candidates, 4G at a time: lane gl tests e = b + u G + gl
    // (u = 0..3, independent loads in flight); the ballots are taken in u
    // order, which is ascending e
    int cnt = 0;
    auto scan_cell = [&](int k) {
        const int4 c = T.pk[k]; // (start, cnt, glob)
        for (int b = 0; b < c.y; b += 4 * G) {
            bool acc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = b + u * G + gl;
                acc[u] = e < c.y && test(e, c.x) && c.z + e != i;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const unsigned long long m = __ballot(acc[u]) & gmask;
                if (acc[u]) {
                    const int k2 = cnt + __popcll(m & below);
                    if (k2 < cap) col[(size_t)(k2 >> 2) * row_stride + (k2 & 3)] = c.z + b + u * G + gl;
                }
                cnt += __popcll(m);
            }
        }
    };
    // visiting order: own cell, then +o, -o for q = 14..26 of the
    // (dz, dy, dx) enumeration of the 27 offsets
    auto cell_k = [&](int dx, int dy, int dz) {
        int lx = lx_m + dx;
        if (full) { lx += lx < 0 ? nd : 0; lx -= lx >= nd ? nd : 0; }
        return ((dz + 1) * 3 + (dy + 1)) * NX + lx;
    };
    int last_cell = 0;
    if (nd == 1) {
        scan_cell(0);
    } else {
        scan_cell(cell_k(0, 0, 0));
        for (int q = 14; q < 27; ++q) {
            const int dz = q / 9 - 1, dy = (q / 3) % 3 - 1, dx = q % 3 - 1;
            scan_cell(cell_k(dx, dy, dz));
            last_cell = cell_k(-dx, -dy, -dz);
            scan_cell(last_cell);
        }
    }
    // pad to a multiple of 8, as in the one-lane build: the first rejected
    // candidate of the last visited cell, else (rare) of any staged cell
    if (cnt & 7) {
        int pad = -1;
        const int4 cl = T.pk[last_cell];
        for (int b = 0; b < cl.y; b += G) {
            const int e = b + gl;
            const bool r = e < cl.y && !test(e, cl.x) && cl.z + e != i;
            const unsigned long long m = __ballot(r) & gmask;
            if (m) { pad = cl.z + b + (__ffsll(m) - 1) - (__ffsll(gmask) - 1); break; }
        }
        if (gl == 0) {
            for (int k = 0; k < (nd == 1 ? 1 : 9 * NX) && pad < 0; ++k) {
                const int st = T.start[k], n = T.cnt[k], g0 = T.glob[k];
                for (int e = 0; e < n && pad < 0; ++e)
                    if (!test(e, st) && g0 + e != i) pad = g0 + e;
            }
            if (pad < 0) atomicOr(a.status + s, 8);
            for (int k = cnt; k < ((cnt + 7) & ~7) && k < cap; ++k)
                col[(size_t)(k >> 2) * row_stride + (k & 3)] = pad < 0 ? i : pad;
        }
    }
    if (gl == 0) {
        A.nbr_cnt_w[i] = cnt < cap ? cnt : cap;
        if (cnt > cap) atomicOr(a.status + s, 1);
    }
}

template <int P>
__device__ __forceinline__ void copy_back(const BuildArgs &a, int i)
{
    constexpr int NW = Traits<P>::NW, NS = Traits<P>::NS;
    const KArena &A = a.A;
    const size_t P_ = (size_t)A.P;
    if (a.from_scratch) {
#pragma unroll
        for (int w = 0; w < NW; ++w) A.st[w][i] = a.sc_st[w][i];
        A.meta[i] = a.sc_meta[i];
#pragma unroll
        for (int w = 0; w < NS; ++w) {
            uint4 x = a.src_x[w * P_ + i];
            a.snap_cur[w * P_ + i] = x;
            A.xref_w[w * P_ + i] = x;
        }
    }
}

template <int P>
__global__ void __launch_bounds__(1024) k_build(const BuildArgs a)
{
    constexpr int NS = Traits<P>::NS;
    __shared__ BuildTabs T;
    extern __shared__ uint4 cand[];
    const int B = blockDim.x, t = threadIdx.x;
    for_items(a.rlist, a.items_pref, a.rep, a.max_slots, a.force_slot, a.ctl, 4,
              remap_block(blockIdx.x, gridDim.x, a.xcd), gridDim.x, [&](int s, int item) {
        const RepDev rp = a.rep[s];
        const int nd = rp.nd;
        const int *cs = a.cs_new + rp.coff;
        int m0, m1, NX = 1, x0 = 0, x1 = 1, rowbase = 0;
        bool full = true;
        if (nd == 1) {
            m0 = rp.off + item * a.single_members;
            m1 = min(m0 + a.single_members, rp.off + rp.n);
            if (t == 0) {
                T.glob[0] = rp.off;
                T.cnt[0] = rp.n;
                T.start[0] = 0;
                T.run_lds[0] = 0; T.run_glob[0] = rp.off; T.run_lds[1] = rp.n;
                T.nruns = 1;
                T.total = rp.n;
                T.fits = rp.n <= a.lds_cap;
                if (!T.fits) T.start[0] = rp.off;
                T.NX = 1;
                if (item == 0 && a.from_scratch) { a.cs[rp.coff] = cs[0]; a.cs[rp.coff + 1] = cs[1]; }
            }
        } else {
            const int W = a.width;
            full = nd <= W + 2;
            const int nseg = full ? 1 : (nd + W - 1) / W;
            const int part = item % rp.bparts, segitem = item / rp.bparts;
            const int seg = segitem % nseg, row = segitem / nseg;
            const int cy = row % nd, cz = row / nd;
            x0 = full ? 0 : (seg * nd) / nseg;           // balanced segments
            x1 = full ? nd : ((seg + 1) * nd) / nseg;
            NX = full ? nd : x1 - x0 + 2;
            rowbase = nd * (cy + nd * cz);
            {   // this item's share of the segment's members
                const int s0 = cs[rowbase + x0], ms = cs[rowbase + x1] - s0;
                m0 = s0 + (int)(((long long)part * ms) / rp.bparts);
                m1 = s0 + (int)(((long long)(part + 1) * ms) / rp.bparts);
            }
            if (a.from_scratch && part == 0) { // retire the old cell starts of this segment
                for (int k = x0 + t; k < x1; k += B) a.cs[rp.coff + rowbase + k] = cs[rowbase + k];
                if (t == 0 && rowbase + x1 == nd * nd * nd)
                    a.cs[rp.coff + nd * nd * nd] = cs[nd * nd * nd];
            }
            const int gs = full ? 0 : (x0 - 1 + nd) % nd; // first staged x
            for (int k = t; k < 9 * NX; k += B) {
                const int rw = k / NX, lx = k - rw * NX;
                const int dz = rw / 3 - 1, dy = rw % 3 - 1;
                int gx = gs + lx;
                gx -= gx >= nd ? nd : 0;
                int gy = cy + dy, gz = cz + dz;
                gy += gy < 0 ? nd : 0; gy -= gy >= nd ? nd : 0;
                gz += gz < 0 ? nd : 0; gz -= gz >= nd ? nd : 0;
                const int cc = gx + nd * (gy + nd * gz);
                T.glob[k] = cs[cc];
                T.cnt[k] = cs[cc + 1] - cs[cc];
            }
            if (t == 0) T.NX = NX;
            __syncthreads();
            if (t < 64) { // exclusive scan of the staged cell sizes (one wave)
                const int ncells = 9 * NX;
                int carry = 0;
                for (int b = 0; b < ncells; b += 64) {
                    const int k = b + t;
                    const int v = k < ncells ? T.cnt[k] : 0;
                    int incl = v;
#pragma unroll
                    for (int o = 1; o < 64; o <<= 1) {
                        const int u = __shfl_up(incl, o, 64);
                        if (t >= o) incl += u;
                    }
                    if (k < ncells) T.start[k] = carry + incl - v;
                    carry += __shfl(incl, 63, 64);
                }
                if (t == 0) { T.total = carry; T.fits = carry <= a.lds_cap; }
            }
            __syncthreads();
            if (t < 9) { // contiguous global runs of each staged row (<= 2 with wrap)
                const int lenA = full ? NX : min(NX, nd - gs);
                const int k0 = t * NX;
                T.run_lds[2 * t] = T.start[k0];
                T.run_glob[2 * t] = T.glob[k0];
                T.run_lds[2 * t + 1] = lenA < NX ? T.start[k0 + lenA] : T.start[k0 + NX - 1] + T.cnt[k0 + NX - 1];
                T.run_glob[2 * t + 1] = lenA < NX ? T.glob[k0 + lenA] : T.glob[k0 + NX - 1] + T.cnt[k0 + NX - 1];
                if (t == 8) { T.run_lds[18] = T.total; T.nruns = 18; }
            }
            __syncthreads();
            if (!T.fits) // candidates are read from the arena: start = global index
                for (int k = t; k < 9 * NX; k += B) T.start[k] = T.glob[k];
        }
        __syncthreads();
        for (int k = t; k < (nd == 1 ? 1 : 9 * NX); k += B) T.pk[k] = make_int4(T.start[k], T.cnt[k], T.glob[k], 0);
        const bool fits = T.fits != 0;
        if (fits) { // stage: element e lies in the last run whose LDS start is <= e
            const int tot = T.total, nr = T.nruns;
            int r = 0; // only moves forward as e grows
            for (int e = t; e < tot; e += B) {
                while (r + 1 < nr && T.run_lds[r + 1] <= e) ++r;
                const int g = T.run_glob[r] + (e - T.run_lds[r]);
                if (NS == 2) {
                    cand[2 * e] = a.src_x[g];
                    cand[2 * e + 1] = a.src_x[(size_t)a.A.P + g];
                } else cand[e] = a.src_x[g];
            }
        }
        __syncthreads();
        // the member's cell: own-row staged cell whose range holds i
        auto member_cell = [&](int i) {
            if (nd == 1) return 0;
            int lx = full ? 0 : 1;
            const int le = full ? NX - 1 : NX - 2;
            while (lx < le && T.glob[4 * NX + lx + 1] <= i) ++lx;
            return lx;
        };
        // lanes per member: the replica's (fixed by the launch, or one lane
        // for large replicas), else the largest power of two that still
        // gives every member of this work item its own group
        int G = rp.blanes;
        if (G == 0) {
            G = 1;
            while (G < 64 && (2 * G) * (m1 - m0) <= B) G *= 2;
        }
        if (G == 1) {
            for (int i = m0 + t; i < m1; i += B) {
                const int lx_m = member_cell(i);
                if (fits) build_member<P, true>(a, rp, i, lx_m, T, full, cand, s, nd);
                else build_member<P, false>(a, rp, i, lx_m, T, full, cand, s, nd);
                copy_back<P>(a, i);
            }
        } else {
            const int lane = t & 63, gl = t & (G - 1);
            const unsigned long long gmask =
                G == 64 ? ~0ull : ((1ull << G) - 1ull) << (lane & ~(G - 1));
            const unsigned long long below = (1ull << lane) - 1ull;
            for (int i = m0 + t / G; i < m1; i += B / G) {
                const int lx_m = member_cell(i);
                if (fits) build_member_grp<P, true>(a, rp, i, lx_m, T, full, cand, s, nd, G, gl, gmask, below);
                else build_member_grp<P, false>(a, rp, i, lx_m, T, full, cand, s, nd, G, gl, gmask, below);
                if (gl == 0) copy_back<P>(a, i);
            }
        }
        __syncthreads();
    });
}

// ------------------------------------------------------------ k_obs_reduce
// Deterministic two-pass FP64 sums per slot of e_i, w_i, v^2, v and the list
// lengths: pass 1 reduces fixed chunks of OBS_CHUNK particles, pass 2 adds
// the chunk partials of each slot in chunk order.
#define OBS_CHUNK 4096
#define OBS_Q 7

__device__ __forceinline__ void block_sum7(double acc[OBS_Q], double (*red)[256])
{
    for (int q = 0; q < OBS_Q; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = blockDim.x >> 1; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < OBS_Q; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_obs_partial(const ObsArgs a)
{
    __shared__ double red[OBS_Q][256];
    const int total = a.chunk_pref[a.max_slots];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        const int s = find_item_slot(a.chunk_pref, a.max_slots, item);
        const RepDev rp = a.rep[s];
        const int k0 = (item - a.chunk_pref[s]) * OBS_CHUNK;
        const int k1 = min(k0 + OBS_CHUNK, rp.n);
        double acc[OBS_Q] = {0, 0, 0, 0, 0, 0, 0};
        for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
            const double *o = a.obs + (size_t)(rp.off + k) * 8;
            acc[0] += o[3];
            acc[1] += o[4];
            acc[2] += o[5] * o[5] + o[6] * o[6] + o[7] * o[7];
            acc[3] += o[5];
            acc[4] += o[6];
            acc[5] += o[7];
            acc[6] += (double)a.nbr_cnt[rp.off + k];
        }
        block_sum7(acc, red);
        if (threadIdx.x < OBS_Q) a.partial[(size_t)item * 8 + threadIdx.x] = red[threadIdx.x][0];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_obs_reduce(const ObsArgs a)
{
    const int s = blockIdx.x;
    if (s >= a.max_slots || !a.ctl[s].z) return;
    __shared__ double red[OBS_Q][256];
    double acc[OBS_Q] = {0, 0, 0, 0, 0, 0, 0};
    const int c0 = a.chunk_pref[s], c1 = a.chunk_pref[s + 1];
    // chunk partials of the slot, in chunk order within each thread's stride
    for (int c = c0 + threadIdx.x; c < c1; c += blockDim.x)
        for (int q = 0; q < OBS_Q; ++q) acc[q] += a.partial[(size_t)c * 8 + q];
    block_sum7(acc, red);
    if (threadIdx.x < OBS_Q) a.out[s * 8 + threadIdx.x] = red[threadIdx.x][0];
}

// ------------------------------------------------------------ k_scale_vel
template <int P>
__global__ void k_scale_vel(const ScaleArgs a)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const int i = a.off + k;
    State<P> st;
    st.load(a.A, i);
    if constexpr (P == PREC_DS) {
        dsf f = {a.f_hi, a.f_lo};
        st.vx = ds_mul(st.vx, f); st.vy = ds_mul(st.vy, f); st.vz = ds_mul(st.vz, f);
    } else if constexpr (P == PREC_FP32) {
        st.vx *= a.ff; st.vy *= a.ff; st.vz *= a.ff;
    } else {
        st.vx *= a.fd; st.vy *= a.fd; st.vz *= a.fd;
    }
    st.store(a.A, i);
}

// ------------------------------------------------------------ k_ds_eval
__global__ void k_ds_eval(int op, long long n, const float *a, const float *b, float *out)
{
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (op == 3) { // compensated sum of a[k].hi, single workgroup, fixed order
        if (blockIdx.x != 0 || threadIdx.x != 0) return;
        sum2f s;
        s.init();
        for (long long q = 0; q < n; ++q) s.add(a[2 * q]);
        dsf r = s.result();
        out[0] = r.hi;
        out[1] = r.lo;
        return;
    }
    if (k >= n) return;
    dsf x = {a[2 * k], a[2 * k + 1]}, y = {b[2 * k], b[2 * k + 1]}, r;
    if (op == 0) r = ds_add(x, y);
    else if (op == 1) r = ds_sub(x, y);
    else r = ds_mul(x, y);
    out[2 * k] = r.hi;
    out[2 * k + 1] = r.lo;
}

// ------------------------------------------------------------ launchers
#define LAUNCH_CHECK() return hipGetLastError()

template <int P, int LPP>
static hipError_t launch_step_l(const StepArgs &a, int block, bool obs, hipStream_t s)
{
    const long long threads = (long long)a.A.P * LPP;
    const int grid = (int)((threads + block - 1) / block);
    const bool uni = a.pp.uniform != 0 && P != PREC_FP64;
    if (obs && uni) hipLaunchKernelGGL((k_step<P, true, true, LPP>), dim3(grid), dim3(block), 0, s, a);
    else if (obs) hipLaunchKernelGGL((k_step<P, true, false, LPP>), dim3(grid), dim3(block), 0, s, a);
    else if (uni) hipLaunchKernelGGL((k_step<P, false, true, LPP>), dim3(grid), dim3(block), 0, s, a);
    else hipLaunchKernelGGL((k_step<P, false, false, LPP>), dim3(grid), dim3(block), 0, s, a);
    LAUNCH_CHECK();
}

template <int P>
static hipError_t launch_step_t(const StepArgs &a, int block, bool obs, hipStream_t s)
{
    if (a.lpp == 4) return launch_step_l<P, 4>(a, block, obs, s);
    if (a.lpp == 2) return launch_step_l<P, 2>(a, block, obs, s);
    return launch_step_l<P, 1>(a, block, obs, s);
}

hipError_t launch_step(int prec, const StepArgs &a, int block, bool obs, hipStream_t s)
{
    switch (prec) {
    case PREC_FP32: return launch_step_t<PREC_FP32>(a, block, obs, s);
    case PREC_DS: return launch_step_t<PREC_DS>(a, block, obs, s);
    case PREC_MIX: return launch_step_t<PREC_MIX>(a, block, obs, s);
    default: return launch_step_t<PREC_FP64>(a, block, obs, s);
    }
}

hipError_t launch_count(int prec, const CountArgs &a, hipStream_t s)
{
    int grid = (a.P + 255) / 256;
    switch (prec) {
    case PREC_FP64: hipLaunchKernelGGL((k_count<PREC_FP64>), dim3(grid), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((k_count<PREC_FP32>), dim3(grid), dim3(256), 0, s, a); break;
    }
    LAUNCH_CHECK();
}

hipError_t launch_scan(const ScanArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan, dim3(a.max_slots), dim3(1024), 0, s, a);
    LAUNCH_CHECK();
}

hipError_t launch_permute(int prec, const PermArgs &a, int grid, hipStream_t s)
{
    switch (prec) {
    case PREC_FP32: hipLaunchKernelGGL((k_permute<PREC_FP32>), dim3(grid), dim3(256), 0, s, a); break;
    case PREC_DS: hipLaunchKernelGGL((k_permute<PREC_DS>), dim3(grid), dim3(256), 0, s, a); break;
    case PREC_MIX: hipLaunchKernelGGL((k_permute<PREC_MIX>), dim3(grid), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((k_permute<PREC_FP64>), dim3(grid), dim3(256), 0, s, a); break;
    }
    LAUNCH_CHECK();
}

hipError_t launch_build(int prec, const BuildArgs &a, int grid, int block, hipStream_t s)
{
    size_t lds = (size_t)a.lds_cap * 16 * (prec == PREC_FP64 ? 2 : 1);
    switch (prec) {
    case PREC_FP32: hipLaunchKernelGGL((k_build<PREC_FP32>), dim3(grid), dim3(block), lds, s, a); break;
    case PREC_DS: hipLaunchKernelGGL((k_build<PREC_DS>), dim3(grid), dim3(block), lds, s, a); break;
    case PREC_MIX: hipLaunchKernelGGL((k_build<PREC_MIX>), dim3(grid), dim3(block), lds, s, a); break;
    default: hipLaunchKernelGGL((k_build<PREC_FP64>), dim3(grid), dim3(block), lds, s, a); break;
    }
    LAUNCH_CHECK();
}

hipError_t launch_obs_reduce(const ObsArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_obs_partial, dim3(1024), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_obs_reduce, dim3(a.max_slots), dim3(256), 0, s, a);
    LAUNCH_CHECK();
}

hipError_t launch_scale_vel(int prec, const ScaleArgs &a, hipStream_t s)
{
    int grid = (a.n + 255) / 256;
    if (grid == 0) return hipSuccess;
    switch (prec) {
    case PREC_FP32: hipLaunchKernelGGL((k_scale_vel<PREC_FP32>), dim3(grid), dim3(256), 0, s, a); break;
    case PREC_DS: hipLaunchKernelGGL((k_scale_vel<PREC_DS>), dim3(grid), dim3(256), 0, s, a); break;
    case PREC_MIX: hipLaunchKernelGGL((k_scale_vel<PREC_MIX>), dim3(grid), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((k_scale_vel<PREC_FP64>), dim3(grid), dim3(256), 0, s, a); break;
    }
    LAUNCH_CHECK();
}

hipError_t launch_ds_eval(int op, long long n, const float *a, const float *b, float *out, hipStream_t s)
{
    long long grid = op == 3 ? 1 : (n + 255) / 256;
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ds_eval, dim3((unsigned)grid), dim3(256), 0, s, op, n, a, b, out);
    LAUNCH_CHECK();
}

// ------------------------------------------------------------ control pokes
// Stream-ordered writes of control words (graph- and capture-safe; no host
// buffers whose lifetime would have to outlast an asynchronous copy).
__global__ void k_add_targets(int *target, const Ctl *ctl, int max_slots, int delta)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < max_slots && ctl[s].z) target[s] += delta;
}

__global__ void k_poke(int *p, int v) { *p = v; }

hipError_t launch_add_targets(int *target, const Ctl *ctl, int max_slots, int delta, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_targets, dim3((max_slots + 255) / 256), dim3(256), 0, s, target, ctl, max_slots, delta);
    LAUNCH_CHECK();
}

hipError_t launch_poke(int *p, int v, hipStream_t s)
{
    hipLaunchKernelGGL(k_poke, dim3(1), dim3(1), 0, s, p, v);
    LAUNCH_CHECK();
}
