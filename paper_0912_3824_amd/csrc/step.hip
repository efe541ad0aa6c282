// The fused force + velocity-Verlet step kernel (k_step) and its launcher.
#include "dev_common.hpp"

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
// r2s = r^2 / u^2 the pair term needs rc^2/u^2, sigma^2/u^2 and 24 eps / u;
// the host precomputes them per replica (RepDev).
struct LaneConsts {
    float rc2s[2], sig2s[2], e24s[2];
    // smoothing (Sec. 4): rc in fixed-point units, u/(h sigma), 1/(h sigma),
    // 4 eps and the energy shift
    float rcs[2], xsc[2], ihs[2], e4[2], sh[2];
    float e24[2]; // 24 eps (unscaled, for the virial)
};

__device__ __forceinline__ LaneConsts lane_consts(const PairDev &pp, int si, const RepDev &r)
{
    // constant indices and selects on si: an index computed from si would
    // put the replica record in scratch memory
    LaneConsts c;
    const bool b1 = si != 0;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        c.rc2s[b] = b1 ? r.rc2s[2 + b] : r.rc2s[b];
        c.sig2s[b] = b1 ? r.sig2s[2 + b] : r.sig2s[b];
        c.e24s[b] = b1 ? r.e24s[2 + b] : r.e24s[b];
        c.rcs[b] = b1 ? r.rcs[2 + b] : r.rcs[b];
        c.xsc[b] = b1 ? r.xsc[2 + b] : r.xsc[b];
        c.ihs[b] = b1 ? r.ihs[2 + b] : r.ihs[b];
        c.e4[b] = b1 ? pp.eps4[2 + b] : pp.eps4[b];
        c.sh[b] = b1 ? pp.shift[2 + b] : pp.shift[b];
        c.e24[b] = b1 ? pp.eps24[2 + b] : pp.eps24[b];
    }
    return c;
}

// Pair kinds of the force loop: plain truncation with a cutoff per species
// pair, plain truncation with one cutoff ratio rc_ab / sigma_ab for every
// pair (the test needs no per-pair cutoff), and the C2-smoothed potential.
enum { PK_GENERAL = 0, PK_UNIFORM = 1, PK_SMOOTH = 2 };

// The Verlet list of particle i is stored in int4 rows of four entries
// (rows in tiles of 64 slots, see list_row_index; which entry sits in which
// row, see list_entry_row), so one dwordx4 load fetches four indices and the
// lanes of a wave read 512 B runs.
typedef int v4i __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int4 list_row(const KArena &A, int i, int q)
{
    const v4i *p = (const v4i *)A.nbr + list_row_index(i, q, A.cap);
    v4i v = __builtin_nontemporal_load(p); // streamed once per step: keep it out of the caches
    return make_int4(v.x, v.y, v.z, v.w);
}

// One list entry, fixed-point snapshots, FP32 pair term.  With a uniform
// cutoff ratio (rc_ab = c sigma_ab for every pair) the cutoff test is
// sigma^2/r^2 > 1/c^2 and needs no per-pair cutoff.  Smoothed (Sec. 4):
// V_s = V_ts g(x), x = (r - rc)/(h sigma), g = x^4/(1+x^4), and
// -dV_s/dr = F g - V_ts g'(x)/(h sigma), g' = 4x^3/(1+x^4)^2.  In fixed-
// point units r' = r/u, so x = (r' - rc/u) u/(h sigma) and the force factor
// per unit of separation gains -V_ts g' / (h sigma r').
template <int P, bool EN, int KIND>
__device__ __forceinline__ void entry_fixed(uint4 xi, uint4 xj, const LaneConsts &c, const PairDev &pp,
                                            int si, FAcc<P> &acc, double &e_sum, double &w_sum)
{
    const int ix = (int)(xi.x - xj.x), iy = (int)(xi.y - xj.y), iz = (int)(xi.z - xj.z);
    const float dx = (float)ix, dy = (float)iy, dz = (float)iz;
    const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
    const bool b = (int)xj.w < 0; // species B (sign bit of the meta word)
    const float sig2 = b ? c.sig2s[1] : c.sig2s[0];
    const float e24 = b ? c.e24s[1] : c.e24s[0];
    const float ir2 = __builtin_amdgcn_rcpf(r2);
    const float s2 = sig2 * ir2;
    const float s6 = s2 * s2 * s2;
    const float t = __builtin_fmaf(2.0f, s6, -1.0f);
    float fs = e24 * ir2 * s6 * t;
    bool in;
    if (KIND == PK_UNIFORM) in = s2 > pp.s2cut;
    else in = r2 < (b ? c.rc2s[1] : c.rc2s[0]);
    float g = 1.0f, vts = 0.0f, dgr = 0.0f;
    if (KIND == PK_SMOOTH) {
        const float irr = __builtin_amdgcn_rsqf(r2); // 1 / r'
        const float rr = r2 * irr;
        const float x = (rr - (b ? c.rcs[1] : c.rcs[0])) * (b ? c.xsc[1] : c.xsc[0]);
        const float x2 = x * x, x4 = x2 * x2;
        const float iden = __builtin_amdgcn_rcpf(1.0f + x4);
        g = x4 * iden;
        const float dg = 4.0f * x2 * x * iden * iden;
        vts = (b ? c.e4[1] : c.e4[0]) * s6 * (s6 - 1.0f) - (b ? c.sh[1] : c.sh[0]);
        dgr = dg * rr * (b ? c.xsc[1] : c.xsc[0]); // r g'(x) / (h sigma)
        fs = fs * g - vts * dg * (b ? c.ihs[1] : c.ihs[0]) * irr;
    }
    fs = in ? fs : 0.0f;
    acc.add(fs, dx, dy, dz, ix, iy, iz);
    if (EN) {
        const float e24u = b ? c.e24[1] : c.e24[0], e4u = b ? c.e4[1] : c.e4[0], shu = b ? c.sh[1] : c.sh[0];
        if (in) {
            if (KIND == PK_SMOOTH) {
                e_sum += 0.5 * (double)(vts * g);
                w_sum += 0.5 * (double)(g * e24u * s6 * t - vts * dgr);
            } else {
                e_sum += 0.5 * ((double)(e4u * s6 * (s6 - 1.0f)) - (double)shu);
                w_sum += 0.5 * (double)(e24u * s6 * t);
            }
        }
    }
}

// Snapshot record at list entry e: a 32-bit byte offset (see list_entry)
// from a uniform base.
__device__ __forceinline__ uint4 ld_snap(const uint4 *__restrict__ snap, int e)
{
    return *(const uint4 *)((const char *)snap + (uint32_t)e);
}

// The list's row count and the first two rows of lane `sub` (the rows
// force_fixed starts with), read before anything else is known of the slot:
// the count and row indices are clamped to the slot's own rows, so the reads
// stay in bounds for every slot of the arena, used or not, and the rows are
// in flight while the replica's control words are read.
struct ListHead { int nq; int4 r0, r1; };
__device__ __forceinline__ ListHead list_head(const KArena &A, int i, int sub, int lpp)
{
    ListHead h;
    const int cnt = min(max(A.nbr_cnt[i], 0), A.cap);
    h.nq = list_rows(cnt, A.lg); // rows of four (a partial group is completed by padding)
    const int last = max(h.nq - 1, 0);
    h.r0 = list_row(A, i, min(sub, last));
    h.r1 = list_row(A, i, min(sub + lpp, last));
    return h;
}

// Force (and optionally energy/virial) on particle i from its list.  Lists
// are padded to four entries per lane and their entries dealt to the lanes
// in turn (list_entry_row): lane `sub` of the particle's `lpp` lanes takes
// rows sub, sub + lpp, sub + 2 lpp, ... of four entries (every lane the same
// number), two of them per iteration of a software-pipelined loop (while one
// block is computed, the snapshots of the next and the indices of the one
// after it are in flight), and an odd last block after it.  Row indices are
// clamped, so every prefetch is unconditional and no control-flow join
// forces the memory counters to drain inside the loop.
template <int P, bool EN, int KIND>
__device__ __forceinline__ void force_fixed(const KArena &A, const uint4 *__restrict__ snap, int i,
                                            uint4 xi, const LaneConsts &c, const PairDev &pp, int si,
                                            FAcc<P> &acc, double &e_sum, double &w_sum, int sub, int lpp,
                                            const ListHead &h)
{
    const int nq = h.nq;
    acc.init();
    if (sub >= nq) return;
    const int last = nq - 1;
    const int nb = (nq - sub + lpp - 1) / lpp; // this lane's blocks
    auto row = [&](int k) { return list_row(A, i, min(sub + k * lpp, last)); };
    // block k's snapshots in a, indices of block k+1 in jb and of k+2 in ja
    int4 ja = h.r0, jb = h.r1;
    uint4 a0 = ld_snap(snap, ja.x), a1 = ld_snap(snap, ja.y), a2 = ld_snap(snap, ja.z), a3 = ld_snap(snap, ja.w);
    ja = row(2);
    int k = 0;
    for (; k + 1 < nb; k += 2) {
        // (the scheduling barriers keep each batch of loads ahead of the
        // block computed while it is in flight)
        const uint4 b0 = ld_snap(snap, jb.x), b1 = ld_snap(snap, jb.y), b2 = ld_snap(snap, jb.z),
                    b3 = ld_snap(snap, jb.w);
        jb = row(k + 3);
        __builtin_amdgcn_sched_barrier(0);
        entry_fixed<P, EN, KIND>(xi, a0, c, pp, si, acc, e_sum, w_sum);
        entry_fixed<P, EN, KIND>(xi, a1, c, pp, si, acc, e_sum, w_sum);
        entry_fixed<P, EN, KIND>(xi, a2, c, pp, si, acc, e_sum, w_sum);
        entry_fixed<P, EN, KIND>(xi, a3, c, pp, si, acc, e_sum, w_sum);
        __builtin_amdgcn_sched_barrier(0);
        a0 = ld_snap(snap, ja.x);
        a1 = ld_snap(snap, ja.y);
        a2 = ld_snap(snap, ja.z);
        a3 = ld_snap(snap, ja.w);
        ja = row(k + 4);
        __builtin_amdgcn_sched_barrier(0);
        entry_fixed<P, EN, KIND>(xi, b0, c, pp, si, acc, e_sum, w_sum);
        entry_fixed<P, EN, KIND>(xi, b1, c, pp, si, acc, e_sum, w_sum);
        entry_fixed<P, EN, KIND>(xi, b2, c, pp, si, acc, e_sum, w_sum);
        entry_fixed<P, EN, KIND>(xi, b3, c, pp, si, acc, e_sum, w_sum);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (k < nb) { // an odd last block, already loaded
        entry_fixed<P, EN, KIND>(xi, a0, c, pp, si, acc, e_sum, w_sum);
        entry_fixed<P, EN, KIND>(xi, a1, c, pp, si, acc, e_sum, w_sum);
        entry_fixed<P, EN, KIND>(xi, a2, c, pp, si, acc, e_sum, w_sum);
        entry_fixed<P, EN, KIND>(xi, a3, c, pp, si, acc, e_sum, w_sum);
    }
}

// FP64 path: double snapshots, textbook minimum image, FP64 pair term
// (smoothed as in entry_fixed when SMOOTH).
template <bool SMOOTH>
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
    const int nq = list_rows(cnt, A.lg); // rows of four (a partial group is completed by padding)
    for (int q = sub; q < nq; q += lpp) {
        const int4 jj = list_row(A, i, q);
        const int js[4] = {jj.x, jj.y, jj.z, jj.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = list_slot(js[u]); // padding entries lie beyond the cutoff
            double xj, yj, zj, wj;
            u4_to_dbl2(snap[j], xj, yj);
            u4_to_dbl2(snap1[j], zj, wj);
            double dx = xi - xj, dy = yi - yj, dz = zi - zj;
            dx -= r.L * rint(dx * r.invL);
            dy -= r.L * rint(dy * r.invL);
            dz -= r.L * rint(dz * r.invL);
            double r2 = dx * dx + dy * dy + dz * dz;
            int b = species_of(meta_of_bits(wj));
            double ir2 = 1.0 / r2;
            double s2 = sig2[b] * ir2;
            double s6 = s2 * s2 * s2;
            double ff = e24[b] * ir2 * s6 * (2.0 * s6 - 1.0);
            bool in = r2 < rc2[b];
            double vs = 0.0;
            if (en || SMOOTH) {
                const int tt = si * 2 + b;
                vs = pp.eps4d[tt] * s6 * (s6 - 1.0) - pp.shiftd[tt];
                if (SMOOTH) {
                    const double r = sqrt(r2);
                    const double x = (r - pp.rcd[tt]) / pp.hsd[tt];
                    const double x2 = x * x, x4 = x2 * x2;
                    const double g = x4 / (1.0 + x4);
                    const double dg = 4.0 * x2 * x / ((1.0 + x4) * (1.0 + x4));
                    ff = ff * g - vs * dg / pp.hsd[tt] / r;
                    vs *= g;
                }
            }
            ff = in ? ff : 0.0;
            fx += ff * dx;
            fy += ff * dy;
            fz += ff * dz;
            if (en && in) {
                e_sum += 0.5 * vs;
                w_sum += 0.5 * ff * r2;
            }
        }
    }
}

// ------------------------------------------------------------ k_step
enum { M_ADV = 0, M_FIN = 1, M_IDLE = 2 };

template <int P, bool OBS, int KIND, int LPP>
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

    // reads that depend on the slot alone, issued before the replica's
    // control words are known (in bounds for every slot of the arena)
    State<P> st;
    st.load(A, i);
    ListHead lh;
    if constexpr (P != PREC_FP64) lh = list_head(A, i, sub, LPP);

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
        // A replica with an error bit (a list that overflowed its capacity
        // or could not be padded, lost particles, a non-finite position)
        // stops where it is: no step runs on a truncated list.
        const bool halted = (a.status[r] & ST_HALT) != 0;
        mode = halted ? M_IDLE : (ctl.x < tgt ? M_ADV : (ctl.y ? M_IDLE : M_FIN));
        if (i == rp.off && sub == 0) { // the replica's first particle owns its control words
            Ctl nx = ctl;
            if (mode == M_ADV) { nx.x = ctl.x + 1; nx.y = 0; nx.w = 0; }
            else if (!halted) { nx.y = 1; if (mode == M_FIN) nx.w = 1; }
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
    const int si = species_of(meta);
    double e_sum = 0.0, w_sum = 0.0;
    double fxd, fyd, fzd;
    // A step that starts from a finalising launch's state reuses the forces
    // it stored (ctl.w): same positions, same lists, the same bits a new
    // force pass would give.
    const bool stored = !OBS && mode == M_ADV && ctl.y && ctl.w;
    const double *ost = a.obs + (size_t)i * 8;

    // With a curve cell order, read the rank of the particle's current cell
    // now, off the critical path: a particle usually stays in its cell, and
    // the table is read again at the end only when the cell changed.
    int cell0 = -1, rank0 = 0;
    if (!OBS && rp.curve) {
        if constexpr (P == PREC_FP64) {
            double x0, y0, z0, w0;
            u4_to_dbl2(s0, x0, y0);
            u4_to_dbl2(s1, z0, w0);
            cell0 = dbl_cell(x0, y0, z0, rp.L, rp.invL, rp.nd);
        } else cell0 = fixed_cell(s0.x, s0.y, s0.z, rp.nd);
        rank0 = a.corder[rp.coff + cell0];
    }

    if constexpr (P == PREC_FP64) {
        double xi, yi, zi, wi;
        u4_to_dbl2(s0, xi, yi);
        u4_to_dbl2(s1, zi, wi);
        if (stored) {
            if (sub != 0) return;
            fxd = ost[0]; fyd = ost[1]; fzd = ost[2];
        } else {
            force_dbl<KIND == PK_SMOOTH>(A, a.snap_cur, i, xi, yi, zi, si, rp, a.pp, fxd, fyd, fzd, OBS, e_sum,
                                         w_sum, sub, LPP);
#pragma unroll
            for (int m = 1; m < LPP; m <<= 1) {
                lane_sum(fxd, m); lane_sum(fyd, m); lane_sum(fzd, m);
                if (OBS) { lane_sum(e_sum, m); lane_sum(w_sum, m); }
            }
        }
        if (sub != 0) return;
        if (OBS) {
            double *o = a.obs + (size_t)i * 8;
            o[0] = fxd; o[1] = fyd; o[2] = fzd; o[3] = e_sum; o[4] = w_sum;
            o[5] = st.vx; o[6] = st.vy; o[7] = st.vz;
            return;
        }
        if (mode == M_FIN) { // keep the forces for the next step
            double *o = a.obs + (size_t)i * 8;
            o[0] = fxd; o[1] = fyd; o[2] = fzd;
        }
        if (!ctl.y) kickd(st, fxd, fyd, fzd, a.ig);
        if (mode == M_ADV) {
            kickd(st, fxd, fyd, fzd, a.ig);
            driftd(st, a.ig);
        }
    } else {
        FAcc<P> acc;
        DsForce F;
        if (stored) { // each stored word holds its force bit for bit
            if (sub != 0) return;
            if constexpr (P == PREC_DS) F = {ds_unpack(ost[0]), ds_unpack(ost[1]), ds_unpack(ost[2])};
            else if constexpr (P == PREC_FP32) { acc.x = (float)ost[0]; acc.y = (float)ost[1]; acc.z = (float)ost[2]; }
            else { acc.x = ost[0]; acc.y = ost[1]; acc.z = ost[2]; }
        } else {
            const LaneConsts c = lane_consts(a.pp, si, rp);
            force_fixed<P, OBS, KIND>(A, a.snap_cur, i, s0, c, a.pp, si, acc, e_sum, w_sum, sub, LPP, lh);
            // combine the lanes' partial sums (a no-op for one lane per particle)
            if constexpr (P == PREC_DS) F = {acc.x.result(), acc.y.result(), acc.z.result()};
#pragma unroll
            for (int m = 1; m < LPP; m <<= 1) {
                if constexpr (P == PREC_DS) { lane_sum(F.x, m); lane_sum(F.y, m); lane_sum(F.z, m); }
                else { lane_sum(acc.x, m); lane_sum(acc.y, m); lane_sum(acc.z, m); }
                if (OBS) { lane_sum(e_sum, m); lane_sum(w_sum, m); }
            }
        }
        if (sub != 0) return;
        if (mode == M_FIN && !OBS) { // keep the forces for the next step
            double *o = a.obs + (size_t)i * 8;
            // double-single: both words (hi + lo need not fit one double);
            // FP32 and FP64 sums convert exactly
            if constexpr (P == PREC_DS) { o[0] = ds_pack(F.x); o[1] = ds_pack(F.y); o[2] = ds_pack(F.z); }
            else { o[0] = acc.x; o[1] = acc.y; o[2] = acc.z; }
        }
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

    // new snapshot, displacement test (with the lower threshold of an
    // aligned rebuild step when the pool sets one), cell count
    int cell;
    bool far, bad;
    const bool aligned = a.pp.align_every > 0 && (ctl.x + 1) % a.pp.align_every == 0;
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
        far = dx * dx + dy * dy + dz * dz > (aligned ? a.pp.hs2d_early : a.pp.hs2d);
        bad = !isfinite(st.x + st.y + st.z);
        cell = dbl_cell(st.x, st.y, st.z, rp.L, rp.invL, rp.nd);
    } else {
        uint4 X = snap_of(st, rp, meta);
        a.snap_next[i] = X;
        uint4 R = A.xref[i];
        float dx = (float)(int)(X.x - R.x), dy = (float)(int)(X.y - R.y), dz = (float)(int)(X.z - R.z);
        float d2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
        far = d2 > (aligned ? rp.hs2s_early : rp.hs2s);
        if constexpr (P == PREC_FP32) bad = !isfinite(st.x + st.y + st.z);
        else if constexpr (P == PREC_DS) bad = !isfinite(st.x.hi + st.y.hi + st.z.hi);
        else bad = !isfinite(st.x + st.y + st.z);
        cell = rp.nd == 1 ? 0 : fixed_cell(X.x, X.y, X.z, rp.nd);
    }
    const int rank = cell == cell0 ? rank0 : cell_rank(cell, rp, a.corder);
    // Count the particle in its new cell.  The wave's particles are sorted by
    // cell, so most of its lanes count into one or two cells: one lane per
    // distinct cell adds the number of lanes with that cell, instead of
    // every lane contending for the same counter.
    int *ctr = a.count_cur + rp.coff + sort_key(rank, meta, rp.planes, rp.nd);
    for (unsigned long long todo = __ballot(1); todo;) {
        const int leader = __ffsll((long long)todo) - 1;
        int *lc = (int *)__shfl((long long)ctr, leader, 64);
        const unsigned long long same = __ballot(lc == ctr);
        if (__lane_id() == leader) atomicAdd(lc, __popcll(same));
        todo &= ~same;
    }
    if (far && atomicOr(a.need_cur + r, 1) == 0) { // first to flag: enlist the slot
        const int k = atomicAdd(a.rlist_cur, 1);
        a.rlist_cur[1 + k] = r;
    }
    if (bad) atomicOr(a.status + r, 2);
}

// ------------------------------------------------------------ launcher
template <int P, int LPP>
static hipError_t launch_step_l(const StepArgs &a, int block, bool obs, hipStream_t s)
{
    const long long threads = (long long)a.A.P * LPP;
    const int grid = (int)((threads + block - 1) / block);
    if (a.pp.smooth) {
        if (obs) hipLaunchKernelGGL((k_step<P, true, PK_SMOOTH, LPP>), dim3(grid), dim3(block), 0, s, a);
        else hipLaunchKernelGGL((k_step<P, false, PK_SMOOTH, LPP>), dim3(grid), dim3(block), 0, s, a);
        LAUNCH_CHECK();
    }
    if constexpr (P != PREC_FP64) {
        if (a.pp.uniform) {
            if (obs) hipLaunchKernelGGL((k_step<P, true, PK_UNIFORM, LPP>), dim3(grid), dim3(block), 0, s, a);
            else hipLaunchKernelGGL((k_step<P, false, PK_UNIFORM, LPP>), dim3(grid), dim3(block), 0, s, a);
            LAUNCH_CHECK();
        }
    }
    if (obs) hipLaunchKernelGGL((k_step<P, true, PK_GENERAL, LPP>), dim3(grid), dim3(block), 0, s, a);
    else hipLaunchKernelGGL((k_step<P, false, PK_GENERAL, LPP>), dim3(grid), dim3(block), 0, s, a);
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
