// Neighbour-list rebuild kernels (cell count, scan, stable sort, list build)
// and their launchers.
#include "dev_common.hpp"

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
    atomicAdd(a.count + rp.coff + sort_key(cell_rank(cell, rp, a.corder), meta, rp.planes, rp.nd), 1);
}

// ------------------------------------------------------------ k_scan
// One workgroup (1024 threads) per slot: exclusive scan of the cell counts
// (every species plane, in order), cell starts written as absolute slots.
// Tiles of SCAN_CPT x 1024 cells pass through LDS, so that global reads and
// writes are coalesced while each thread scans SCAN_CPT consecutive cells.
#define SCAN_CPT 8
#define SCAN_B 1024
__global__ void __launch_bounds__(SCAN_B) k_scan(const ScanArgs a)
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
    const int ncell = rp.planes * rp.nd * rp.nd * rp.nd;
    const int t = threadIdx.x;
    const int lane = t & 63, wv = t >> 6, nw = SCAN_B >> 6;
    const int *cnt = a.count + rp.coff;
    int *out = a.cs_new + rp.coff;
    __shared__ int tile[SCAN_CPT * SCAN_B];
    __shared__ int wsum[SCAN_B / 64];
    __shared__ int tile_total;
    int carry = 0;
    for (int base = 0; base < ncell; base += SCAN_CPT * SCAN_B) {
#pragma unroll
        for (int u = 0; u < SCAN_CPT; ++u) {
            const int c = base + u * SCAN_B + t;
            tile[u * SCAN_B + t] = c < ncell ? cnt[c] : 0;
        }
        __syncthreads();
        int v[SCAN_CPT];
        int local = 0;
#pragma unroll
        for (int u = 0; u < SCAN_CPT; ++u) {
            v[u] = tile[SCAN_CPT * t + u];
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
        for (int u = 0; u < SCAN_CPT; ++u) {
            tile[SCAN_CPT * t + u] = run;
            run += v[u];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < SCAN_CPT; ++u) {
            const int c = base + u * SCAN_B + t;
            if (c < ncell) out[c] = tile[u * SCAN_B + t];
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
// One wave per new cell: stable scatter of its members into scratch, in two
// phases.  The test phase reads the snapshots of the candidates (the members
// of the 27 neighbouring old cells, in old slot order) PERM_U x 64 at a time,
// all in flight together, and lists each member found with its destination
// in LDS; it issues no store.  The move phase then loads the listed members
// and folds and stores them.  A cell's membership is thus found in a few
// round trips to memory instead of one load-then-store pass per 256
// candidates (on this hardware one counter tracks loads and stores alike, so
// a load issued after a store also waits for that store).
#define PERM_U 8                     // candidate tests per lane in flight
#define PERM_LIST (64 + 64 * PERM_U) // listed members per wave before a move phase
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
        for (int d = 0; d < 3; ++d) { // fold by the exact edge (the box need not be a float)
            if (*c[d] < 0.0f) { *c[d] = (float)((double)*c[d] + rp.L); *im[d] -= 1; }
            if ((double)*c[d] >= rp.L) { *c[d] = (float)((double)*c[d] - rp.L); *im[d] += 1; }
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

// The sort waits on chains of memory round trips rather than on issue, so in
// double-single and FP64 it is compiled for 6 waves per SIMD (at most 80
// VGPRs, no spills) instead of the 4 its unconstrained register use allows;
// its grid takes one full residency at that occupancy.  The FP32 and
// MIXED64 forms would spill at 80 VGPRs and keep their own allocation.
template <int P>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu((P == PREC_DS || P == PREC_FP64) ? 6 : 1))) k_permute(const PermArgs a)
{
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    const int wv = threadIdx.x >> 6;
    __shared__ int pref[4][55], pst[4][54], srt[4][27];
    __shared__ int2 lst[4][PERM_LIST]; // (old slot, scratch slot) of the members found
    for_items(a.rlist, a.items_pref, a.rep, a.max_slots, a.force_slot, a.ctl, 3,
              blockIdx.x * wpb + wv, gridDim.x * wpb, [&](int s, int c) {
        const RepDev rp = a.rep[s];
        const int nd = rp.nd, nc = nd * nd * nd, planes = rp.planes;
        const int *cs = a.cs + rp.coff;
        // new cell c of every plane: plane-0 members go to [dst0, dst0 +
        // want0), plane-1 members to [dst1, dst1 + want1)
        const int rc = cell_rank(c, rp, a.corder);
        const int dst0 = a.cs_new[rp.coff + rc], want0 = a.cs_new[rp.coff + rc + 1] - dst0;
        const int dst1 = planes > 1 ? a.cs_new[rp.coff + nc + rc] : 0;
        const int want1 = planes > 1 ? a.cs_new[rp.coff + nc + rc + 1] - dst1 : 0;
        // the old cells that can hold members of new cell c, in ascending
        // rank: plane 0's, then plane 1's (so that the flattened candidates
        // are in old slot order); one range per lane
        const int nold = nd == 1 ? 1 : 27, nr = planes * nold;
        if (nd > 1) { // rank the 27 neighbour cells (distinct for nd >= 3)
            int orank = 0x7fffffff;
            if (lane < 27) {
                const int cx = c % nd, cy = (c / nd) % nd, cz = c / (nd * nd);
                int ox = cx + lane % 3 - 1, oy = cy + (lane / 3) % 3 - 1, oz = cz + lane / 9 - 1;
                ox += ox < 0 ? nd : 0; ox -= ox >= nd ? nd : 0;
                oy += oy < 0 ? nd : 0; oy -= oy >= nd ? nd : 0;
                oz += oz < 0 ? nd : 0; oz -= oz >= nd ? nd : 0;
                orank = cell_rank(ox + nd * (oy + nd * oz), rp, a.corder);
            }
            int pos = 0;
            for (int l = 0; l < 27; ++l) pos += __shfl(orank, l, 64) < orank;
            if (lane < 27) srt[wv][pos] = orank;
            __builtin_amdgcn_wave_barrier();
        }
        int len = 0, st0 = 0;
        if (lane < nr) {
            const int pl = lane >= nold, kk = lane - pl * nold;
            const int oc = pl * nc + (nd > 1 ? srt[wv][kk] : 0);
            st0 = cs[oc];
            len = cs[oc + 1] - st0;
        }
        int incl = len;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int u = __shfl_up(incl, o, 64);
            if (lane >= o) incl += u;
        }
        if (lane < nr) { pst[wv][lane] = st0; pref[wv][lane + 1] = incl; }
        if (lane == 0) pref[wv][0] = 0;
        __builtin_amdgcn_wave_barrier();
        const int tot = pref[wv][nr], tot0 = pref[wv][nold];
        // move phase: every listed member, loaded before any is stored
        auto move_listed = [&](int n) {
            __builtin_amdgcn_wave_barrier();
            for (int k = lane; k < n; k += 64) {
                const int2 e = lst[wv][k];
                Moved<P> mv;
                move_load<P>(a, e.x, mv);
                move_store<P>(a, rp, mv, e.y);
            }
            __builtin_amdgcn_wave_barrier();
        };
        int run0 = 0, run1 = 0, nl = 0;
        int r = 0; // range of the lane's current candidate (only moves forward)
        const unsigned long long below = (1ull << lane) - 1ull;
        for (int b = 0; b < tot; b += 64 * PERM_U) {
            int q[PERM_U];
            bool m[PERM_U];
#pragma unroll
            for (int u = 0; u < PERM_U; ++u) {
                const int e = b + 64 * u + lane;
                q[u] = -1;
                if (e < tot) {
                    while (r + 1 < nr && pref[wv][r + 1] <= e) ++r;
                    q[u] = pst[wv][r] + (e - pref[wv][r]);
                }
            }
#pragma unroll
            for (int u = 0; u < PERM_U; ++u) m[u] = q[u] >= 0 && (nd == 1 || in_cell<P>(a, rp, q[u], c));
            // list the members found, in candidate order (at most 64 x
            // PERM_U, so the list, emptied below once it holds more than
            // 64, never overflows)
#pragma unroll
            for (int u = 0; u < PERM_U; ++u) {
                const bool p1 = b + 64 * u + lane >= tot0;
                const unsigned long long bal0 = __ballot(m[u] && !p1), bal1 = __ballot(m[u] && p1);
                if (m[u]) {
                    const int dst = p1 ? dst1 + run1 + __popcll(bal1 & below) : dst0 + run0 + __popcll(bal0 & below);
                    lst[wv][nl + __popcll((bal0 | bal1) & below)] = make_int2(q[u], dst);
                }
                run0 += __popcll(bal0);
                run1 += __popcll(bal1);
                nl += __popcll(bal0 | bal1);
            }
            if (nl > PERM_LIST - 64 * PERM_U) { move_listed(nl); nl = 0; }
        }
        move_listed(nl);
        // every particle counted in this cell must have come from a
        // neighbouring old cell; a shortfall means a particle jumped further
        if (lane == 0 && (run0 != want0 || run1 != want1)) atomicOr(a.status + s, 4);
    });
}

// ------------------------------------------------------------ k_build
// One workgroup per row segment of cells (cells x0..x1-1 of row (y, z)):
// the 9 neighbouring rows over x0-1..x1 are staged in LDS, each cell's
// plane-0 members followed by its plane-1 members, then every member of the
// segment (of either plane) writes its list in the canonical order: the own
// cell, then each half-space offset o followed by -o, and within each cell
// the A members before the B members, in slot order.
#define BUILD_LDS_CAP 3072 // staged candidates (x 16 B = 48 KB, fixed point)
#define BUILD_MAX_NX 18    // cells per staged row (width + 2 halo)
#define BUILD_TAB (9 * BUILD_MAX_NX)

struct BuildTabs {
    // staged cell k = row * NX + lx: (LDS start of its members, members of
    // both planes, global start in plane 0, global start in plane 1)
    int4 pk[BUILD_TAB];
    int na[BUILD_TAB]; // members in plane 0
    int mp[2 * BUILD_MAX_NX + 1]; // member prefix: own-row cells' plane-0 members, then plane-1
    int ncell, total, fits, NX, own0, nown;
};

// Candidate e of a staged cell: plane-0 member e, else plane-1 member e - na
// (its global slot), and where it is read from (LDS, or the arena when the
// neighbourhood did not fit).
__device__ __forceinline__ int cand_glob(const int4 &c, int na, int e) { return e < na ? c.z + e : c.w + (e - na); }
template <bool FROM_LDS>
__device__ __forceinline__ int cand_at(const int4 &c, int na, int e) { return FROM_LDS ? c.x + e : cand_glob(c, na, e); }

// Staged cell of the v-th visit (v = 0..26) of a member in staged column
// lx_m: the own cell, then each half-space offset o followed by -o, where
// the half space is indices 14..26 of the (dz, dy, dx) enumeration of the 27
// offsets (odd v: +o, even v: -o).
__device__ __forceinline__ int visit_cell(int v, int lx_m, bool full, int nd, int NX)
{
    int dx = 0, dy = 0, dz = 0;
    if (v > 0) {
        const int q = 14 + ((v - 1) >> 1);
        const int sg = (v & 1) ? 1 : -1;
        dz = sg * (q / 9 - 1);
        dy = sg * ((q / 3) % 3 - 1);
        dx = sg * (q % 3 - 1);
    }
    int lx = lx_m + dx;
    if (full) { lx += lx < 0 ? nd : 0; lx -= lx >= nd ? nd : 0; }
    return ((dz + 1) * 3 + (dy + 1)) * NX + lx;
}

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
    const int si = species_of(meta);
    float rl2s0, rl2s1;
    double rl2d0 = a.pp.rl2d[si * 2], rl2d1 = a.pp.rl2d[si * 2 + 1];
    {
        const double u = (double)rp.sc;
        rl2s0 = (float)(rl2d0 / (u * u));
        rl2s1 = (float)(rl2d1 / (u * u));
    }
    const int cap = A.cap;
    // entry k of slot i: int4 row list_entry_row(k), column list_entry_col(k)
    int *col = A.nbr_w + 4 * list_row_index(i, 0, cap);
    const size_t row_stride = 4 * LIST_TILE;
    const int lg = A.lg, lm = (1 << lg) - 1, gm = (4 << lg) - 1;
    int cnt = 0;
    // a candidate's snapshot (two words for double snapshots) at staged
    // index x (a global slot when nothing is staged), then the test
    struct Cand { uint4 a, b; };
    auto load = [&](int x) -> Cand {
        Cand q;
        if (NS == 2) {
            q.a = FROM_LDS ? cand[2 * x] : a.src_x[x];
            q.b = FROM_LDS ? cand[2 * x + 1] : a.src_x[P_ + x];
        } else {
            q.a = FROM_LDS ? cand[x] : a.src_x[x];
            q.b = q.a;
        }
        return q;
    };
    auto eval = [&](const Cand &q) -> bool {
        if (NS == 2) {
            double xj, yj, zj, wj;
            u4_to_dbl2(q.a, xj, yj);
            u4_to_dbl2(q.b, zj, wj);
            double dx = xd - xj, dy = yd - yj, dz = zd - zj;
            dx -= rp.L * rint(dx * rp.invL);
            dy -= rp.L * rint(dy * rp.invL);
            dz -= rp.L * rint(dz * rp.invL);
            const double r2 = dx * dx + dy * dy + dz * dz;
            return r2 < (species_of(meta_of_bits(wj)) ? rl2d1 : rl2d0);
        }
        const uint4 xj = q.a;
        const float dx = (float)(int)(xi.x - xj.x), dy = (float)(int)(xi.y - xj.y),
                    dz = (float)(int)(xi.z - xj.z);
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
        return r2 < (((int)xj.w < 0) ? rl2s1 : rl2s0);
    };
    // The candidates of staged cell k in order (i itself is skipped).  Each
    // chunk of up to 64 (32 when staged) candidates is tested four at a
    // time (independent reads in flight, no stores and no branches in the
    // test loop: a wave would otherwise run the store path whenever any of
    // its lanes accepts) into an acceptance mask, whose set bits are then
    // stored in order.
    //
    // Staged candidates are read at fixed offsets from the chunk's start,
    // past the cell's end too (into the next cell's records or the padding
    // that follows the staged array): those tests are masked off once per
    // chunk instead of clamping every read.  The list is written through a
    // running pointer to entry cnt.
    int *wp = col; // entry cnt (see list_entry_row): the next lane's row, else
                   // the next column of the first lane's row, else the next group
    auto put = [&](int g) {
        if (cnt < cap) *wp = list_entry(g);
        ++cnt;
        wp += (cnt & lm) ? (ptrdiff_t)row_stride : (cnt & gm) ? 1 - (ptrdiff_t)lm * (ptrdiff_t)row_stride
                                                                : (ptrdiff_t)row_stride - 3;
    };
    auto scan_cell = [&](int k) {
        const int4 c = T.pk[k];
        const int na = T.na[k], n = c.y;
        auto at = [&](int e) { return cand_at<FROM_LDS>(c, na, e); };
        const int self = (unsigned)(i - c.z) < (unsigned)na ? i - c.z
                       : (unsigned)(i - c.w) < (unsigned)(n - na) ? na + (i - c.w) : -1;
        if constexpr (FROM_LDS) {
            const uint4 *cp = cand + NS * c.x; // the cell's staged records
            for (int base = 0; base < n; base += 32) {
                unsigned mask = 0;
                for (int e = 0; e < n - base; e += 4) {
                    const uint4 *q = cp + NS * (base + e);
                    const Cand q0 = {q[0], q[NS - 1]}, q1 = {q[NS], q[2 * NS - 1]},
                               q2 = {q[2 * NS], q[3 * NS - 1]}, q3 = {q[3 * NS], q[4 * NS - 1]};
                    const unsigned bits = (eval(q0) ? 1u : 0u) | (eval(q1) ? 2u : 0u) | (eval(q2) ? 4u : 0u) |
                                          (eval(q3) ? 8u : 0u);
                    mask |= bits << e;
                    if (e == 28) break; // a full chunk of 32
                }
                const int m = n - base;
                if (m < 32) mask &= (1u << m) - 1u;
                if ((unsigned)(self - base) < 32u) mask &= ~(1u << (self - base));
                while (mask) {
                    const int b = __ffs(mask) - 1;
                    mask &= mask - 1u;
                    put(cand_glob(c, na, base + b));
                }
            }
            return;
        }
        for (int base = 0; base < n; base += 64) {
            const int m = min(64, n - base), last = base + m - 1;
            unsigned long long mask = 0;
            for (int e = 0; e < m; e += 4) {
                // past the chunk's end: re-test its last candidate, masked off
                const Cand q0 = load(at(base + e)), q1 = load(at(min(base + e + 1, last))),
                           q2 = load(at(min(base + e + 2, last))), q3 = load(at(min(base + e + 3, last)));
                const bool c0 = eval(q0);
                const bool c1 = eval(q1) && e + 1 < m;
                const bool c2 = eval(q2) && e + 2 < m;
                const bool c3 = eval(q3) && e + 3 < m;
                const unsigned bits = (unsigned)c0 | ((unsigned)c1 << 1) | ((unsigned)c2 << 2) | ((unsigned)c3 << 3);
                mask |= (unsigned long long)bits << e;
            }
            if (self >= base && self < base + 64) mask &= ~(1ull << (self - base));
            while (mask) {
                const int b = __ffsll((long long)mask) - 1;
                mask &= mask - 1;
                put(cand_glob(c, na, base + b));
            }
        }
    };
    // own cell, then each half-space offset o followed by -o (see
    // visit_cell), as one loop: a single copy of the scan code
    const int nvis = nd == 1 ? 1 : 27;
#pragma unroll 1
    for (int v = 0; v < nvis; ++v) scan_cell(nd == 1 ? 0 : visit_cell(v, lx_m, full, nd, NX));
    const int last_cell = nd == 1 ? 0 : visit_cell(26, lx_m, full, nd, NX);
    // Pad the list to a multiple of 4 entries per lane of a particle
    // (list_entry_row) with a particle that is outside the
    // list radius at this build: it stays beyond the force cutoff until the
    // next build (each particle moves at most skin/2), so the force loop
    // needs no per-entry validity test.  The pad is the first rejected
    // candidate of the last cell visited (a corner cell), else of any
    // staged cell.
    if (cnt & gm) {
        int pad = -1;
        for (int k = 0, kk = last_cell; k <= T.ncell && pad < 0; kk = k++) {
            const int4 c = T.pk[kk];
            const int na = T.na[kk];
            for (int e = 0; e < c.y && pad < 0; ++e) {
                const int g = cand_glob(c, na, e);
                if (!eval(load(cand_at<FROM_LDS>(c, na, e))) && g != i) pad = g;
            }
        }
        if (pad < 0) atomicOr(a.status + s, 8);
        for (int k = cnt; k < ((cnt + gm) & ~gm) && k < cap; ++k)
            col[(size_t)list_entry_row(k, lg) * row_stride + list_entry_col(k, lg)] = list_entry(pad < 0 ? i : pad);
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
                                                 int nd, int G, int gl, unsigned long long gmask)
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
    const int si = species_of(meta);
    float rl2s0, rl2s1;
    double rl2d0 = a.pp.rl2d[si * 2], rl2d1 = a.pp.rl2d[si * 2 + 1];
    {
        const double u = (double)rp.sc;
        rl2s0 = (float)(rl2d0 / (u * u));
        rl2s1 = (float)(rl2d1 / (u * u));
    }
    const int cap = A.cap;
    int *col = A.nbr_w + 4 * list_row_index(i, 0, cap);
    const size_t row_stride = 4 * LIST_TILE;
    const int lg = A.lg, gm = (4 << lg) - 1;
    // test the candidate at staged index x (a global slot when nothing is staged)
    auto test = [&](int x) -> bool {
        if (NS == 2) {
            double xj, yj, zj, wj;
            if (FROM_LDS) {
                u4_to_dbl2(cand[2 * x], xj, yj);
                u4_to_dbl2(cand[2 * x + 1], zj, wj);
            } else {
                u4_to_dbl2(a.src_x[x], xj, yj);
                u4_to_dbl2(a.src_x[P_ + x], zj, wj);
            }
            double dx = xd - xj, dy = yd - yj, dz = zd - zj;
            dx -= rp.L * rint(dx * rp.invL);
            dy -= rp.L * rint(dy * rp.invL);
            dz -= rp.L * rint(dz * rp.invL);
            const double r2 = dx * dx + dy * dy + dz * dz;
            return r2 < (species_of(meta_of_bits(wj)) ? rl2d1 : rl2d0);
        }
        const uint4 xj = FROM_LDS ? cand[x] : a.src_x[x];
        const float dx = (float)(int)(xi.x - xj.x), dy = (float)(int)(xi.y - xj.y),
                    dz = (float)(int)(xi.z - xj.z);
        const float r2 = __builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz));
        return r2 < (((int)xj.w < 0) ? rl2s1 : rl2s0);
    };
    // one cell's candidates (in the one-lane build's order), 4G at a time:
    // lane gl tests e = b + u G + gl (u = 0..3, independent loads in
    // flight); the ballots are taken in u order, which is ascending e
    // (the member's own candidate index is excluded by position, its global
    // slot is formed only for the entries stored, and the store address is
    // one 32 x 32 -> 64-bit multiply-add)
    int cnt = 0;
    const unsigned rs32 = (unsigned)row_stride;
    auto scan_cell = [&](int k) {
        const int4 c = T.pk[k];
        const int na = T.na[k], n = c.y;
        const int self = (unsigned)(i - c.z) < (unsigned)na ? i - c.z
                       : (unsigned)(i - c.w) < (unsigned)(n - na) ? na + (i - c.w) : -1;
        for (int b = 0; b < n; b += 4 * G) {
            bool acc[4];
            int ev[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) { // past the end: test the last candidate, masked off
                const int e = b + u * G + gl, ec = min(e, n - 1);
                ev[u] = e;
                acc[u] = test(cand_at<FROM_LDS>(c, na, ec)) && e < n && e != self;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const unsigned long long m = __ballot(acc[u]) & gmask;
                if (acc[u]) { // rank among the group's accepting lanes below this one
                    const unsigned k2 = (unsigned)cnt +
                        __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                    if (k2 < (unsigned)cap) {
                        const size_t idx = (size_t)(unsigned)list_entry_row((int)k2, lg) * rs32 +
                                           (unsigned)list_entry_col((int)k2, lg);
                        col[idx] = list_entry(cand_glob(c, na, ev[u]));
                    }
                }
                cnt += __popcll(m);
            }
        }
    };
    // the canonical visiting order (see visit_cell), as one loop
    const int nvis = nd == 1 ? 1 : 27;
#pragma unroll 1
    for (int v = 0; v < nvis; ++v) scan_cell(nd == 1 ? 0 : visit_cell(v, lx_m, full, nd, NX));
    const int last_cell = nd == 1 ? 0 : visit_cell(26, lx_m, full, nd, NX);
    // pad to a multiple of 4 entries per lane of a particle, as in the
    // one-lane build: the first rejected candidate of the last visited
    // cell, else (rare) of any staged cell
    if (cnt & gm) {
        int pad = -1;
        {
            const int4 cl = T.pk[last_cell];
            const int na = T.na[last_cell];
            for (int b = 0; b < cl.y; b += G) {
                const int e = b + gl;
                const int g = cand_glob(cl, na, min(e, cl.y - 1));
                const bool r = e < cl.y && !test(cand_at<FROM_LDS>(cl, na, min(e, cl.y - 1))) && g != i;
                const unsigned long long m = __ballot(r) & gmask;
                if (m) { pad = cand_glob(cl, na, b + (__ffsll(m) - 1) - (__ffsll(gmask) - 1)); break; }
            }
        }
        if (gl == 0) {
            for (int k = 0; k < T.ncell && pad < 0; ++k) {
                const int4 c = T.pk[k];
                const int na = T.na[k];
                for (int e = 0; e < c.y && pad < 0; ++e) {
                    const int g = cand_glob(c, na, e);
                    if (!test(cand_at<FROM_LDS>(c, na, e)) && g != i) pad = g;
                }
            }
            if (pad < 0) atomicOr(a.status + s, 8);
            for (int k = cnt; k < ((cnt + gm) & ~gm) && k < cap; ++k)
                col[(size_t)list_entry_row(k, lg) * row_stride + list_entry_col(k, lg)] =
                    list_entry(pad < 0 ? i : pad);
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
    // a bulk build (many replicas rebuilding together) gives each member of a
    // multi-cell replica one lane and each row segment one work item
    const bool bulk = a.bulk > 0 && a.force_slot == -1 && a.rlist[0] >= a.bulk;
    for_items(a.rlist, a.items_pref, a.rep, a.max_slots, a.force_slot, a.ctl, bulk ? 5 : 4,
              remap_block(blockIdx.x, gridDim.x, a.xcd), gridDim.x, [&](int s, int item) {
        const RepDev rp = a.rep[s];
        const int bparts = bulk ? 1 : rp.bparts;
        const int nd = rp.nd, planes = rp.planes, nc = nd * nd * nd;
        const int *cs = a.cs_new + rp.coff;
        int NX = 1, part = 0;
        bool full = true;
        if (nd == 1) {
            if (t == 0) {
                const int na = cs[1] - cs[0];
                T.pk[0] = make_int4(0, rp.n, cs[0], planes > 1 ? cs[1] : cs[0] + na);
                T.na[0] = na;
                T.ncell = 1;
                T.NX = 1;
                T.own0 = 0;
                T.nown = 1;
                T.total = rp.n;
                T.fits = rp.n <= a.lds_cap;
                if (item == 0 && a.from_scratch)
                    for (int k = 0; k <= planes; ++k) a.cs[rp.coff + k] = cs[k];
            }
        } else {
            const int W = a.width;
            full = nd <= W + 2;
            const int nseg = full ? 1 : (nd + W - 1) / W;
            part = item % bparts;
            const int segitem = item / bparts;
            const int seg = segitem % nseg, row = segitem / nseg;
            const int cy = row % nd, cz = row / nd;
            const int x0 = full ? 0 : (seg * nd) / nseg; // balanced segments
            const int x1 = full ? nd : ((seg + 1) * nd) / nseg;
            NX = full ? nd : x1 - x0 + 2;
            const int rowbase = nd * (cy + nd * cz);
            if (a.from_scratch && part == 0) { // retire the old cell starts of this segment
                for (int k = x0 + t; k < x1; k += B) {
                    const int rk = cell_rank(rowbase + k, rp, a.corder);
                    for (int pl = 0; pl < planes; ++pl) a.cs[rp.coff + pl * nc + rk] = cs[pl * nc + rk];
                }
                if (t == 0 && rowbase + x1 == nc) a.cs[rp.coff + planes * nc] = cs[planes * nc];
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
                const int rk = cell_rank(gx + nd * (gy + nd * gz), rp, a.corder);
                const int ga = cs[rk], na = cs[rk + 1] - ga;
                const int gb = planes > 1 ? cs[nc + rk] : ga + na;
                const int nb = planes > 1 ? cs[nc + rk + 1] - gb : 0;
                T.pk[k] = make_int4(0, na + nb, ga, gb);
                T.na[k] = na;
            }
            if (t == 0) {
                T.NX = NX;
                T.ncell = 9 * NX;
                T.own0 = 4 * NX + (full ? 0 : 1); // own row (dz = dy = 0), segment cells
                T.nown = full ? NX : NX - 2;
            }
            __syncthreads();
            if (t < 64) { // exclusive scan of the staged cell sizes (one wave)
                const int ncells = 9 * NX;
                int carry = 0;
                for (int b = 0; b < ncells; b += 64) {
                    const int k = b + t;
                    const int v = k < ncells ? T.pk[k].y : 0;
                    int incl = v;
#pragma unroll
                    for (int o = 1; o < 64; o <<= 1) {
                        const int u = __shfl_up(incl, o, 64);
                        if (t >= o) incl += u;
                    }
                    if (k < ncells) T.pk[k].x = carry + incl - v;
                    carry += __shfl(incl, 63, 64);
                }
                if (t == 0) { T.total = carry; T.fits = carry <= a.lds_cap; }
            }
        }
        __syncthreads();
        if (t == 0) { // member prefix over the segment's cells: plane 0 members, then plane 1
            const int o = T.own0, no = T.nown;
            int acc = 0;
            T.mp[0] = 0;
            for (int j = 0; j < no; ++j) { acc += T.na[o + j]; T.mp[j + 1] = acc; }
            for (int j = 0; j < no; ++j) { acc += T.pk[o + j].y - T.na[o + j]; T.mp[no + j + 1] = acc; }
        }
        const bool fits = T.fits != 0;
        if (fits) { // stage: element e belongs to the last cell whose LDS start is <= e
            const int tot = T.total, ncl = T.ncell;
            for (int e = t; e < tot; e += B) {
                int lo = 0, hi = ncl;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (T.pk[mid].x <= e) lo = mid; else hi = mid;
                }
                const int4 c = T.pk[lo];
                const int g = cand_glob(c, T.na[lo], e - c.x);
                if (NS == 2) {
                    cand[2 * e] = a.src_x[g];
                    cand[2 * e + 1] = a.src_x[(size_t)a.A.P + g];
                } else cand[e] = a.src_x[g];
            }
        }
        __syncthreads();
        // this item's share of the segment's members
        const int no = T.nown, ms = T.mp[2 * no];
        int m0, m1;
        if (nd == 1) {
            m0 = item * a.single_members;
            m1 = min(m0 + a.single_members, rp.n);
        } else {
            m0 = (int)(((long long)part * ms) / bparts);
            m1 = (int)(((long long)(part + 1) * ms) / bparts);
        }
        // member index k -> slot i and the member's own-row staged cell lx
        auto member = [&](int k, int &i, int &lx) {
            int lo = 0, hi = 2 * no; // last j with mp[j] <= k
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (T.mp[mid] <= k) lo = mid; else hi = mid;
            }
            const int jj = lo < no ? lo : lo - no;
            const int4 c = T.pk[T.own0 + jj];
            i = (lo < no ? c.z : c.w) + (k - T.mp[lo]);
            lx = nd == 1 ? 0 : T.own0 + jj - 4 * NX;
        };
        // lanes per member: the replica's (fixed by the launch, or one lane
        // for large replicas), else the largest power of two that still
        // gives every member of this work item its own group
        int G = bulk && nd > 1 ? 1 : rp.blanes;
        if (G == 0) {
            G = 1;
            while (G < 64 && (2 * G) * (m1 - m0) <= B) G *= 2;
        }
        if (G == 1) {
            for (int k = m0 + t; k < m1; k += B) {
                int i, lx_m;
                member(k, i, lx_m);
                if (fits) build_member<P, true>(a, rp, i, lx_m, T, full, cand, s, nd);
                else build_member<P, false>(a, rp, i, lx_m, T, full, cand, s, nd);
                copy_back<P>(a, i);
            }
        } else {
            const int lane = t & 63, gl = t & (G - 1);
            const unsigned long long gmask =
                G == 64 ? ~0ull : ((1ull << G) - 1ull) << (lane & ~(G - 1));
            for (int k = m0 + t / G; k < m1; k += B / G) {
                int i, lx_m;
                member(k, i, lx_m);
                if (fits) build_member_grp<P, true>(a, rp, i, lx_m, T, full, cand, s, nd, G, gl, gmask);
                else build_member_grp<P, false>(a, rp, i, lx_m, T, full, cand, s, nd, G, gl, gmask);
                if (gl == 0) copy_back<P>(a, i);
            }
        }
        __syncthreads();
    });
}

// ------------------------------------------------------------ launchers
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
    hipLaunchKernelGGL(k_scan, dim3(a.max_slots), dim3(SCAN_B), 0, s, a);
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

// Resident workgroups per CU of the sort and list-build kernels (their grids
// are sized to one full residency: the kernels walk their work items in a
// grid-stride loop, and a second partial round of workgroups would idle most
// of the chip while it runs).
hipError_t occupancy_permute(int prec, int *per_cu)
{
    const void *f;
    switch (prec) {
    case PREC_FP32: f = (const void *)k_permute<PREC_FP32>; break;
    case PREC_DS: f = (const void *)k_permute<PREC_DS>; break;
    case PREC_MIX: f = (const void *)k_permute<PREC_MIX>; break;
    default: f = (const void *)k_permute<PREC_FP64>; break;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, f, 256, 0);
}

// Staged records plus four of padding: the one-lane scan reads up to three
// records past a cell's end (masked off), also past the last staged cell.
static size_t build_lds_bytes(int prec, int lds_cap)
{
    return (size_t)(lds_cap + 4) * 16 * (prec == PREC_FP64 ? 2 : 1);
}

hipError_t occupancy_build(int prec, int block, int lds_cap, int *per_cu)
{
    const size_t lds = build_lds_bytes(prec, lds_cap);
    const void *f;
    switch (prec) {
    case PREC_FP32: f = (const void *)k_build<PREC_FP32>; break;
    case PREC_DS: f = (const void *)k_build<PREC_DS>; break;
    case PREC_MIX: f = (const void *)k_build<PREC_MIX>; break;
    default: f = (const void *)k_build<PREC_FP64>; break;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, f, block, lds);
}

hipError_t launch_build(int prec, const BuildArgs &a, int grid, int block, hipStream_t s)
{
    const size_t lds = build_lds_bytes(prec, a.lds_cap);
    switch (prec) {
    case PREC_FP32: hipLaunchKernelGGL((k_build<PREC_FP32>), dim3(grid), dim3(block), lds, s, a); break;
    case PREC_DS: hipLaunchKernelGGL((k_build<PREC_DS>), dim3(grid), dim3(block), lds, s, a); break;
    case PREC_MIX: hipLaunchKernelGGL((k_build<PREC_MIX>), dim3(grid), dim3(block), lds, s, a); break;
    default: hipLaunchKernelGGL((k_build<PREC_FP64>), dim3(grid), dim3(block), lds, s, a); break;
    }
    LAUNCH_CHECK();
}
