// Host engine and C ABI of libmdx (declared in include/md.h).
//
// The engine owns no device memory: it carves the caller's workspace into the
// arrays described in md_dev.hpp, keeps host mirrors of the slot table and the
// arena allocators, launches the kernels on the caller's stream and captures
// the per-step launch sequence into hipGraphs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/md.h"
#include "kernels.hpp"
#include "md_dev.hpp"
#include "tcf.hpp"

namespace {

constexpr int64_t ALIGN = 256;
constexpr uint32_t CKPT_MAGIC = 0x4d445843; // "MDXC"
constexpr int CKPT_VERSION = 3;
constexpr int MD_DEFAULT_LPP = 2;

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// First-fit allocator over [0, cap) with coalescing of free ranges.
struct RangeAlloc {
    int64_t cap = 0;
    std::vector<std::pair<int64_t, int64_t>> free_; // (off, len), sorted by off
    void reset(int64_t c)
    {
        cap = c;
        free_.clear();
        if (c > 0) free_.push_back({0, c});
    }
    bool alloc(int64_t len, int64_t &off)
    {
        for (size_t k = 0; k < free_.size(); ++k)
            if (free_[k].second >= len) {
                off = free_[k].first;
                free_[k].first += len;
                free_[k].second -= len;
                if (free_[k].second == 0) free_.erase(free_.begin() + k);
                return true;
            }
        return false;
    }
    void release(int64_t off, int64_t len)
    {
        auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(off, (int64_t)0));
        it = free_.insert(it, {off, len});
        size_t k = it - free_.begin();
        if (k + 1 < free_.size() && free_[k].first + free_[k].second == free_[k + 1].first) {
            free_[k].second += free_[k + 1].second;
            free_.erase(free_.begin() + k + 1);
        }
        if (k > 0 && free_[k - 1].first + free_[k - 1].second == free_[k].first) {
            free_[k - 1].second += free_[k].second;
            free_.erase(free_.begin() + k);
        }
    }
};

struct SlotHost {
    bool attached = false;
    int n = 0, nd = 1;
    int64_t off = 0, coff = 0, ncell_alloc = 0;
    double L = 0;
    int64_t target = 0;
    int failed = 0; // error bits (MD_ST_*) seen at the last synchronising call
};

struct Layout {
    int NW, NS;
    int64_t P, cap, slots, cells;
};

} // namespace

struct md_system {
    md_config cfg{};
    int prec = 0;
    Layout lay{};
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    int64_t ws_bytes = 0;
    // device arrays
    uint4 *st[3]{}, *sc_st[3]{}, *snap[2]{}, *sc_snap = nullptr, *xref = nullptr;
    int4 *meta = nullptr, *sc_meta = nullptr;
    int *nbr = nullptr, *nbr_cnt = nullptr;
    double *obs = nullptr, *obs_out = nullptr;
    int *count[2]{}, *cs = nullptr, *cs_new = nullptr;
    int *corder = nullptr; // per-replica cell rank tables (cell arena offsets)
    RepDev *rep = nullptr;
    Ctl *ctl[2]{};
    int *target = nullptr, *need[2]{}, *rlist[2]{}, *status = nullptr, *nreb = nullptr;
    int *items3 = nullptr, *items4 = nullptr, *chunks = nullptr;
    double *partial = nullptr;
    // host state
    PairDev pp{};
    IntegDev ig{};
    md_launch launch{};
    double rlist_max = 0;
    std::vector<SlotHost> slots;
    RangeAlloc parena, carena;
    int parity = 0; // parity of the snapshot the next step reads
    int lpp = 1;    // lanes per particle of the force sum
    int n_cu = 0;   // compute units of the device
    int dev = 0;    // the device current at md_create
    int grid_perm = 0, grid_build = 0; // one full residency of the rebuild kernels
    std::map<int, hipGraphExec_t> graphs;
    std::string err;
};

// ------------------------------------------------------------------ errors
static md_status fail(md_system *s, md_status st, const char *fmt, ...)
{
    if (s) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        s->err = buf;
    }
    return st;
}

#define HIPCHK(sys, call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail((sys), MD_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

// ----------------------------------------------------------- configuration
static double lj_v(double r2, double eps, double sig)
{
    double s2 = sig * sig / r2, s6 = s2 * s2 * s2;
    return 4.0 * eps * (s6 * s6 - s6);
}

static int nsp_of(const md_config *c) { return c->n_species; }

static double rlist_max_of(const md_config *c)
{
    double m = 0;
    int k = nsp_of(c);
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) m = std::max(m, c->rcut[a * 2 + b] + c->skin);
    return m;
}

static md_status validate_cfg(const md_config *c, std::string *why)
{
    auto bad = [&](const char *m) { if (why) *why = m; return MD_E_ARG; };
    if (!c) return bad("null config");
    if (c->n_species != 1 && c->n_species != 2) return bad("n_species must be 1 or 2");
    if (c->precision < 0 || c->precision > 3) return bad("precision must be 0..3");
    int k = c->n_species;
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            int t = a * 2 + b;
            if (!(c->eps[t] > 0) || !(c->sigma[t] > 0) || !(c->rcut[t] > 0) || !std::isfinite(c->eps[t]) ||
                !std::isfinite(c->sigma[t]) || !std::isfinite(c->rcut[t]))
                return bad("eps, sigma and rcut must be positive and finite");
        }
    if (k == 2 && (c->eps[1] != c->eps[2] || c->sigma[1] != c->sigma[2] || c->rcut[1] != c->rcut[2]))
        return bad("pair table must be symmetric");
    if (!(c->mass > 0) || !(c->dt > 0) || !(c->skin > 0) || !std::isfinite(c->dt) || !std::isfinite(c->skin))
        return bad("mass, dt and skin must be positive");
    if (c->max_slots < 1 || c->max_slots > 65536) return bad("max_slots must be in [1, 65536]");
    if (c->max_particles < 1 || c->max_particles > MAX_ARENA_SLOTS - 256) return bad("max_particles must be in [1, 2^28 - 256]");
    if (c->nbr_capacity < 0 || c->nbr_capacity > 4096) return bad("nbr_capacity must be in [0, 4096]");
    if (c->max_cells < 0) return bad("max_cells must be >= 0");
    if (c->max_density < 0) return bad("max_density must be >= 0");
    if (c->lanes_per_particle != 0 && c->lanes_per_particle != 1 && c->lanes_per_particle != 2 &&
        c->lanes_per_particle != 4)
        return bad("lanes_per_particle must be 0, 1, 2 or 4");
    if (!(c->smooth >= 0) || !std::isfinite(c->smooth)) return bad("smooth must be >= 0 and finite");
    if (c->rebuild_every != 0 && (c->rebuild_every < 2 || c->rebuild_every > 1000000))
        return bad("rebuild_every must be 0 or in [2, 1e6]");
    if (c->rebuild_every != 0 && !(c->rebuild_early > 0 && c->rebuild_early <= 1))
        return bad("rebuild_early must be in (0, 1] when rebuild_every is set");
    if (c->cell_order != MD_ORDER_ROW && c->cell_order != MD_ORDER_MORTON && c->cell_order != MD_ORDER_HILBERT)
        return bad("cell_order must be MD_ORDER_ROW, MD_ORDER_MORTON or MD_ORDER_HILBERT");
    return MD_OK;
}

static Layout layout_of(const md_config *c)
{
    Layout L;
    L.NW = c->precision == PREC_FP32 ? 2 : 3;
    L.NS = c->precision == PREC_FP64 ? 2 : 1;
    L.P = align_up(c->max_particles, 256);
    double rho = c->max_density > 0 ? c->max_density : 1.2;
    double rl = rlist_max_of(c);
    // a multiple of 16: lists are padded to four entries per lane of a particle
    if (c->nbr_capacity > 0) L.cap = align_up(c->nbr_capacity, 16);
    else {
        double mean = 4.18879020478639 * rl * rl * rl * rho; // (4/3) pi r^3 rho
        L.cap = align_up((int64_t)std::ceil(1.3 * mean + 16.0), 16);
    }
    L.slots = c->max_slots;
    L.cells = (c->max_cells > 0 ? c->max_cells : c->max_particles / 2 + 64) + c->max_slots;
    return L;
}

// Carve (or size, when base == nullptr) the workspace.
struct Carver {
    char *base;
    int64_t off = 0;
    template <class T> T *take(int64_t count)
    {
        off = align_up(off, ALIGN);
        T *p = base ? (T *)(base + off) : nullptr;
        off += count * (int64_t)sizeof(T);
        return p;
    }
};

static int64_t carve(md_system *s, const Layout &L, char *base)
{
    Carver c{base};
    md_system dummy;
    md_system *d = s ? s : &dummy;
    for (int k = 0; k < 3; ++k) d->st[k] = k < L.NW ? c.take<uint4>(L.P) : nullptr;
    for (int k = 0; k < 3; ++k) d->sc_st[k] = k < L.NW ? c.take<uint4>(L.P) : nullptr;
    d->snap[0] = c.take<uint4>(L.P * L.NS);
    d->snap[1] = c.take<uint4>(L.P * L.NS);
    d->sc_snap = c.take<uint4>(L.P * L.NS);
    d->xref = c.take<uint4>(L.P * L.NS);
    d->meta = c.take<int4>(L.P);
    d->sc_meta = c.take<int4>(L.P);
    d->nbr_cnt = c.take<int>(L.P);
    d->nbr = c.take<int>(L.P * L.cap);
    d->obs = c.take<double>(L.P * 8);
    d->count[0] = c.take<int>(L.cells);
    d->count[1] = c.take<int>(L.cells);
    d->cs = c.take<int>(L.cells);
    d->cs_new = c.take<int>(L.cells);
    d->corder = c.take<int>(L.cells);
    d->rep = c.take<RepDev>(L.slots);
    d->ctl[0] = c.take<Ctl>(L.slots);
    d->ctl[1] = c.take<Ctl>(L.slots);
    d->target = c.take<int>(L.slots);
    d->need[0] = c.take<int>(L.slots);
    d->need[1] = c.take<int>(L.slots);
    d->rlist[0] = c.take<int>(L.slots + 1);
    d->rlist[1] = c.take<int>(L.slots + 1);
    d->status = c.take<int>(L.slots);
    d->nreb = c.take<int>(L.slots);
    d->items3 = c.take<int>(L.slots + 1);
    d->items4 = c.take<int>(L.slots + 1);
    d->chunks = c.take<int>(L.slots + 1);
    d->partial = c.take<double>((L.P / 4096 + L.slots + 1) * 8);
    d->obs_out = c.take<double>(L.slots * 8);
    return align_up(c.off, ALIGN);
}

static void make_tables(md_system *s)
{
    const md_config *c = &s->cfg;
    PairDev &p = s->pp;
    memset(&p, 0, sizeof p);
    for (int t = 0; t < 4; ++t) {
        int a = t >> 1, b = t & 1;
        int u = c->n_species == 1 ? 0 : a * 2 + b;
        double eps = c->eps[u], sig = c->sigma[u], rc = c->rcut[u];
        double rl = rc + c->skin;
        p.rl2d[t] = rl * rl;
        p.rc2d[t] = rc * rc;
        p.sig2d[t] = sig * sig;
        p.eps24d[t] = 24.0 * eps;
        p.eps4d[t] = 4.0 * eps;
        p.shiftd[t] = lj_v(rc * rc, eps, sig);
        p.rl2[t] = (float)p.rl2d[t];
        p.rc2[t] = (float)p.rc2d[t];
        p.sig2[t] = (float)p.sig2d[t];
        p.eps24[t] = (float)p.eps24d[t];
        p.eps4[t] = (float)p.eps4d[t];
        p.shift[t] = (float)p.shiftd[t];
        p.hsd[t] = c->smooth * sig;
        p.rcd[t] = rc;
    }
    p.smooth = c->smooth > 0 ? 1 : 0;
    // uniform cutoff ratio: rc_ab / sigma_ab equal (to rounding) for every pair
    {
        const int k = c->n_species;
        const double r0 = c->rcut[0] / c->sigma[0];
        bool uni = true;
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b)
                if (std::fabs(c->rcut[a * 2 + b] / c->sigma[a * 2 + b] - r0) > 1e-12 * r0) uni = false;
        p.uniform = uni ? 1 : 0;
        p.s2cut = (float)(1.0 / (r0 * r0));
    }
    p.hs2d = 0.25 * c->skin * c->skin;
    p.hs2 = (float)p.hs2d;
    p.align_every = c->rebuild_every;
    p.hs2d_early = c->rebuild_every ? p.hs2d * c->rebuild_early * c->rebuild_early : p.hs2d;
    p.nsp = c->n_species;
    IntegDev &g = s->ig;
    g.m = c->mass;
    g.dt = c->dt;
    g.h = 0.5 * c->dt / c->mass;
    g.dtf = (float)g.dt;
    g.hf = (float)g.h;
    g.dt_hi = (float)g.dt;
    g.dt_lo = (float)(g.dt - (double)g.dt_hi);
    g.h_hi = (float)g.h;
    g.h_lo = (float)(g.h - (double)g.h_hi);
    s->rlist_max = rlist_max_of(c);
}

static int cells_per_edge(double L, double rl)
{
    int nd = (int)std::floor(L / rl);
    if (nd < 3) nd = 1;
    return nd;
}

// staged candidates per list-build workgroup (48 KB of LDS)
static int lds_cap_of(int prec) { return prec == PREC_FP64 ? 1536 : 3072; }

// Grids of the sort and list-build kernels: one full residency of the
// device (queried for the current block size).
static md_status size_grids(md_system *s)
{
    int per_cu = 0;
    HIPCHK(s, occupancy_permute(s->prec, &per_cu));
    s->grid_perm = std::max(1, per_cu) * s->n_cu;
    per_cu = 0;
    HIPCHK(s, occupancy_build(s->prec, s->launch.build_block, lds_cap_of(s->prec), &per_cu));
    if (per_cu < 1) return fail(s, MD_E_ARG, "list-build block of %d threads does not fit a CU", s->launch.build_block);
    s->grid_build = per_cu * s->n_cu;
    return MD_OK;
}

// members per list-build work item of a single-cell replica: one group of
// build_lanes lanes (16 when automatic) per member
static int single_members(const md_system *s)
{
    const int G = s->launch.build_lanes ? s->launch.build_lanes : 16;
    return std::max(1, s->launch.build_block / G);
}

// Work decomposition of the list build of one replica.  A replica with at
// least one row segment per compute unit builds one segment per work item,
// one lane per member.  A smaller one (whose build would otherwise run on a
// few CUs, each testing every member against hundreds of candidates) splits
// each segment's members over up to 256 / segments work items (at least 16
// members each) and lets a group of lanes share each member's candidates.
// None of this changes a list entry.
static void build_shape(const md_system *s, int n, int nd, int &parts, int &lanes)
{
    parts = 1;
    lanes = s->launch.build_lanes;
    if (nd == 1) return;
    const int W = s->launch.build_width;
    const int nseg = nd <= W + 2 ? 1 : (nd + W - 1) / W;
    const int base = nd * nd * nseg;
    if (base >= 256) {
        if (!lanes) lanes = 1;
        return;
    }
    parts = std::max(1, std::min((256 + base - 1) / base, n / base / 16));
    if (s->launch.build_split > 0) parts = std::min(parts, s->launch.build_split);
}

static int items4_of(const md_system *s, int n, int nd)
{
    if (nd == 1) {
        const int M = single_members(s);
        return (n + M - 1) / M;
    }
    int parts, lanes;
    build_shape(s, n, nd, parts, lanes);
    int W = s->launch.build_width;
    int nseg = nd <= W + 2 ? 1 : (nd + W - 1) / W;
    return nd * nd * nseg * parts;
}

// Work items of a bulk list build (one per row segment; a single-cell
// replica keeps its usual items).
static int bulk_items_of(const md_system *s, int n, int nd)
{
    if (nd == 1) return items4_of(s, n, nd);
    const int W = s->launch.build_width;
    return nd * nd * (nd <= W + 2 ? 1 : (nd + W - 1) / W);
}

static md_status upload_items(md_system *s)
{
    int S = (int)s->lay.slots;
    std::vector<int> p3(S + 1, 0), p4(S + 1, 0), p5(S + 1, 0);
    for (int k = 0; k < S; ++k) {
        const SlotHost &h = s->slots[k];
        int a3 = 0, a4 = 0, a5 = 0;
        if (h.attached) {
            a3 = h.nd * h.nd * h.nd;
            a4 = items4_of(s, h.n, h.nd);
            a5 = (h.n + 4095) / 4096;
        }
        p3[k + 1] = p3[k] + a3;
        p4[k + 1] = p4[k] + a4;
        p5[k + 1] = p5[k] + a5;
    }
    HIPCHK(s, hipMemcpyAsync(s->chunks, p5.data(), sizeof(int) * (S + 1), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->items3, p3.data(), sizeof(int) * (S + 1), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->items4, p4.data(), sizeof(int) * (S + 1), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return MD_OK;
}

static void drop_graphs(md_system *s)
{
    for (auto &kv : s->graphs) (void)hipGraphExecDestroy(kv.second);
    s->graphs.clear();
}

// ------------------------------------------------------------- arg blocks
static KArena arena_of(const md_system *s)
{
    KArena A;
    A.P = (int)s->lay.P;
    A.cap = (int)s->lay.cap;
    A.lg = s->lpp == 4 ? 2 : s->lpp == 2 ? 1 : 0;
    for (int k = 0; k < 3; ++k) A.st[k] = s->st[k];
    A.xref = s->xref;
    A.xref_w = s->xref;
    A.meta = s->meta;
    A.nbr = s->nbr;
    A.nbr_w = s->nbr;
    A.nbr_cnt = s->nbr_cnt;
    A.nbr_cnt_w = s->nbr_cnt;
    return A;
}

static StepArgs step_args(const md_system *s, int p)
{
    StepArgs a;
    memset(&a, 0, sizeof a);
    a.A = arena_of(s);
    a.cell_cap = (int)s->lay.cells;
    a.max_slots = (int)s->lay.slots;
    a.xcd = s->launch.xcd_remap;
    a.lpp = s->lpp;
    a.snap_cur = s->snap[p];
    a.snap_next = s->snap[p ^ 1];
    a.rep = s->rep;
    a.ctl_cur = s->ctl[p];
    a.ctl_next = s->ctl[p ^ 1];
    a.target = s->target;
    a.need_cur = s->need[p];
    a.need_other = s->need[p ^ 1];
    a.rlist_cur = s->rlist[p];
    a.rlist_other = s->rlist[p ^ 1];
    a.count_cur = s->count[p];
    a.count_other = s->count[p ^ 1];
    a.corder = s->corder;
    a.status = s->status;
    a.obs = s->obs;
    a.pp = s->pp;
    a.ig = s->ig;
    return a;
}

// The three rebuild launches that follow a step of parity p (force_slot -1:
// flagged replicas; -2: all attached; >= 0: that slot).
static md_status launch_rebuild(md_system *s, int p, int force_slot, bool from_scratch)
{
    const int prec = s->prec;
    ScanArgs sa;
    sa.max_slots = (int)s->lay.slots;
    sa.force_slot = force_slot;
    sa.rep = s->rep;
    sa.need = s->need[p];
    sa.rlist = s->rlist[p];
    sa.ctl = s->ctl[p ^ 1];
    sa.count = s->count[p];
    sa.cs_new = s->cs_new;
    sa.status = s->status;
    sa.nreb = s->nreb;
    HIPCHK(s, launch_scan(sa, s->stream));

    PermArgs pa;
    memset(&pa, 0, sizeof pa);
    pa.A = arena_of(s);
    pa.max_slots = (int)s->lay.slots;
    pa.force_slot = force_slot;
    pa.items_pref = s->items3;
    pa.rep = s->rep;
    pa.need = s->need[p];
    pa.rlist = s->rlist[p];
    pa.ctl = s->ctl[p ^ 1];
    pa.cs = s->cs;
    pa.cs_new = s->cs_new;
    pa.corder = s->corder;
    pa.snap = s->snap[p ^ 1];
    for (int k = 0; k < 3; ++k) pa.sc_st[k] = s->sc_st[k];
    pa.sc_snap = s->sc_snap;
    pa.sc_meta = s->sc_meta;
    pa.status = s->status;
    HIPCHK(s, launch_permute(prec, pa, s->grid_perm, s->stream));

    BuildArgs ba;
    memset(&ba, 0, sizeof ba);
    ba.A = arena_of(s);
    ba.max_slots = (int)s->lay.slots;
    ba.force_slot = force_slot;
    ba.from_scratch = from_scratch ? 1 : 0;
    ba.width = s->launch.build_width;
    ba.lds_cap = lds_cap_of(prec);
    ba.single_members = single_members(s);
    ba.bulk = s->launch.build_bulk;
    ba.xcd = s->launch.xcd_remap;
    ba.items_pref = s->items4;
    ba.rep = s->rep;
    ba.need = s->need[p];
    ba.rlist = s->rlist[p];
    ba.ctl = s->ctl[p ^ 1];
    ba.cs = s->cs;
    ba.cs_new = s->cs_new;
    ba.corder = s->corder;
    ba.src_x = s->sc_snap;
    ba.snap_cur = s->snap[p ^ 1];
    for (int k = 0; k < 3; ++k) ba.sc_st[k] = s->sc_st[k];
    ba.sc_meta = s->sc_meta;
    ba.status = s->status;
    ba.pp = s->pp;
    HIPCHK(s, launch_build(prec, ba, s->grid_build, s->launch.build_block, s->stream));
    return MD_OK;
}

// List build only, from the main arrays (attach / restore).
static md_status launch_build_main(md_system *s, int slot)
{
    BuildArgs ba;
    memset(&ba, 0, sizeof ba);
    ba.A = arena_of(s);
    ba.max_slots = (int)s->lay.slots;
    ba.force_slot = slot;
    ba.from_scratch = 0;
    ba.width = s->launch.build_width;
    ba.lds_cap = lds_cap_of(s->prec);
    ba.single_members = single_members(s);
    ba.xcd = s->launch.xcd_remap;
    ba.items_pref = s->items4;
    ba.rep = s->rep;
    ba.need = s->need[0];
    ba.rlist = s->rlist[0];
    ba.ctl = s->ctl[0];
    ba.cs = s->cs;
    ba.cs_new = s->cs_new;
    ba.corder = s->corder;
    ba.src_x = s->xref;
    ba.snap_cur = s->snap[0];
    ba.status = s->status;
    ba.pp = s->pp;
    HIPCHK(s, launch_build(s->prec, ba, s->grid_build, s->launch.build_block, s->stream));
    return MD_OK;
}

static md_status launch_one_step(md_system *s, int p)
{
    StepArgs a = step_args(s, p);
    HIPCHK(s, launch_step(s->prec, a, s->launch.step_block, false, s->stream));
    return launch_rebuild(s, p, -1, true);
}

// The launches of `steps` consecutive steps starting at snapshot parity
// `parity`, captured once into a hipGraph and cached by (steps, parity).
static md_status get_graph(md_system *s, int steps, int parity, hipGraphExec_t *out)
{
    const int key = 2 * steps + parity;
    auto it = s->graphs.find(key);
    if (it != s->graphs.end()) { *out = it->second; return MD_OK; }
    if (s->graphs.size() >= 64) drop_graphs(s); // callers cycling through many step counts
    hipGraph_t g = nullptr;
    HIPCHK(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    md_status st = MD_OK;
    for (int k = 0; k < steps && st == MD_OK; ++k) st = launch_one_step(s, (parity + k) & 1);
    hipError_t e = hipStreamEndCapture(s->stream, &g);
    if (st != MD_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return fail(s, MD_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(s, MD_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    s->graphs[key] = ex;
    *out = ex;
    return MD_OK;
}

// n step launches: replays of graphs of graph_steps launches, the remainder
// (however short) as one more captured graph; eager launches when graphs
// are off.
static md_status run_launches(md_system *s, int64_t n)
{
    const int G = s->launch.graph_steps;
    while (n > 0) {
        if (G < 2) {
            md_status st = launch_one_step(s, s->parity);
            if (st != MD_OK) return st;
            s->parity ^= 1;
            --n;
            continue;
        }
        const int k = (int)std::min<int64_t>(n, G);
        hipGraphExec_t ex;
        md_status st = get_graph(s, k, s->parity, &ex);
        if (st != MD_OK) return st;
        HIPCHK(s, hipGraphLaunch(ex, s->stream));
        n -= k;
        s->parity ^= k & 1;
    }
    return MD_OK;
}

// Small control kernels live in aux_kernels.hip; declare the launchers here.
hipError_t launch_add_targets(int *target, const Ctl *ctl, int max_slots, int delta, hipStream_t s);
hipError_t launch_poke(int *p, int v, hipStream_t s);
hipError_t launch_void_stored(Ctl *ctl, int max_slots, hipStream_t s);

// ------------------------------------------------------------ host helpers
struct HostRep {
    std::vector<uint4> st[3];
    std::vector<uint4> snap; // NS * n
    std::vector<int4> meta;
    std::vector<int> cs;     // planes * ncell + 1, absolute
};

static void put_dbl2(uint4 &u, double a, double b)
{
    unsigned long long x, y;
    memcpy(&x, &a, 8);
    memcpy(&y, &b, 8);
    u.x = (uint32_t)x; u.y = (uint32_t)(x >> 32); u.z = (uint32_t)y; u.w = (uint32_t)(y >> 32);
}
static void get_dbl2(const uint4 &u, double &a, double &b)
{
    unsigned long long x = ((unsigned long long)u.y << 32) | u.x, y = ((unsigned long long)u.w << 32) | u.z;
    memcpy(&a, &x, 8);
    memcpy(&b, &y, 8);
}
static void put_f4(uint4 &u, float a, float b, float c, float d)
{
    memcpy(&u.x, &a, 4); memcpy(&u.y, &b, 4); memcpy(&u.z, &c, 4); memcpy(&u.w, &d, 4);
}
static void get_f4(const uint4 &u, float &a, float &b, float &c, float &d)
{
    memcpy(&a, &u.x, 4); memcpy(&b, &u.y, 4); memcpy(&c, &u.z, 4); memcpy(&d, &u.w, 4);
}

// ------------------------------------------------------------ cell order
// Keys of cell (x, y, z) on a 2^bits grid.  Morton: the coordinates' bits
// interleaved (x lowest).  Hilbert: Skilling's method (J. Skilling,
// "Programming the Hilbert curve", AIP Conf. Proc. 707, 381 (2004)) turns
// the coordinates into the transposed Hilbert index, whose bits, read level
// by level from the top, give the position along the curve; consecutive
// positions are face-adjacent cells.
static uint64_t morton_key(uint32_t x, uint32_t y, uint32_t z, int bits)
{
    uint64_t k = 0;
    for (int l = bits - 1; l >= 0; --l)
        k = (k << 3) | ((uint64_t)((z >> l) & 1u) << 2) | ((uint64_t)((y >> l) & 1u) << 1) | ((x >> l) & 1u);
    return k;
}

static uint64_t hilbert_key(uint32_t x, uint32_t y, uint32_t z, int bits)
{
    uint32_t X[3] = {x, y, z};
    const uint32_t top = 1u << (bits - 1);
    for (uint32_t q = top; q > 1; q >>= 1) { // undo the excess work of the curve's reflections
        const uint32_t low = q - 1;
        for (int i = 0; i < 3; ++i) {
            if (X[i] & q) {
                X[0] ^= low; // invert the low bits of the first axis
            } else { // exchange the low bits of the first axis and axis i
                const uint32_t t = (X[0] ^ X[i]) & low;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 1; i < 3; ++i) X[i] ^= X[i - 1]; // Gray encode
    uint32_t t = 0;
    for (uint32_t q = top; q > 1; q >>= 1)
        if (X[2] & q) t ^= q - 1;
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    uint64_t k = 0;
    for (int l = bits - 1; l >= 0; --l)
        for (int i = 0; i < 3; ++i) k = (k << 1) | ((X[i] >> l) & 1u);
    return k;
}

// rank[c] of each cell c = x + nd (y + nd z) of an nd^3 grid in the order
// `order`: row-major (rank = c), or along the Morton or Hilbert curve of the
// enclosing 2^bits grid (cells outside the nd^3 grid are skipped).
static void cell_ranks(int nd, int order, int *rank)
{
    const int64_t nc = (int64_t)nd * nd * nd;
    if (order == MD_ORDER_ROW || nd == 1) {
        for (int64_t c = 0; c < nc; ++c) rank[c] = (int)c;
        return;
    }
    int bits = 1;
    while ((1 << bits) < nd) ++bits;
    std::vector<std::pair<uint64_t, int>> key(nc);
    for (int64_t c = 0; c < nc; ++c) {
        const uint32_t x = (uint32_t)(c % nd), y = (uint32_t)((c / nd) % nd), z = (uint32_t)(c / ((int64_t)nd * nd));
        key[c] = {order == MD_ORDER_MORTON ? morton_key(x, y, z, bits) : hilbert_key(x, y, z, bits), (int)c};
    }
    std::sort(key.begin(), key.end());
    for (int64_t r = 0; r < nc; ++r) rank[key[r].second] = (int)r;
}

// The replica's cell rank table (used when RepDev::curve is set).
static std::vector<int> ranks_of(const md_system *s, const SlotHost &h)
{
    std::vector<int> rk((size_t)h.nd * h.nd * h.nd);
    cell_ranks(h.nd, s->cfg.cell_order, rk.data());
    return rk;
}

static RepDev repdev_of(const md_system *s, const SlotHost &h)
{
    RepDev r;
    memset(&r, 0, sizeof r);
    r.n = h.n;
    r.off = (int)h.off;
    r.nd = h.nd;
    r.coff = (int)h.coff;
    r.planes = s->cfg.n_species;
    r.curve = s->cfg.cell_order != MD_ORDER_ROW && h.nd > 1;
    r.L = h.L;
    r.invL = 1.0 / h.L;
    r.fxs = 4294967296.0 / h.L;
    r.sc = (float)(h.L / 4294967296.0);
    r.L_hi = (float)h.L;
    r.L_lo = (float)(h.L - (double)r.L_hi);
    {   // pair constants in fixed-point units (see RepDev)
        const PairDev &p = s->pp;
        const double u = (double)r.sc;
        const double iu2 = 1.0 / (u * u);
        for (int t = 0; t < 4; ++t) {
            r.rc2s[t] = (float)(p.rc2d[t] * iu2);
            r.sig2s[t] = (float)(p.sig2d[t] * iu2);
            r.e24s[t] = (float)(p.eps24d[t] / u);
            r.rcs[t] = (float)(p.rcd[t] / u);
            r.xsc[t] = p.smooth ? (float)(u / p.hsd[t]) : 0.0f;
            r.ihs[t] = p.smooth ? (float)(1.0 / p.hsd[t]) : 0.0f;
        }
        r.hs2s = (float)(p.hs2d / (u * u));
        r.hs2s_early = (float)(p.hs2d_early / (u * u));
    }
    r.items3 = h.nd * h.nd * h.nd; // a sort work item covers a cell in every plane
    r.items4 = items4_of(s, h.n, h.nd);
    r.items4b = bulk_items_of(s, h.n, h.nd);
    build_shape(s, h.n, h.nd, r.bparts, r.blanes);
    return r;
}

// Convert one particle's FP64 position (already folded into [0, L)) and
// velocity into state words and its snapshot.
static void encode_particle(const md_system *s, const RepDev &r, double x[3], double v[3], int *img,
                            uint32_t meta, uint4 *w, uint4 *snap)
{
    const double h_L = r.L;
    switch (s->prec) {
    case PREC_FP32: {
        float f[3];
        for (int d = 0; d < 3; ++d) {
            // x is in [0, L); its float may round up to L or past it, which
            // is folded by the exact edge (the box need not be a float)
            f[d] = (float)x[d];
            if ((double)f[d] >= h_L) { f[d] = (float)((double)f[d] - h_L); img[d] += 1; }
            x[d] = (double)f[d];
        }
        put_f4(w[0], f[0], f[1], f[2], 0.0f);
        put_f4(w[1], (float)v[0], (float)v[1], (float)v[2], 0.0f);
        break;
    }
    case PREC_DS: {
        float h[3], l[3], vh[3], vl[3];
        for (int d = 0; d < 3; ++d) {
            h[d] = (float)x[d];
            l[d] = (float)(x[d] - (double)h[d]);
            x[d] = (double)h[d] + (double)l[d];
            vh[d] = (float)v[d];
            vl[d] = (float)(v[d] - (double)vh[d]);
        }
        put_f4(w[0], h[0], h[1], h[2], l[0]);
        put_f4(w[1], l[1], l[2], vh[0], vh[1]);
        put_f4(w[2], vh[2], vl[0], vl[1], vl[2]);
        break;
    }
    default:
        put_dbl2(w[0], x[0], x[1]);
        put_dbl2(w[1], x[2], v[0]);
        put_dbl2(w[2], v[1], v[2]);
        break;
    }
    if (s->prec == PREC_FP64) {
        put_dbl2(snap[0], x[0], x[1]);
        put_dbl2(snap[1], x[2], bits_of_meta(meta));
    } else {
        snap[0] = make_uint4(to_fixed(x[0], r.fxs), to_fixed(x[1], r.fxs), to_fixed(x[2], r.fxs), meta);
    }
}

static int cell_of_snap(const md_system *s, const RepDev &r, const uint4 *sn)
{
    if (r.nd == 1) return 0;
    if (s->prec == PREC_FP64) {
        double x, y, z, w;
        get_dbl2(sn[0], x, y);
        get_dbl2(sn[1], z, w);
        return dbl_cell(x, y, z, r.L, r.invL, r.nd);
    }
    return fixed_cell(sn[0].x, sn[0].y, sn[0].z, r.nd);
}

static uint32_t meta_word(int slot, int species) { return ((uint32_t)(species & 1) << 31) | ((uint32_t)slot << SLOT_SHIFT); }

static md_status validate_rep(md_system *s, const md_replica *rep)
{
    if (!rep) return fail(s, MD_E_ARG, "null replica");
    if (rep->n < 1) return fail(s, MD_E_ARG, "replica needs n >= 1");
    if (!(rep->box > 0) || !std::isfinite(rep->box)) return fail(s, MD_E_ARG, "box must be positive");
    if (rep->box < 2.0 * s->rlist_max)
        return fail(s, MD_E_BOX, "box %.6g shorter than twice the largest list radius %.6g", rep->box, s->rlist_max);
    return MD_OK;
}

static md_status upload_slot(md_system *s, int slot, const SlotHost &h, const HostRep &hr,
                             const std::vector<uint4> *xref_override, Ctl c, int64_t nreb, int status)
{
    const int64_t n = h.n, P = s->lay.P;
    const int NW = s->lay.NW, NS = s->lay.NS;
    hipStream_t st = s->stream;
    for (int k = 0; k < NW; ++k)
        HIPCHK(s, hipMemcpyAsync(s->st[k] + h.off, hr.st[k].data(), 16 * n, hipMemcpyHostToDevice, st));
    for (int w = 0; w < NS; ++w) {
        for (int p = 0; p < 2; ++p)
            HIPCHK(s, hipMemcpyAsync(s->snap[p] + w * P + h.off, hr.snap.data() + w * n, 16 * n,
                                     hipMemcpyHostToDevice, st));
        const std::vector<uint4> &xr = xref_override ? *xref_override : hr.snap;
        HIPCHK(s, hipMemcpyAsync(s->xref + w * P + h.off, xr.data() + w * n, 16 * n, hipMemcpyHostToDevice, st));
    }
    HIPCHK(s, hipMemcpyAsync(s->meta + h.off, hr.meta.data(), 16 * n, hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->cs + h.coff, hr.cs.data(), 4 * hr.cs.size(), hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->cs_new + h.coff, hr.cs.data(), 4 * hr.cs.size(), hipMemcpyHostToDevice, st));
    RepDev r = repdev_of(s, h);
    const std::vector<int> rk = ranks_of(s, h); // kept until the stream synchronises below
    if (r.curve) HIPCHK(s, hipMemcpyAsync(s->corder + h.coff, rk.data(), 4 * rk.size(), hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->rep + slot, &r, sizeof r, hipMemcpyHostToDevice, st));
    for (int p = 0; p < 2; ++p) {
        HIPCHK(s, hipMemcpyAsync(s->ctl[p] + slot, &c, sizeof c, hipMemcpyHostToDevice, st));
        HIPCHK(s, launch_poke(s->need[p] + slot, 0, st));
    }
    HIPCHK(s, launch_poke(s->target + slot, c.x, st));
    HIPCHK(s, launch_poke(s->status + slot, status, st));
    HIPCHK(s, launch_poke(s->nreb + slot, (int)nreb, st));
    HIPCHK(s, hipStreamSynchronize(st));
    return MD_OK;
}

static md_status alloc_slot_ranges(md_system *s, int slot, int n, double L, SlotHost &h)
{
    h.n = n;
    h.L = L;
    h.nd = cells_per_edge(L, s->rlist_max);
    int64_t ncell = (int64_t)h.nd * h.nd * h.nd;
    if (ncell > (int64_t)1 << 30) return fail(s, MD_E_ARG, "too many cells");
    if (!s->parena.alloc(n, h.off)) return fail(s, MD_E_CAPACITY, "particle arena full (need %d)", n);
    h.ncell_alloc = s->cfg.n_species * ncell + 1; // a cell range per species plane
    if (!s->carena.alloc(h.ncell_alloc, h.coff)) {
        s->parena.release(h.off, n);
        return fail(s, MD_E_CAPACITY, "cell arena full (need %lld)", (long long)h.ncell_alloc);
    }
    (void)slot;
    return MD_OK;
}

static void release_slot_ranges(md_system *s, SlotHost &h)
{
    s->parena.release(h.off, h.n);
    s->carena.release(h.coff, h.ncell_alloc);
    h.attached = false;
}

// Error bits that stop a replica, and the status a call reports for them.
constexpr int MD_ST_ERRORS = MD_ST_LIST_OVERFLOW | MD_ST_NONFINITE | MD_ST_LOST | MD_ST_NO_PAD;

static md_status status_of_bits(int bits)
{
    if (bits & (MD_ST_NONFINITE | MD_ST_LOST)) return MD_E_NONFINITE;
    if (bits & (MD_ST_LIST_OVERFLOW | MD_ST_NO_PAD)) return MD_E_CAPACITY;
    return MD_OK;
}

// Record the device status bits read at a synchronising call; report the
// first failed slot.
static md_status note_failures(md_system *s, const int *bits)
{
    md_status worst = MD_OK;
    for (size_t k = 0; k < s->slots.size(); ++k) {
        SlotHost &h = s->slots[k];
        if (!h.attached) continue;
        h.failed = bits[k] & MD_ST_ERRORS;
        const md_status st = status_of_bits(h.failed);
        if (st != MD_OK && worst == MD_OK) {
            worst = fail(s, st, "replica in slot %d stopped: status bits 0x%x (%s)", (int)k, h.failed,
                         st == MD_E_CAPACITY ? "a Verlet list exceeded its capacity or could not be padded"
                                             : "non-finite coordinates");
        }
    }
    return worst;
}

// Launching calls refuse to run while a replica known to have failed is
// attached (it would only idle): the caller detaches or restores it first.
static md_status refuse_if_failed(md_system *s)
{
    for (size_t k = 0; k < s->slots.size(); ++k) {
        const SlotHost &h = s->slots[k];
        if (h.attached && h.failed)
            return fail(s, status_of_bits(h.failed),
                        "replica in slot %d stopped with status bits 0x%x; detach or restore it first", (int)k,
                        h.failed);
    }
    return MD_OK;
}

static md_status check_slot(md_system *s, int slot, bool want_attached)
{
    if (!s) return MD_E_ARG;
    if (slot < 0 || slot >= (int)s->lay.slots) return fail(s, MD_E_NOSLOT, "slot %d out of range", slot);
    if (s->slots[slot].attached != want_attached)
        return fail(s, MD_E_NOSLOT, "slot %d is %s", slot, want_attached ? "empty" : "in use");
    return MD_OK;
}

static md_status finish_attach(md_system *s, int slot)
{
    md_status st = upload_items(s);
    if (st != MD_OK) return st;
    st = launch_build_main(s, slot);
    if (st != MD_OK) return st;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    int status = 0;
    HIPCHK(s, hipMemcpy(&status, s->status + slot, 4, hipMemcpyDeviceToHost));
    if (status & MD_ST_LIST_OVERFLOW)
        return fail(s, MD_E_CAPACITY, "neighbour list overflow at attach (capacity %lld)", (long long)s->lay.cap);
    return MD_OK;
}

// ================================================================== C ABI
extern "C" {

int32_t md_abi_version(void) { return MD_ABI_VERSION; }

md_status md_cell_order(int32_t nd, int32_t order, int32_t *rank)
{
    if (nd < 1 || nd > 1024 || !rank) return MD_E_ARG;
    if (order != MD_ORDER_ROW && order != MD_ORDER_MORTON && order != MD_ORDER_HILBERT) return MD_E_ARG;
    cell_ranks(nd, order, rank);
    return MD_OK;
}

const char *md_strerror(md_status st)
{
    switch (st) {
    case MD_OK: return "ok";
    case MD_E_ARG: return "invalid argument";
    case MD_E_BOX: return "box shorter than twice the list radius";
    case MD_E_WORKSPACE: return "workspace missing, misaligned or too small";
    case MD_E_CAPACITY: return "capacity exceeded";
    case MD_E_NONFINITE: return "non-finite coordinates";
    case MD_E_HIP: return "HIP runtime error";
    case MD_E_NOSLOT: return "bad slot";
    case MD_E_STATE: return "invalid state";
    }
    return "unknown status";
}

const char *md_last_error(const md_system *s) { return s ? s->err.c_str() : ""; }

md_status md_validate(const md_config *cfg, const md_replica *rep)
{
    md_status st = validate_cfg(cfg, nullptr);
    if (st != MD_OK) return st;
    if (rep) {
        if (rep->n < 1 || !(rep->box > 0) || !std::isfinite(rep->box)) return MD_E_ARG;
        const double rl = rlist_max_of(cfg);
        if (rep->box < 2.0 * rl) return MD_E_BOX;
        // would it fit an empty pool: particles in the arena, cells of every
        // species plane in the cell arena
        const Layout L = layout_of(cfg);
        const int64_t nd = cells_per_edge(rep->box, rl);
        if (rep->n > cfg->max_particles || cfg->n_species * nd * nd * nd + 1 > L.cells) return MD_E_CAPACITY;
    }
    return MD_OK;
}

int64_t md_workspace_bytes(const md_config *cfg)
{
    md_status st = validate_cfg(cfg, nullptr);
    if (st != MD_OK) return st;
    Layout L = layout_of(cfg);
    return carve(nullptr, L, nullptr);
}

md_status md_create(const md_config *cfg, void *workspace, int64_t ws_bytes, void *hip_stream, md_system **out)
{
    if (!out) return MD_E_ARG;
    *out = nullptr;
    std::string why;
    if (validate_cfg(cfg, &why) != MD_OK) return MD_E_ARG;
    Layout L = layout_of(cfg);
    int64_t need = carve(nullptr, L, nullptr);
    if (!workspace || ws_bytes < need || ((uintptr_t)workspace % ALIGN) != 0) return MD_E_WORKSPACE;
    md_system *s = new md_system();
    s->cfg = *cfg;
    s->prec = cfg->precision;
    s->lpp = cfg->lanes_per_particle > 0 ? cfg->lanes_per_particle : MD_DEFAULT_LPP;
    s->lay = L;
    s->stream = (hipStream_t)hip_stream;
    s->ws = (char *)workspace;
    s->ws_bytes = ws_bytes;
    carve(s, L, s->ws);
    s->launch.step_block = 512;
    s->launch.build_width = 8;
    s->launch.build_block = 512;
    s->launch.graph_steps = 32;
    s->launch.xcd_remap = 0;
    s->launch.build_lanes = 0;
    s->launch.build_split = 0;
    s->launch.build_bulk = 0;
    make_tables(s);
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&s->n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            size_grids(s) != MD_OK || thermo_scratch_init(dev) != hipSuccess) {
            delete s;
            return MD_E_HIP;
        }
        s->dev = dev;
    }
    s->slots.assign(L.slots, SlotHost());
    s->parena.reset(L.P);
    s->carena.reset(L.cells);
    // every snapshot slot starts as "no replica"; control words zero
    hipStream_t st = s->stream;
    auto done = [&](hipError_t e) {
        if (e != hipSuccess) { delete s; return false; }
        return true;
    };
    if (!done(hipMemsetAsync(s->snap[0], 0xFF, 16 * L.P * L.NS, st))) return MD_E_HIP;
    if (!done(hipMemsetAsync(s->snap[1], 0xFF, 16 * L.P * L.NS, st))) return MD_E_HIP;
    if (!done(hipMemsetAsync(s->nbr_cnt, 0, 4 * L.P, st))) return MD_E_HIP;
    if (!done(hipMemsetAsync(s->count[0], 0, 4 * L.cells, st))) return MD_E_HIP;
    if (!done(hipMemsetAsync(s->count[1], 0, 4 * L.cells, st))) return MD_E_HIP;
    if (!done(hipMemsetAsync(s->rep, 0, sizeof(RepDev) * L.slots, st))) return MD_E_HIP;
    for (int p = 0; p < 2; ++p) {
        if (!done(hipMemsetAsync(s->ctl[p], 0, sizeof(Ctl) * L.slots, st))) return MD_E_HIP;
        if (!done(hipMemsetAsync(s->need[p], 0, 4 * L.slots, st))) return MD_E_HIP;
        if (!done(hipMemsetAsync(s->rlist[p], 0, 4 * (L.slots + 1), st))) return MD_E_HIP;
    }
    if (!done(hipMemsetAsync(s->target, 0, 4 * L.slots, st))) return MD_E_HIP;
    if (!done(hipMemsetAsync(s->status, 0, 4 * L.slots, st))) return MD_E_HIP;
    if (!done(hipMemsetAsync(s->nreb, 0, 4 * L.slots, st))) return MD_E_HIP;
    if (!done(hipStreamSynchronize(st))) return MD_E_HIP;
    if (upload_items(s) != MD_OK) { delete s; return MD_E_HIP; }
    *out = s;
    return MD_OK;
}

void md_destroy(md_system *s)
{
    if (!s) return;
    drop_graphs(s);
    delete s;
}

md_status md_attach(md_system *s, int32_t slot, const md_replica *rep, const int32_t *species, const double *pos,
                    const double *vel)
{
    md_status st = check_slot(s, slot, false);
    if (st != MD_OK) return st;
    if ((st = validate_rep(s, rep)) != MD_OK) return st;
    if (!pos || !vel || (!species && s->cfg.n_species == 2)) return fail(s, MD_E_ARG, "null input array");
    const int n = rep->n;
    for (int64_t k = 0; k < 3LL * n; ++k)
        if (!std::isfinite(pos[k]) || !std::isfinite(vel[k])) return fail(s, MD_E_NONFINITE, "non-finite input");
    if (species)
        for (int k = 0; k < n; ++k)
            if (species[k] < 0 || species[k] >= s->cfg.n_species) return fail(s, MD_E_ARG, "species out of range");
    SlotHost h;
    if ((st = alloc_slot_ranges(s, slot, n, rep->box, h)) != MD_OK) return st;
    RepDev r = repdev_of(s, h);
    const std::vector<int> rank = ranks_of(s, h);
    const int NW = s->lay.NW, NS = s->lay.NS;
    std::vector<uint4> w(3 * (size_t)n), sn(2 * (size_t)n);
    std::vector<int4> mt(n);
    std::vector<int> cell(n);
    for (int k = 0; k < n; ++k) {
        double x[3], v[3];
        int img[3];
        for (int d = 0; d < 3; ++d) {
            double q = pos[3 * k + d];
            double f = std::floor(q / h.L);
            x[d] = q - f * h.L;
            img[d] = (int)f;
            if (x[d] >= h.L) { x[d] -= h.L; img[d] += 1; }
            if (x[d] < 0) { x[d] += h.L; img[d] -= 1; }
            v[d] = vel[3 * k + d];
        }
        uint32_t m = meta_word(slot, species ? species[k] : 0);
        encode_particle(s, r, x, v, img, m, &w[3 * (size_t)k], &sn[2 * (size_t)k]);
        mt[k] = make_int4(img[0], img[1], img[2], k);
        cell[k] = sort_key(rank[cell_of_snap(s, r, &sn[2 * (size_t)k])], m, r.planes, r.nd);
    }
    // stable counting sort by species plane and cell
    const int ncell = r.planes * h.nd * h.nd * h.nd;
    HostRep hr;
    hr.cs.assign(ncell + 1, 0);
    for (int k = 0; k < n; ++k) hr.cs[cell[k] + 1]++;
    for (int c = 0; c < ncell; ++c) hr.cs[c + 1] += hr.cs[c];
    std::vector<int> pos_in(ncell);
    for (int c = 0; c < ncell; ++c) pos_in[c] = hr.cs[c];
    std::vector<int> order(n);
    for (int k = 0; k < n; ++k) order[pos_in[cell[k]]++] = k;
    for (int c = 0; c <= ncell; ++c) hr.cs[c] += (int)h.off;
    for (int q = 0; q < NW; ++q) hr.st[q].resize(n);
    hr.snap.resize((size_t)NS * n);
    hr.meta.resize(n);
    for (int k = 0; k < n; ++k) {
        int o = order[k];
        for (int q = 0; q < NW; ++q) hr.st[q][k] = w[3 * (size_t)o + q];
        for (int q = 0; q < NS; ++q) hr.snap[(size_t)q * n + k] = sn[2 * (size_t)o + q];
        hr.meta[k] = mt[o];
    }
    h.attached = true;
    h.target = 0;
    s->slots[slot] = h;
    Ctl c = make_int4(0, 1, 1, 0);
    st = upload_slot(s, slot, h, hr, nullptr, c, 1, 0);
    if (st == MD_OK) st = finish_attach(s, slot);
    if (st != MD_OK) {
        release_slot_ranges(s, s->slots[slot]);
        Ctl z = make_int4(0, 0, 0, 0);
        for (int p = 0; p < 2; ++p) (void)hipMemcpyAsync(s->ctl[p] + slot, &z, sizeof z, hipMemcpyHostToDevice, s->stream);
        (void)hipStreamSynchronize(s->stream);
        upload_items(s);
        return st;
    }
    return MD_OK;
}

md_status md_init(const md_config *cfg, const md_replica *reps, int32_t n_rep, const int32_t *species,
                  const double *pos, const double *vel, void *workspace, int64_t ws_bytes, void *hip_stream,
                  md_system **out)
{
    if (!out || !reps || n_rep < 1 || !cfg || n_rep > cfg->max_slots) return MD_E_ARG;
    md_status st = md_create(cfg, workspace, ws_bytes, hip_stream, out);
    if (st != MD_OK) return st;
    int64_t off = 0;
    for (int k = 0; k < n_rep; ++k) {
        st = md_attach(*out, k, &reps[k], species ? species + off : nullptr, pos + 3 * off, vel + 3 * off);
        if (st != MD_OK) return st; // *out stays valid: the caller reads md_last_error, then md_destroy
        off += reps[k].n;
    }
    return MD_OK;
}

md_status md_detach(md_system *s, int32_t slot)
{
    md_status st = check_slot(s, slot, true);
    if (st != MD_OK) return st;
    SlotHost &h = s->slots[slot];
    Ctl z = make_int4(0, 0, 0, 0);
    for (int p = 0; p < 2; ++p) {
        HIPCHK(s, hipMemcpyAsync(s->ctl[p] + slot, &z, sizeof z, hipMemcpyHostToDevice, s->stream));
        for (int w = 0; w < s->lay.NS; ++w)
            HIPCHK(s, hipMemsetAsync(s->snap[p] + w * s->lay.P + h.off, 0xFF, 16 * (size_t)h.n, s->stream));
    }
    HIPCHK(s, hipStreamSynchronize(s->stream));
    release_slot_ranges(s, h);
    h.failed = 0;
    return upload_items(s);
}

// The observation launch writes each force as one double into the rows
// where a finalising launch keeps its forces for the next step.  In double-
// single those rows hold both words of each sum, which one double need not
// represent, so the next step evaluates the forces again.
static hipError_t void_stored_after_obs(md_system *s)
{
    if (s->prec != MD_DS) return hipSuccess;
    return launch_void_stored(s->ctl[s->parity], (int)s->lay.slots, s->stream);
}

md_status md_rebuild_neighbours(md_system *s)
{
    if (!s) return MD_E_ARG;
    const int p = s->parity, kp = p ^ 1;
    // the re-sort moves particles between slots: forces stored by slot are void
    HIPCHK(s, launch_void_stored(s->ctl[p], (int)s->lay.slots, s->stream));
    HIPCHK(s, hipMemsetAsync(s->count[kp], 0, 4 * s->lay.cells, s->stream));
    CountArgs ca;
    memset(&ca, 0, sizeof ca);
    ca.P = (int)s->lay.P;
    ca.max_slots = (int)s->lay.slots;
    ca.force_slot = -2;
    ca.snap = s->snap[p];
    ca.rep = s->rep;
    ca.ctl = s->ctl[p];
    ca.count = s->count[kp];
    ca.corder = s->corder;
    HIPCHK(s, launch_count(s->prec, ca, s->stream));
    // the rebuild kernels of a step of parity kp read snap[kp ^ 1] == snap[p]
    return launch_rebuild(s, kp, -2, true);
}

md_status md_forces(md_system *s, int32_t slot, double *f_host, double *e_host)
{
    if (!s) return MD_E_ARG;
    StepArgs a = step_args(s, s->parity);
    HIPCHK(s, launch_step(s->prec, a, s->launch.step_block, true, s->stream));
    HIPCHK(s, void_stored_after_obs(s));
    if (!f_host && !e_host) return MD_OK;
    md_status st = check_slot(s, slot, true);
    if (st != MD_OK) return st;
    const SlotHost &h = s->slots[slot];
    std::vector<double> o((size_t)h.n * 8);
    std::vector<int4> mt(h.n);
    HIPCHK(s, hipMemcpyAsync(o.data(), s->obs + h.off * 8, 8 * o.size(), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(mt.data(), s->meta + h.off, 16 * (size_t)h.n, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (int k = 0; k < h.n; ++k) {
        int id = mt[k].w;
        if (id < 0 || id >= h.n) return fail(s, MD_E_STATE, "corrupt particle ids");
        if (f_host) for (int d = 0; d < 3; ++d) f_host[3 * id + d] = o[8 * k + d];
        if (e_host) e_host[id] = o[8 * k + 3];
    }
    return MD_OK;
}

md_status md_step(md_system *s, int64_t n_steps)
{
    if (!s) return MD_E_ARG;
    if (n_steps < 0 || n_steps > (1LL << 30)) return fail(s, MD_E_ARG, "n_steps out of range");
    if (n_steps == 0) return MD_OK;
    if (md_status st = refuse_if_failed(s); st != MD_OK) return st;
    for (auto &h : s->slots)
        if (h.attached) {
            if (h.target + n_steps > 2000000000LL) return fail(s, MD_E_ARG, "step counter would overflow");
            h.target += n_steps;
        }
    HIPCHK(s, launch_add_targets(s->target, s->ctl[s->parity], (int)s->lay.slots, (int)n_steps, s->stream));
    return run_launches(s, n_steps + 1);
}

md_status md_set_target(md_system *s, int32_t slot, int64_t target_step)
{
    md_status st = check_slot(s, slot, true);
    if (st != MD_OK) return st;
    if (target_step < 0 || target_step > 2000000000LL) return fail(s, MD_E_ARG, "target out of range");
    s->slots[slot].target = target_step;
    HIPCHK(s, launch_poke(s->target + slot, (int)target_step, s->stream));
    return MD_OK;
}

md_status md_advance(md_system *s, int64_t n_launch)
{
    if (!s) return MD_E_ARG;
    if (n_launch < 0) return fail(s, MD_E_ARG, "n_launch < 0");
    if (md_status st = refuse_if_failed(s); st != MD_OK) return st;
    return run_launches(s, n_launch);
}

md_status md_poll(md_system *s, int64_t *steps, int32_t *status)
{
    if (!s) return MD_E_ARG;
    const int S = (int)s->lay.slots;
    std::vector<Ctl> c(S);
    std::vector<int> stv(S);
    HIPCHK(s, hipMemcpyAsync(c.data(), s->ctl[s->parity], sizeof(Ctl) * S, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(stv.data(), s->status, 4 * S, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (int k = 0; k < S; ++k) {
        bool att = s->slots[k].attached;
        if (steps) steps[k] = att ? c[k].x : -1;
        if (status) status[k] = att ? (stv[k] | (c[k].y ? MD_ST_AT_FULL_STEP : 0)) : 0;
    }
    return note_failures(s, stv.data());
}

md_status md_observables(md_system *s, md_obs *out)
{
    if (!s || !out) return MD_E_ARG;
    const int S = (int)s->lay.slots;
    StepArgs a = step_args(s, s->parity);
    HIPCHK(s, launch_step(s->prec, a, s->launch.step_block, true, s->stream));
    HIPCHK(s, void_stored_after_obs(s));
    ObsArgs oa;
    oa.max_slots = S;
    oa.rep = s->rep;
    oa.ctl = s->ctl[s->parity];
    oa.obs = s->obs;
    oa.nbr_cnt = s->nbr_cnt;
    oa.chunk_pref = s->chunks;
    oa.partial = s->partial;
    oa.out = s->obs_out;
    HIPCHK(s, launch_obs_reduce(oa, s->stream));
    std::vector<double> r((size_t)S * 8);
    std::vector<Ctl> c(S);
    std::vector<int> stv(S), nr(S);
    HIPCHK(s, hipMemcpyAsync(r.data(), s->obs_out, 8 * r.size(), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(c.data(), s->ctl[s->parity], sizeof(Ctl) * S, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(stv.data(), s->status, 4 * S, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(nr.data(), s->nreb, 4 * S, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (int k = 0; k < S; ++k) {
        md_obs &o = out[k];
        memset(&o, 0, sizeof o);
        const SlotHost &h = s->slots[k];
        if (!h.attached) continue;
        const double m = s->cfg.mass, V = h.L * h.L * h.L;
        o.n = h.n;
        o.epot = r[8 * k + 0];
        o.virial = r[8 * k + 1];
        o.ekin = 0.5 * m * r[8 * k + 2];
        o.etot = o.epot + o.ekin;
        o.temperature = 2.0 * o.ekin / (3.0 * h.n);
        o.pressure = (2.0 * o.ekin + o.virial) / (3.0 * V);
        for (int d = 0; d < 3; ++d) o.momentum[d] = m * r[8 * k + 3 + d];
        o.step = c[k].x;
        o.list_entries = (int64_t)r[8 * k + 6];
        o.n_rebuilds = nr[k];
        o.status = stv[k];
    }
    return note_failures(s, stv.data());
}

md_status md_scale_velocities(md_system *s, int32_t slot, double factor)
{
    md_status st = check_slot(s, slot, true);
    if (st != MD_OK) return st;
    if (!std::isfinite(factor)) return fail(s, MD_E_ARG, "factor not finite");
    const SlotHost &h = s->slots[slot];
    ScaleArgs a;
    memset(&a, 0, sizeof a);
    a.A = arena_of(s);
    a.off = (int)h.off;
    a.n = h.n;
    a.f_hi = (float)factor;
    a.f_lo = (float)(factor - (double)a.f_hi);
    a.ff = (float)factor;
    a.fd = factor;
    HIPCHK(s, launch_scale_vel(s->prec, a, s->stream));
    return MD_OK;
}

md_status md_thermostat(md_system *s, int32_t slot, double temperature, uint64_t seed, int64_t call,
                        int32_t remove_mean)
{
    md_status st = check_slot(s, slot, true);
    if (st != MD_OK) return st;
    if (!(temperature > 0) || !std::isfinite(temperature)) return fail(s, MD_E_ARG, "temperature must be positive");
    if (call < 0 || call > ((int64_t)1 << 40)) return fail(s, MD_E_ARG, "call index out of range");
    const SlotHost &h = s->slots[slot];
    int chunk0 = 0; // this slot's first row of chunk partials (4096 particles per chunk)
    for (int k = 0; k < slot; ++k)
        if (s->slots[k].attached) chunk0 += (s->slots[k].n + 4095) / 4096;
    ThermoArgs a;
    memset(&a, 0, sizeof a);
    a.A = arena_of(s);
    a.obs = s->obs;
    a.partial = s->partial;
    a.off = (int)h.off;
    a.n = h.n;
    a.chunk0 = chunk0;
    a.nchunk = (h.n + 4095) / 4096;
    a.remove_mean = remove_mean ? 1 : 0;
    a.x0 = ((seed & 0xFFFFFFFFULL) << 16) | 0x330EULL; // the state srand48(seed) sets
    a.call = call;
    a.temperature = temperature;
    a.mass = s->cfg.mass;
    a.scale = std::sqrt(temperature / s->cfg.mass);
    HIPCHK(s, launch_thermostat(s->prec, a, s->stream));
    // the draws went through the scratch rows that hold stored forces
    HIPCHK(s, launch_poke((int *)(s->ctl[s->parity] + slot) + 3, 0, s->stream));
    return MD_OK;
}

md_status md_thermostat_noalloc(md_system *s, int32_t slot, double temperature, uint64_t seed, int64_t call,
                                int32_t remove_mean)
{
    // The same kernels and arithmetic as md_thermostat; the chunk partial
    // sums go to the library's file-scope scratch array of this device, the
    // drawn velocities are drawn again when applied, and nothing here
    // allocates (host or device).
    md_status st = check_slot(s, slot, true);
    if (st != MD_OK) return st;
    if (!(temperature > 0) || !std::isfinite(temperature)) return fail(s, MD_E_ARG, "temperature must be positive");
    if (call < 0 || call > ((int64_t)1 << 40)) return fail(s, MD_E_ARG, "call index out of range");
    const SlotHost &h = s->slots[slot];
    const int nchunk = (h.n + 4095) / 4096;
    if (nchunk > THERMO_SCRATCH_CHUNKS)
        return fail(s, MD_E_CAPACITY, "md_thermostat_noalloc: %d particles exceed its scratch limit of %d",
                    h.n, THERMO_SCRATCH_CHUNKS * 4096);
    double *scr = thermo_scratch(s->dev);
    if (!scr) return fail(s, MD_E_STATE, "scratch array of device %d not set up", s->dev);
    ThermoArgs a;
    memset(&a, 0, sizeof a);
    a.A = arena_of(s);
    a.obs = nullptr;
    a.partial = scr;
    a.off = (int)h.off;
    a.n = h.n;
    a.chunk0 = 0;
    a.nchunk = nchunk;
    a.remove_mean = remove_mean ? 1 : 0;
    a.x0 = ((seed & 0xFFFFFFFFULL) << 16) | 0x330EULL;
    a.call = call;
    a.temperature = temperature;
    a.mass = s->cfg.mass;
    a.scale = std::sqrt(temperature / s->cfg.mass);
    HIPCHK(s, launch_thermostat(s->prec, a, s->stream));
    return MD_OK;
}

md_status md_profile_steps(md_system *s, int64_t n_steps, double *out)
{
    if (!s || !out) return MD_E_ARG;
    if (n_steps < 1 || n_steps > 65536) return fail(s, MD_E_ARG, "n_steps out of range [1, 65536]");
    const int S = (int)s->lay.slots;
    const int64_t R = n_steps + 2; // counter rows: before, after each launch
    int *hn = nullptr;
    HIPCHK(s, hipHostMalloc((void **)&hn, (size_t)R * S * 4, hipHostMallocDefault));
    std::vector<hipEvent_t> ev;
    ev.reserve(3 * (size_t)(n_steps + 1));
    md_status st = MD_OK;
    auto cleanup = [&]() {
        for (auto &e : ev) (void)hipEventDestroy(e);
        (void)hipHostFree(hn);
    };
    for (int64_t k = 0; k < 3 * (n_steps + 1) && st == MD_OK; ++k) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) st = fail(s, MD_E_HIP, "hipEventCreate failed");
        else ev.push_back(e);
    }
    if (st != MD_OK) { cleanup(); return st; }
    for (auto &h : s->slots)
        if (h.attached) h.target += n_steps;
    auto chk = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && st == MD_OK) st = fail(s, MD_E_HIP, what);
    };
    chk(launch_add_targets(s->target, s->ctl[s->parity], S, (int)n_steps, s->stream), "add targets");
    chk(hipMemcpyAsync(hn, s->nreb, 4 * S, hipMemcpyDeviceToHost, s->stream), "copy counters");
    for (int64_t k = 0; k <= n_steps && st == MD_OK; ++k) { // the last launch finalises
        const int p = s->parity;
        StepArgs a = step_args(s, p);
        chk(hipEventRecord(ev[3 * k], s->stream), "event");
        chk(launch_step(s->prec, a, s->launch.step_block, false, s->stream), "step launch");
        chk(hipEventRecord(ev[3 * k + 1], s->stream), "event");
        if (st == MD_OK) st = launch_rebuild(s, p, -1, true);
        chk(hipEventRecord(ev[3 * k + 2], s->stream), "event");
        chk(hipMemcpyAsync(hn + (k + 1) * S, s->nreb, 4 * S, hipMemcpyDeviceToHost, s->stream), "copy counters");
        s->parity ^= 1;
    }
    chk(hipStreamSynchronize(s->stream), "synchronise");
    if (st != MD_OK) { cleanup(); return st; }
    double t_step = 0, t_reb = 0, t_reb_hit = 0, n_hit = 0;
    auto rowsum = [&](int64_t r) {
        long long t = 0;
        for (int q = 0; q < S; ++q) t += hn[r * S + q];
        return t;
    };
    for (int64_t k = 0; k < n_steps && st == MD_OK; ++k) {
        float a01 = 0, a12 = 0;
        chk(hipEventElapsedTime(&a01, ev[3 * k], ev[3 * k + 1]), "elapsed");
        chk(hipEventElapsedTime(&a12, ev[3 * k + 1], ev[3 * k + 2]), "elapsed");
        t_step += a01;
        t_reb += a12;
        if (rowsum(k + 1) != rowsum(k)) { t_reb_hit += a12; n_hit += 1; }
    }
    float tot = 0;
    chk(hipEventElapsedTime(&tot, ev[0], ev[3 * (n_steps - 1) + 2]), "elapsed");
    cleanup();
    if (st != MD_OK) return st;
    out[0] = t_step / n_steps;
    out[1] = t_reb / n_steps;
    out[2] = n_hit > 0 ? t_reb_hit / n_hit : 0.0;
    out[3] = n_hit;
    out[4] = tot;
    return MD_OK;
}

md_status md_sync(md_system *s)
{
    if (!s) return MD_E_ARG;
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return MD_OK;
}

static md_status download_slot(md_system *s, const SlotHost &h, HostRep &hr, std::vector<uint4> &xref)
{
    const int64_t n = h.n, P = s->lay.P;
    const int NW = s->lay.NW, NS = s->lay.NS;
    for (int q = 0; q < NW; ++q) {
        hr.st[q].resize(n);
        HIPCHK(s, hipMemcpyAsync(hr.st[q].data(), s->st[q] + h.off, 16 * n, hipMemcpyDeviceToHost, s->stream));
    }
    hr.snap.resize(NS * n);
    xref.resize(NS * n);
    for (int w = 0; w < NS; ++w) {
        HIPCHK(s, hipMemcpyAsync(hr.snap.data() + w * n, s->snap[s->parity] + w * P + h.off, 16 * n,
                                 hipMemcpyDeviceToHost, s->stream));
        HIPCHK(s, hipMemcpyAsync(xref.data() + w * n, s->xref + w * P + h.off, 16 * n, hipMemcpyDeviceToHost,
                                 s->stream));
    }
    hr.meta.resize(n);
    HIPCHK(s, hipMemcpyAsync(hr.meta.data(), s->meta + h.off, 16 * n, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return MD_OK;
}

// Decode a particle's state words into FP64 position and velocity.
static void decode_particle(const md_system *s, const uint4 *w, double x[3], double v[3])
{
    switch (s->prec) {
    case PREC_FP32: {
        float a, b, c, d;
        get_f4(w[0], a, b, c, d);
        x[0] = a; x[1] = b; x[2] = c;
        get_f4(w[1], a, b, c, d);
        v[0] = a; v[1] = b; v[2] = c;
        break;
    }
    case PREC_DS: {
        float a0, a1, a2, a3, b0, b1, b2, b3, c0, c1, c2, c3;
        get_f4(w[0], a0, a1, a2, a3);
        get_f4(w[1], b0, b1, b2, b3);
        get_f4(w[2], c0, c1, c2, c3);
        x[0] = (double)a0 + (double)a3;
        x[1] = (double)a1 + (double)b0;
        x[2] = (double)a2 + (double)b1;
        v[0] = (double)b2 + (double)c1;
        v[1] = (double)b3 + (double)c2;
        v[2] = (double)c0 + (double)c3;
        break;
    }
    default:
        get_dbl2(w[0], x[0], x[1]);
        get_dbl2(w[1], x[2], v[0]);
        get_dbl2(w[2], v[1], v[2]);
    }
}

md_status md_get_state(md_system *s, int32_t slot, double *pos, double *vel, int32_t *image)
{
    md_status st = check_slot(s, slot, true);
    if (st != MD_OK) return st;
    const SlotHost &h = s->slots[slot];
    HostRep hr;
    std::vector<uint4> xr;
    if ((st = download_slot(s, h, hr, xr)) != MD_OK) return st;
    for (int k = 0; k < h.n; ++k) {
        uint4 w[3] = {hr.st[0][k], hr.st[1][k], s->lay.NW > 2 ? hr.st[2][k] : make_uint4(0, 0, 0, 0)};
        double x[3], v[3];
        decode_particle(s, w, x, v);
        int img[3] = {hr.meta[k].x, hr.meta[k].y, hr.meta[k].z};
        int id = hr.meta[k].w;
        if (id < 0 || id >= h.n) return fail(s, MD_E_STATE, "corrupt particle ids");
        for (int d = 0; d < 3; ++d) {
            double f = std::floor(x[d] / h.L);
            double q = x[d] - f * h.L;
            int im = img[d] + (int)f;
            if (q >= h.L) { q -= h.L; im += 1; }
            if (q < 0) { q += h.L; im -= 1; }
            if (pos) pos[3 * id + d] = q;
            if (vel) vel[3 * id + d] = v[d];
            if (image) image[3 * id + d] = im;
        }
    }
    return MD_OK;
}

struct CkptHeader {
    uint32_t magic;
    int32_t version, precision, n_species, n, NW, NS, nd, lpp;
    double L, dt, skin, mass, eps[4], sigma[4], rcut[4];
    int64_t step, fresh, nreb, status;
    int64_t rebuild_every;
    double rebuild_early, smooth;
};

int64_t md_checkpoint_bytes(md_system *s, int32_t slot)
{
    md_status st = check_slot(s, slot, true);
    if (st != MD_OK) return st;
    const int64_t n = s->slots[slot].n;
    return (int64_t)sizeof(CkptHeader) + 16 * n * (s->lay.NW + 2 * s->lay.NS + 1);
}

md_status md_save(md_system *s, int32_t slot, void *blob, int64_t bytes)
{
    md_status st = check_slot(s, slot, true);
    if (st != MD_OK) return st;
    if (!blob || bytes < md_checkpoint_bytes(s, slot)) return fail(s, MD_E_ARG, "checkpoint buffer too small");
    const SlotHost &h = s->slots[slot];
    HostRep hr;
    std::vector<uint4> xr;
    if ((st = download_slot(s, h, hr, xr)) != MD_OK) return st;
    Ctl c;
    int stv = 0, nr = 0;
    HIPCHK(s, hipMemcpy(&c, s->ctl[s->parity] + slot, sizeof c, hipMemcpyDeviceToHost));
    HIPCHK(s, hipMemcpy(&stv, s->status + slot, 4, hipMemcpyDeviceToHost));
    HIPCHK(s, hipMemcpy(&nr, s->nreb + slot, 4, hipMemcpyDeviceToHost));
    CkptHeader H;
    memset(&H, 0, sizeof H);
    H.magic = CKPT_MAGIC;
    H.version = CKPT_VERSION;
    H.precision = s->prec;
    H.n_species = s->cfg.n_species;
    H.n = h.n;
    H.NW = s->lay.NW;
    H.NS = s->lay.NS;
    H.nd = h.nd;
    H.lpp = s->lpp;
    H.L = h.L;
    H.dt = s->cfg.dt;
    H.skin = s->cfg.skin;
    H.mass = s->cfg.mass;
    memcpy(H.eps, s->cfg.eps, sizeof H.eps);
    memcpy(H.sigma, s->cfg.sigma, sizeof H.sigma);
    memcpy(H.rcut, s->cfg.rcut, sizeof H.rcut);
    H.step = c.x;
    H.fresh = c.y;
    H.rebuild_every = s->cfg.rebuild_every;
    H.rebuild_early = s->cfg.rebuild_every ? s->cfg.rebuild_early : 0.0;
    H.smooth = s->cfg.smooth;
    H.nreb = nr;
    H.status = stv;
    char *b = (char *)blob;
    memcpy(b, &H, sizeof H);
    b += sizeof H;
    const int64_t n = h.n;
    for (int q = 0; q < s->lay.NW; ++q) { memcpy(b, hr.st[q].data(), 16 * n); b += 16 * n; }
    memcpy(b, hr.snap.data(), 16 * n * s->lay.NS); b += 16 * n * s->lay.NS;
    memcpy(b, xr.data(), 16 * n * s->lay.NS); b += 16 * n * s->lay.NS;
    memcpy(b, hr.meta.data(), 16 * n);
    return MD_OK;
}

md_status md_restore(md_system *s, int32_t slot, const void *blob, int64_t bytes)
{
    md_status st = check_slot(s, slot, false);
    if (st != MD_OK) return st;
    if (!blob || bytes < (int64_t)sizeof(CkptHeader)) return fail(s, MD_E_ARG, "checkpoint too small");
    CkptHeader H;
    memcpy(&H, blob, sizeof H);
    if (H.magic != CKPT_MAGIC || H.version != CKPT_VERSION) return fail(s, MD_E_ARG, "not a checkpoint");
    if (H.precision != s->prec || H.lpp != s->lpp || H.n_species != s->cfg.n_species || H.dt != s->cfg.dt || H.skin != s->cfg.skin ||
        H.mass != s->cfg.mass || memcmp(H.eps, s->cfg.eps, sizeof H.eps) || memcmp(H.sigma, s->cfg.sigma, sizeof H.sigma) ||
        memcmp(H.rcut, s->cfg.rcut, sizeof H.rcut) || H.rebuild_every != s->cfg.rebuild_every ||
        H.rebuild_early != (s->cfg.rebuild_every ? s->cfg.rebuild_early : 0.0) || H.smooth != s->cfg.smooth)
        return fail(s, MD_E_ARG, "checkpoint from an incompatible pool");
    const int64_t n = H.n;
    if (n < 1 || bytes < (int64_t)sizeof(CkptHeader) + 16 * n * (H.NW + 2 * H.NS + 1))
        return fail(s, MD_E_ARG, "checkpoint truncated");
    md_replica rep;
    rep.n = (int)n;
    rep.box = H.L;
    if ((st = validate_rep(s, &rep)) != MD_OK) return st;
    SlotHost h;
    if ((st = alloc_slot_ranges(s, slot, (int)n, H.L, h)) != MD_OK) return st;
    if (h.nd != H.nd) { release_slot_ranges(s, h); return fail(s, MD_E_ARG, "cell grid mismatch"); }
    RepDev r = repdev_of(s, h);
    const std::vector<int> rank = ranks_of(s, h);
    const char *b = (const char *)blob + sizeof H;
    HostRep hr;
    for (int q = 0; q < H.NW; ++q) { hr.st[q].resize(n); memcpy(hr.st[q].data(), b, 16 * n); b += 16 * n; }
    hr.snap.resize(n * H.NS);
    memcpy(hr.snap.data(), b, 16 * n * H.NS); b += 16 * n * H.NS;
    std::vector<uint4> xr(n * H.NS);
    memcpy(xr.data(), b, 16 * n * H.NS); b += 16 * n * H.NS;
    hr.meta.resize(n);
    memcpy(hr.meta.data(), b, 16 * n);
    // re-tag the slot in the meta words and recover the cell starts
    const int ncell = r.planes * h.nd * h.nd * h.nd;
    hr.cs.assign(ncell + 1, 0);
    int prev = 0;
    for (int64_t k = 0; k < n; ++k) {
        for (std::vector<uint4> *v : {&hr.snap, &xr}) {
            if (H.NS == 2) {
                double z, w;
                get_dbl2((*v)[n + k], z, w);
                put_dbl2((*v)[n + k], z, bits_of_meta(meta_word(slot, species_of(meta_of_bits(w)))));
            } else {
                (*v)[k].w = meta_word(slot, species_of((*v)[k].w));
            }
        }
        uint4 sn[2] = {xr[k], H.NS == 2 ? xr[n + k] : make_uint4(0, 0, 0, 0)};
        uint32_t mw = sn[0].w;
        if (H.NS == 2) {
            double z, w;
            get_dbl2(sn[1], z, w);
            mw = meta_of_bits(w);
        }
        int c = sort_key(rank[cell_of_snap(s, r, sn)], mw, r.planes, r.nd);
        if (c < prev) { release_slot_ranges(s, h); return fail(s, MD_E_ARG, "checkpoint order is not by cell"); }
        prev = c;
        hr.cs[c + 1]++;
    }
    for (int c = 0; c < ncell; ++c) hr.cs[c + 1] += hr.cs[c];
    for (int c = 0; c <= ncell; ++c) hr.cs[c] += (int)h.off;
    h.attached = true;
    h.target = H.step;
    s->slots[slot] = h;
    Ctl c = make_int4((int)H.step, (int)H.fresh, 1, 0);
    st = upload_slot(s, slot, h, hr, &xr, c, H.nreb, (int)H.status);
    if (st == MD_OK) st = finish_attach(s, slot);
    if (st != MD_OK) { release_slot_ranges(s, s->slots[slot]); return st; }
    return MD_OK;
}

md_status md_debug_neighbours(md_system *s, int32_t slot, int32_t *counts, int32_t *ids, int32_t cap)
{
    md_status st = check_slot(s, slot, true);
    if (st != MD_OK) return st;
    if (!counts || !ids || cap < 1) return fail(s, MD_E_ARG, "null output");
    const SlotHost &h = s->slots[slot];
    const int64_t n = h.n, lc = s->lay.cap;
    // the list tiles that hold the replica's slots: one contiguous range
    const int64_t t0 = h.off / LIST_TILE, t1 = (h.off + n + LIST_TILE - 1) / LIST_TILE;
    const size_t row0 = list_row_index((int)(t0 * LIST_TILE), 0, (int)lc);
    std::vector<int> cnt(n), lst((size_t)(t1 - t0) * LIST_TILE * lc);
    std::vector<int4> mt(n);
    HIPCHK(s, hipMemcpyAsync(cnt.data(), s->nbr_cnt + h.off, 4 * n, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(lst.data(), s->nbr + 4 * row0, 4 * lst.size(), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(mt.data(), s->meta + h.off, 16 * n, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    for (int64_t k = 0; k < n; ++k) {
        int id = mt[k].w;
        if (id < 0 || id >= n) return fail(s, MD_E_STATE, "corrupt particle ids");
        counts[id] = cnt[k];
        for (int q = 0; q < cap; ++q) {
            int v = -1;
            if (q < cnt[k] && q < lc) {
                const int lg = s->lpp == 4 ? 2 : s->lpp == 2 ? 1 : 0;
                const size_t r = list_row_index((int)(h.off + k), list_entry_row(q, lg), (int)lc) - row0;
                int j = list_slot(lst[4 * r + list_entry_col(q, lg)]) - (int)h.off;
                v = (j >= 0 && j < n) ? mt[j].w : -2;
            }
            ids[(size_t)id * cap + q] = v;
        }
    }
    return MD_OK;
}

md_status md_get_launch(const md_system *s, md_launch *out)
{
    if (!s || !out) return MD_E_ARG;
    *out = s->launch;
    return MD_OK;
}

md_status md_set_launch(md_system *s, const md_launch *in)
{
    if (!s || !in) return MD_E_ARG;
    const md_launch &l = *in;
    if (l.step_block < 64 || l.step_block > 1024 || l.step_block % 64) return fail(s, MD_E_ARG, "bad step_block");
    if (l.build_block < 64 || l.build_block > 1024 || l.build_block % 64) return fail(s, MD_E_ARG, "bad build_block");
    if (l.build_width < 1 || l.build_width > 16) return fail(s, MD_E_ARG, "bad build_width");
    if (l.build_lanes < 0 || l.build_lanes > 64 || (l.build_lanes & (l.build_lanes - 1)))
        return fail(s, MD_E_ARG, "bad build_lanes");
    if (l.graph_steps != 0 && (l.graph_steps < 2 || l.graph_steps > 256 || l.graph_steps % 2))
        return fail(s, MD_E_ARG, "bad graph_steps");
    if (l.build_split < 0 || l.build_split > 256) return fail(s, MD_E_ARG, "bad build_split");
    if (l.build_bulk < 0) return fail(s, MD_E_ARG, "bad build_bulk");
    drop_graphs(s);
    const md_launch prev = s->launch;
    s->launch = l;
    s->launch.xcd_remap = l.xcd_remap ? 1 : 0;
    const md_status gs = size_grids(s);
    if (gs != MD_OK) {
        const std::string why = s->err;
        s->launch = prev;
        (void)size_grids(s);
        s->err = why;
        return gs;
    }
    // refresh per-slot item counts (list-build items depend on the shapes)
    for (int k = 0; k < (int)s->lay.slots; ++k)
        if (s->slots[k].attached) {
            RepDev r = repdev_of(s, s->slots[k]);
            HIPCHK(s, hipMemcpyAsync(s->rep + k, &r, sizeof r, hipMemcpyHostToDevice, s->stream));
        }
    return upload_items(s);
}

// ------------------------------------------------- time-correlation functions
struct md_tcf {
    md_system *s = nullptr;
    int slot = 0, n = 0, levels = 0, block = 0;
    double q = 0, L = 0;
    int64_t samples = 0;
    std::vector<int64_t> inserted; // entries inserted per level
    std::vector<int64_t> terms;    // correlation passes per level (every lag alike)
    double4 *pos = nullptr;
    double4 *vel = nullptr;
    int *species = nullptr;
    double *partial = nullptr, *acc = nullptr;
};

namespace {
struct TcfLayout {
    int64_t pos, vel, species, partial, acc, total;
};

TcfLayout tcf_layout(int64_t n, int levels, int block)
{
    TcfLayout t;
    int64_t off = 0;
    const int64_t entries = (int64_t)levels * block;
    t.pos = off; off = align_up(off + entries * n * 32, ALIGN);
    t.vel = off; off = align_up(off + entries * n * 32, ALIGN);
    t.species = off; off = align_up(off + n * 4, ALIGN);
    t.partial = off; off = align_up(off + (int64_t)tcf_blocks((int)n) * (block - 1) * 8 * 8, ALIGN);
    t.acc = off; off = align_up(off + (int64_t)levels * (block - 1) * 6 * 8, ALIGN);
    t.total = off;
    return t;
}

bool tcf_shape_ok(int64_t n, int levels, int block)
{
    return n >= 1 && n <= ((int64_t)1 << 30) && levels >= 1 && levels <= 16 && block >= 2 && block <= 33;
}
} // namespace

int64_t md_tcf_workspace_bytes(int32_t n, int32_t levels, int32_t block)
{
    if (!tcf_shape_ok(n, levels, block)) return MD_E_ARG;
    return tcf_layout(n, levels, block).total;
}

md_status md_tcf_create(md_system *s, int32_t slot, int32_t levels, int32_t block, double q, void *workspace,
                        int64_t ws_bytes, md_tcf **out)
{
    if (!s || !out) return MD_E_ARG;
    *out = nullptr;
    if (slot < 0 || slot >= (int)s->lay.slots || !s->slots[slot].attached)
        return fail(s, MD_E_NOSLOT, "slot %d is not attached", slot);
    const SlotHost &h = s->slots[slot];
    if (!tcf_shape_ok(h.n, levels, block)) return fail(s, MD_E_ARG, "levels in [1, 16], block in [2, 33]");
    if (!(q > 0) || !std::isfinite(q)) return fail(s, MD_E_ARG, "q must be positive and finite");
    const TcfLayout t = tcf_layout(h.n, levels, block);
    if (!workspace || ws_bytes < t.total || ((uintptr_t)workspace % ALIGN) != 0)
        return fail(s, MD_E_WORKSPACE, "time-correlation workspace missing, misaligned or smaller than %lld bytes",
                    (long long)t.total);
    md_tcf *c = new md_tcf();
    c->s = s;
    c->slot = slot;
    c->n = h.n;
    c->levels = levels;
    c->block = block;
    c->q = q;
    c->L = h.L;
    c->inserted.assign(levels, 0);
    c->terms.assign(levels, 0);
    char *w = (char *)workspace;
    c->pos = (double4 *)(w + t.pos);
    c->vel = (double4 *)(w + t.vel);
    c->species = (int *)(w + t.species);
    c->partial = (double *)(w + t.partial);
    c->acc = (double *)(w + t.acc);
    if (hipMemsetAsync(c->acc, 0, (size_t)levels * (block - 1) * 6 * 8, s->stream) != hipSuccess) {
        delete c;
        return fail(s, MD_E_HIP, "hipMemsetAsync failed");
    }
    *out = c;
    return MD_OK;
}

md_status md_tcf_sample(md_tcf *c)
{
    if (!c) return MD_E_ARG;
    md_system *s = c->s;
    const SlotHost &h = s->slots[c->slot];
    if (!h.attached || h.n != c->n) return fail(s, MD_E_STATE, "the replica of this scheme was detached");
    TcfArgs a;
    memset(&a, 0, sizeof a);
    a.A = arena_of(s);
    a.snap = s->snap[s->parity];
    a.off = (int)h.off;
    a.n = c->n;
    a.block = c->block;
    a.L = c->L;
    a.q = c->q;
    a.pos = c->pos;
    a.vel = c->vel;
    a.species = c->species;
    a.partial = c->partial;
    a.acc = c->acc;
    int64_t stride = 1; // block^level, the level's resolution in samples
    for (int lev = 0; lev < c->levels; ++lev) {
        if (c->samples % stride) break;
        const int r = (int)(c->inserted[lev] % c->block);
        HIPCHK(s, launch_tcf_store(s->prec, a, lev * c->block + r, s->stream));
        c->inserted[lev] += 1;
        if (c->inserted[lev] >= c->block) { // full: oldest entry against the others, then dropped
            const int head = (int)((c->inserted[lev] - c->block) % c->block);
            HIPCHK(s, launch_tcf_correlate(a, lev, head, s->stream));
            c->terms[lev] += 1;
        }
        if (stride > ((int64_t)1 << 40) / c->block) break;
        stride *= c->block;
    }
    c->samples += 1;
    return MD_OK;
}

md_status md_tcf_read(md_tcf *c, int64_t *lags, double *values, int64_t *terms)
{
    if (!c) return MD_E_ARG;
    md_system *s = c->s;
    const int nl = c->block - 1;
    std::vector<double> acc((size_t)c->levels * nl * 6);
    HIPCHK(s, hipMemcpyAsync(acc.data(), c->acc, acc.size() * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    int64_t stride = 1;
    for (int lev = 0; lev < c->levels; ++lev) {
        for (int j = 1; j <= nl; ++j) {
            const size_t k = (size_t)lev * nl + (j - 1);
            if (lags) lags[k] = j * stride;
            if (terms) terms[k] = c->terms[lev];
            if (values)
                for (int q = 0; q < 6; ++q)
                    values[k * 6 + q] = c->terms[lev] ? acc[k * 6 + q] / (double)c->terms[lev] : NAN;
        }
        stride = stride > ((int64_t)1 << 40) / c->block ? stride : stride * c->block;
    }
    return MD_OK;
}

void md_tcf_destroy(md_tcf *c) { delete c; }

md_status md_ds_eval(int32_t op, int64_t n, const float *a, const float *b, float *out, void *hip_stream)
{
    if (op < 0 || op > 3 || n < 0 || !a || !out || (op < 3 && !b)) return MD_E_ARG;
    hipError_t e = launch_ds_eval(op, n, a, b, out, (hipStream_t)hip_stream);
    return e == hipSuccess ? MD_OK : MD_E_HIP;
}

} // extern "C"
