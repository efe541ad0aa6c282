// Kernel argument blocks and launchers of libmdx (shared by the .hip kernel
// sources and abi.cpp).  Plain structs passed by value as kernel arguments.
#pragma once
#include <hip/hip_runtime.h>
#include "md_dev.hpp"

struct KArena {
    int P;            // arena stride (particle slots)
    int cap;          // neighbour-list capacity per particle (a multiple of 16)
    int lg;           // log2 of the lanes per particle that read a list (entry layout)
    uint4 *st[3];     // state words
    const uint4 *xref;
    uint4 *xref_w;    // same memory as xref
    int4 *meta;
    const int *nbr;
    int *nbr_w;       // same memory as nbr
    const int *nbr_cnt;
    int *nbr_cnt_w;   // same memory as nbr_cnt
};

struct StepArgs {
    KArena A;
    int cell_cap, max_slots, xcd, lpp; // lpp: lanes per particle (1, 2, 4)
    const uint4 *snap_cur;
    uint4 *snap_next;
    const RepDev *rep;
    const Ctl *ctl_cur;
    Ctl *ctl_next;
    const int *target;
    int *need_cur, *need_other;
    int *rlist_cur, *rlist_other; // [0] = count, [1..] = slots that must rebuild
    int *count_cur, *count_other;
    const int *corder; // per-replica cell rank tables (cell arena offsets)
    int *status;
    double *obs;
    PairDev pp;
    IntegDev ig;
};

struct CountArgs {
    int P, max_slots, force_slot, pad0;
    const uint4 *snap;
    const RepDev *rep;
    const Ctl *ctl;
    int *count;
    const int *corder;
};

struct ScanArgs {
    int max_slots, force_slot;
    const RepDev *rep;
    const int *need;
    const int *rlist;
    const Ctl *ctl;
    const int *count;
    int *cs_new;
    int *status;
    int *nreb;
};

struct PermArgs {
    KArena A;
    int max_slots, force_slot;
    const int *items_pref;
    const RepDev *rep;
    const int *need;
    const int *rlist;
    const Ctl *ctl;
    const int *cs, *cs_new;
    const int *corder;
    const uint4 *snap;
    uint4 *sc_st[3];
    uint4 *sc_snap;
    int4 *sc_meta;
    int *status;
};

struct BuildArgs {
    KArena A;
    int max_slots, force_slot, from_scratch, width, lds_cap, xcd;
    int single_members; // members per work item of a single-cell replica
    int bulk;           // rebuilding replicas from which a step's build is a bulk build; 0 = never
    const int *items_pref;
    const RepDev *rep;
    const int *need;
    const int *rlist;
    const Ctl *ctl;
    int *cs;
    const int *cs_new;
    const int *corder;
    const uint4 *src_x;
    uint4 *snap_cur;
    const uint4 *sc_st[3];
    const int4 *sc_meta;
    int *status;
    PairDev pp;
};

struct ObsArgs {
    int max_slots, pad0;
    const RepDev *rep;
    const Ctl *ctl;
    const double *obs;
    const int *nbr_cnt;
    const int *chunk_pref; // per slot prefix of ceil(n / 4096) chunks
    double *partial;       // [chunks][8]
    double *out;           // [max_slots][8]
};

struct ScaleArgs {
    KArena A;
    int off, n;
    float f_hi, f_lo, ff, pad0;
    double fd;
};

// Modified Andersen thermostat (Sec. 2.3): rand48 draws, leap-frogged with
// stride n over the replica's particles.
struct ThermoArgs {
    KArena A;
    double *obs;      // per-slot scratch rows (8 doubles); velocities drawn here
                      // (nullptr: drawn again when applied, nothing stored)
    double *partial;  // chunk partial sums (8 doubles per chunk)
    int off, n, chunk0, nchunk, remove_mean, pad0;
    unsigned long long x0; // rand48 state of the seed (stream element 0)
    long long call;        // thermostat call index
    double scale;          // sqrt(T / m)
    double temperature, mass;
};

hipError_t launch_thermostat(int prec, const ThermoArgs &a, hipStream_t s);
// Chunk rows of the allocation-free thermostat's scratch array (aux_kernels.hip):
// at most THERMO_SCRATCH_CHUNKS chunks of 4096 particles per call.
#define THERMO_SCRATCH_CHUNKS 16384
hipError_t thermo_scratch_init(int dev); // once per device, with that device current
double *thermo_scratch(int dev);         // its device address (nullptr before init)
hipError_t launch_step(int prec, const StepArgs &a, int block, bool obs, hipStream_t s);
hipError_t launch_count(int prec, const CountArgs &a, hipStream_t s);
hipError_t launch_scan(const ScanArgs &a, hipStream_t s);
hipError_t launch_permute(int prec, const PermArgs &a, int grid, hipStream_t s);
hipError_t launch_build(int prec, const BuildArgs &a, int grid, int block, hipStream_t s);
hipError_t occupancy_permute(int prec, int *per_cu);
hipError_t occupancy_build(int prec, int block, int lds_cap, int *per_cu);
hipError_t launch_obs_reduce(const ObsArgs &a, hipStream_t s);
hipError_t launch_scale_vel(int prec, const ScaleArgs &a, hipStream_t s);
hipError_t launch_ds_eval(int op, long long n, const float *a, const float *b, float *out, hipStream_t s);
