// Argument block and launchers of the time-correlation kernels (tcf.hip).
#pragma once
#include "kernels.hpp"

struct TcfArgs {
    KArena A;
    const uint4 *snap; // the replica's current snapshot (species bits)
    int off, n;        // arena slots of the replica
    int block;         // entries per level (l)
    int pad;
    double L, q;
    double4 *pos;      // [levels * l][n] unwrapped positions, by particle id
    double4 *vel;      // [levels * l][n] velocities, by particle id
    int *species;      // [n]
    double *partial;   // [blocks][l - 1][8] per-workgroup sums of one pass
    double *acc;       // [levels][l - 1][2][3] sums of per-pass species means
};

hipError_t launch_tcf_store(int prec, const TcfArgs &a, int entry, hipStream_t s);
hipError_t launch_tcf_correlate(const TcfArgs &a, int level, int head, hipStream_t s);
int tcf_blocks(int n);
