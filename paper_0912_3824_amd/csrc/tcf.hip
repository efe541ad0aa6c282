// Time-correlation functions by the blocking scheme of Sec. 2.5, on device.
//
// A scheme of k levels of l entries is bound to one replica.  Entry storage
// is by particle id (the sort permutes slots between samples): unwrapped
// positions (state position + image counter x L) and velocities, in FP64.
// Sample m enters every level n with l^n | m; a level holding l entries
// correlates its oldest entry with the l - 1 others (lags j l^n samples) and
// drops it.  Per correlation pass and lag, each workgroup reduces its
// particles' MSD, VACF and F_s terms per species into a partial row; a
// second kernel adds the partial rows in a fixed order, divides by the
// species counts and accumulates the per-pass means (deterministic).
#include "dev_common.hpp"
#include "tcf.hpp"

#define TCF_BLOCK 256

// unwrapped position and velocity of arena slot i, in double
template <int P>
__device__ __forceinline__ void tcf_state(const TcfArgs &a, int i, double r[3], double v[3])
{
    const KArena &A = a.A;
    const int4 m = A.meta[i];
    const double L = a.L;
    if constexpr (P == PREC_FP32) {
        const float4 p = ((const float4 *)A.st[0])[i], w = ((const float4 *)A.st[1])[i];
        r[0] = (double)p.x + m.x * L; r[1] = (double)p.y + m.y * L; r[2] = (double)p.z + m.z * L;
        v[0] = w.x; v[1] = w.y; v[2] = w.z;
    } else if constexpr (P == PREC_DS) {
        const float4 p = ((const float4 *)A.st[0])[i], q = ((const float4 *)A.st[1])[i],
                     c = ((const float4 *)A.st[2])[i];
        r[0] = ((double)p.x + (double)p.w) + m.x * L;
        r[1] = ((double)p.y + (double)q.x) + m.y * L;
        r[2] = ((double)p.z + (double)q.y) + m.z * L;
        v[0] = (double)q.z + (double)c.y;
        v[1] = (double)q.w + (double)c.z;
        v[2] = (double)c.x + (double)c.w;
    } else {
        const double2 p = ((const double2 *)A.st[0])[i], q = ((const double2 *)A.st[1])[i],
                      c = ((const double2 *)A.st[2])[i];
        r[0] = p.x + m.x * L; r[1] = p.y + m.y * L; r[2] = q.x + m.z * L;
        v[0] = q.y; v[1] = c.x; v[2] = c.y;
    }
}

// Store the replica's current state as entry `entry` (level * l + ring slot).
template <int P>
__global__ void __launch_bounds__(TCF_BLOCK) k_tcf_store(const TcfArgs a, int entry)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const int i = a.off + k;
    double r[3], v[3];
    tcf_state<P>(a, i, r, v);
    const int id = a.A.meta[i].w;
    if (id < 0 || id >= a.n) return; // not a particle of this replica
    uint32_t meta;
    if (Traits<P>::NS == 2) {
        double zz, ww;
        u4_to_dbl2(a.snap[(size_t)a.A.P + i], zz, ww);
        meta = meta_of_bits(ww);
    } else meta = a.snap[i].w;
    const size_t e = (size_t)entry * a.n + id;
    a.pos[e] = make_double4(r[0], r[1], r[2], 0.0);
    a.vel[e] = make_double4(v[0], v[1], v[2], 0.0);
    a.species[id] = species_of(meta);
}

__device__ __forceinline__ double tcf_wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// One correlation pass: origin entry `head` against entries head+1 .. head+l-1
// (mod l) of level `level`.  partial[block][j][species][4] = sums of MSD,
// VACF, F_s and the particle count over this workgroup's particles.
__global__ void __launch_bounds__(TCF_BLOCK) k_tcf_corr(const TcfArgs a, int level, int head)
{
    __shared__ double red[TCF_BLOCK / 64][8];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int id = blockIdx.x * blockDim.x + t;
    const int l = a.block;
    const bool live = id < a.n;
    const size_t base = (size_t)level * l;
    double4 p0 = make_double4(0, 0, 0, 0);
    double4 v0 = make_double4(0, 0, 0, 0);
    int sp = 0;
    if (live) {
        p0 = a.pos[(base + head) * a.n + id];
        v0 = a.vel[(base + head) * a.n + id];
        sp = a.species[id];
    }
    for (int j = 1; j < l; ++j) {
        int e = head + j;
        e -= e >= l ? l : 0;
        double msd = 0, vacf = 0, fs = 0;
        if (live) {
            const double4 p = a.pos[(base + e) * a.n + id];
            const double4 v = a.vel[(base + e) * a.n + id];
            const double dx = p.x - p0.x, dy = p.y - p0.y, dz = p.z - p0.z;
            msd = dx * dx + dy * dy + dz * dz;
            vacf = v.x * v0.x + v.y * v0.y + v.z * v0.z;
            fs = (cos(a.q * dx) + cos(a.q * dy) + cos(a.q * dz)) / 3.0;
        }
        // species-split sums: (msd, vacf, fs, count) for A then B
        double s[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) s[c] = 0.0;
        const int o = sp ? 4 : 0;
        if (live) {
            s[o] = msd; s[o + 1] = vacf; s[o + 2] = fs; s[o + 3] = 1.0;
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) s[c] = tcf_wave_sum(s[c]);
        if (lane == 0)
#pragma unroll
            for (int c = 0; c < 8; ++c) red[wv][c] = s[c];
        __syncthreads();
        if (t < 8) {
            double acc = 0;
            for (int w = 0; w < TCF_BLOCK / 64; ++w) acc += red[w][t];
            a.partial[((size_t)blockIdx.x * (l - 1) + (j - 1)) * 8 + t] = acc;
        }
        __syncthreads();
    }
}

// Add the partial rows of one pass (one workgroup per lag and species: each
// thread sums a fixed stride of rows, then a fixed tree), and accumulate the
// per-pass species means into acc[level][j][species][3].
__global__ void __launch_bounds__(TCF_BLOCK) k_tcf_reduce(const TcfArgs a, int level, int nblk)
{
    __shared__ double red[4][TCF_BLOCK];
    const int t = threadIdx.x;
    const int l = a.block;
    const int j = blockIdx.x >> 1, s = blockIdx.x & 1;
    double sum[4] = {0, 0, 0, 0};
    for (int b = t; b < nblk; b += TCF_BLOCK)
#pragma unroll
        for (int c = 0; c < 4; ++c) sum[c] += a.partial[((size_t)b * (l - 1) + j) * 8 + s * 4 + c];
#pragma unroll
    for (int c = 0; c < 4; ++c) red[c][t] = sum[c];
    __syncthreads();
    for (int w = TCF_BLOCK >> 1; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int c = 0; c < 4; ++c) red[c][t] += red[c][t + w];
        __syncthreads();
    }
    if (t == 0 && red[3][0] > 0) {
        double *acc = a.acc + (((size_t)level * (l - 1) + j) * 2 + s) * 3;
        for (int c = 0; c < 3; ++c) acc[c] += red[c][0] / red[3][0];
    }
}

hipError_t launch_tcf_store(int prec, const TcfArgs &a, int entry, hipStream_t s)
{
    const int grid = (a.n + TCF_BLOCK - 1) / TCF_BLOCK;
    switch (prec) {
    case PREC_FP32: hipLaunchKernelGGL((k_tcf_store<PREC_FP32>), dim3(grid), dim3(TCF_BLOCK), 0, s, a, entry); break;
    case PREC_DS: hipLaunchKernelGGL((k_tcf_store<PREC_DS>), dim3(grid), dim3(TCF_BLOCK), 0, s, a, entry); break;
    case PREC_MIX: hipLaunchKernelGGL((k_tcf_store<PREC_MIX>), dim3(grid), dim3(TCF_BLOCK), 0, s, a, entry); break;
    default: hipLaunchKernelGGL((k_tcf_store<PREC_FP64>), dim3(grid), dim3(TCF_BLOCK), 0, s, a, entry); break;
    }
    LAUNCH_CHECK();
}

int tcf_blocks(int n) { return (n + TCF_BLOCK - 1) / TCF_BLOCK; }

hipError_t launch_tcf_correlate(const TcfArgs &a, int level, int head, hipStream_t s)
{
    const int grid = tcf_blocks(a.n);
    hipLaunchKernelGGL(k_tcf_corr, dim3(grid), dim3(TCF_BLOCK), 0, s, a, level, head);
    hipLaunchKernelGGL(k_tcf_reduce, dim3(2 * (a.block - 1)), dim3(TCF_BLOCK), 0, s, a, level, grid);
    LAUNCH_CHECK();
}
