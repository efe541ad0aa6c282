// Observables, velocity scaling, the double-single self-test and stream-
// ordered control writes, with their launchers.
#include <mutex>

#include "dev_common.hpp"

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

// ------------------------------------------------------------ thermostat
// rand48 (Sec. 2.3): x_{k+1} = (a x_k + c) mod 2^48.  Element j from x0 is
// A_j x0 + C_j, the j-fold composition of the affine map, by repeated
// squaring; particle id i at call k takes elements i + n (4k + r), r = 0..3
// (the leap-frog of stride n over the particles), so no generator state is
// stored and the draws do not depend on slot order or launch shape.
#define R48_A 0x5DEECE66DULL
#define R48_C 0xBULL
#define R48_M ((1ULL << 48) - 1ULL)

__device__ __forceinline__ unsigned long long r48_element(unsigned long long x0, unsigned long long j)
{
    unsigned long long A = 1, C = 0, a = R48_A, c = R48_C;
    while (j) {
        if (j & 1) { A = (a * A) & R48_M; C = (a * C + c) & R48_M; }
        c = (a * c + c) & R48_M;
        a = (a * a) & R48_M;
        j >>= 1;
    }
    return (A * x0 + C) & R48_M;
}

#define TH_CHUNK 4096

// The Maxwell-Boltzmann velocity of particle id at this call (Box-Muller on
// four leap-frogged rand48 elements); a pure function of (seed, call, id).
__device__ __noinline__ void thermo_velocity(const ThermoArgs &a, int id, double v[3])
{
    const unsigned long long base = (unsigned long long)id + (unsigned long long)a.n * (4ULL * a.call);
    double u[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        u[r] = (double)r48_element(a.x0, base + (unsigned long long)a.n * r) * (1.0 / 281474976710656.0);
    const double ra = sqrt(-2.0 * log(1.0 - u[0])), rb = sqrt(-2.0 * log(1.0 - u[2]));
    const double ph = 6.283185307179586 * u[1], ph2 = 6.283185307179586 * u[3];
    v[0] = a.scale * ra * cos(ph);
    v[1] = a.scale * ra * sin(ph);
    v[2] = a.scale * rb * cos(ph2);
}

// Draw Maxwell-Boltzmann velocities into the scratch rows (when a.obs is
// set; the allocation-free form draws them again when it applies them) and
// reduce sum(v) and sum(v^2) per chunk of TH_CHUNK particles into
// a.partial[(chunk0 + c) * 8 + q].
__global__ void __launch_bounds__(256) k_thermo_draw(const ThermoArgs a)
{
    __shared__ double red[4][256];
    const int c = blockIdx.x;
    const int k0 = c * TH_CHUNK, k1 = min(k0 + TH_CHUNK, a.n);
    double acc[4] = {0, 0, 0, 0};
    for (int k = k0 + threadIdx.x; k < k1; k += blockDim.x) {
        const int i = a.off + k;
        const int id = a.A.meta[i].w;
        if (id < 0 || id >= a.n) continue;
        double v[3];
        thermo_velocity(a, id, v);
        if (a.obs) {
            double *o = a.obs + (size_t)i * 8;
            o[0] = v[0]; o[1] = v[1]; o[2] = v[2];
        }
        acc[0] += v[0]; acc[1] += v[1]; acc[2] += v[2];
        acc[3] += v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    }
    for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int w = blockDim.x >> 1; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) a.partial[(size_t)(a.chunk0 + c) * 8 + threadIdx.x] = red[threadIdx.x][0];
}

// Subtract the mean (optional), scale to exactly the bath temperature and
// store the velocities in the mode's precision.  Every workgroup adds the
// chunk partials in the same order, so all use the same factor.
template <int P>
__global__ void __launch_bounds__(256) k_thermo_apply(const ThermoArgs a)
{
    __shared__ double tot[4];
    if (threadIdx.x < 4) {
        double t = 0;
        for (int c = 0; c < a.nchunk; ++c) t += a.partial[(size_t)(a.chunk0 + c) * 8 + threadIdx.x];
        tot[threadIdx.x] = t;
    }
    __syncthreads();
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const double n = (double)a.n;
    double mean[3] = {0, 0, 0};
    if (a.remove_mean)
        for (int d = 0; d < 3; ++d) mean[d] = tot[d] / n;
    const double ss = tot[3] - n * (mean[0] * mean[0] + mean[1] * mean[1] + mean[2] * mean[2]);
    const double f = sqrt(a.temperature / (a.mass * ss / (3.0 * n)));
    const int i = a.off + k;
    double w[3];
    if (a.obs) {
        const double *o = a.obs + (size_t)i * 8;
        w[0] = o[0]; w[1] = o[1]; w[2] = o[2];
    } else { // allocation-free form: the same draw again (a pure function of the id)
        const int id = a.A.meta[i].w;
        if (id < 0 || id >= a.n) return;
        thermo_velocity(a, id, w);
    }
    const double v[3] = {(w[0] - mean[0]) * f, (w[1] - mean[1]) * f, (w[2] - mean[2]) * f};
    State<P> st;
    st.load(a.A, i);
    if constexpr (P == PREC_FP32) {
        st.vx = (float)v[0]; st.vy = (float)v[1]; st.vz = (float)v[2];
    } else if constexpr (P == PREC_DS) {
        dsf *w[3] = {&st.vx, &st.vy, &st.vz};
        for (int d = 0; d < 3; ++d) {
            w[d]->hi = (float)v[d];
            w[d]->lo = (float)(v[d] - (double)w[d]->hi);
        }
    } else {
        st.vx = v[0]; st.vy = v[1]; st.vz = v[2];
    }
    st.store(a.A, i);
}

hipError_t launch_thermostat(int prec, const ThermoArgs &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_thermo_draw, dim3(a.nchunk), dim3(256), 0, s, a);
    const int grid = (a.n + 255) / 256;
    switch (prec) {
    case PREC_FP32: hipLaunchKernelGGL((k_thermo_apply<PREC_FP32>), dim3(grid), dim3(256), 0, s, a); break;
    case PREC_DS: hipLaunchKernelGGL((k_thermo_apply<PREC_DS>), dim3(grid), dim3(256), 0, s, a); break;
    case PREC_MIX: hipLaunchKernelGGL((k_thermo_apply<PREC_MIX>), dim3(grid), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((k_thermo_apply<PREC_FP64>), dim3(grid), dim3(256), 0, s, a); break;
    }
    LAUNCH_CHECK();
}

// ------------------------------------------- allocation-free thermostat
// For callers that cannot allocate device memory (code under graph capture,
// tight serving loops): the chunk partial sums of md_thermostat_noalloc live
// in this file-scope device array instead of the pool's workspace, and the
// drawn velocities are not stored at all (they are drawn again when
// applied).  Each GPU holds its own copy; host code must use the address
// hipGetSymbolAddress returns for the current device, never the array's
// name.  Every chunk row a call reads was written by the same call, so
// nothing needs clearing; calls that overlap on one GPU race on it.
static __device__ __align__(256) double scratch[THERMO_SCRATCH_CHUNKS * 8];

#define THERMO_MAX_DEVICES 64
static double *scratch_ptr[THERMO_MAX_DEVICES];
static std::mutex scratch_mutex;

hipError_t thermo_scratch_init(int dev)
{
    if (dev < 0 || dev >= THERMO_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (scratch_ptr[dev]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev) return hipErrorInvalidDevice; // must be called with that device current
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[dev] = (double *)p;
    return hipSuccess;
}

double *thermo_scratch(int dev)
{
    if (dev < 0 || dev >= THERMO_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    return scratch_ptr[dev];
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

// Forget the forces a finalising launch stored (control word w) for every slot.
__global__ void k_void_stored(Ctl *ctl, int max_slots)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < max_slots) ctl[s].w = 0;
}

hipError_t launch_add_targets(int *target, const Ctl *ctl, int max_slots, int delta, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_targets, dim3((max_slots + 255) / 256), dim3(256), 0, s, target, ctl, max_slots, delta);
    LAUNCH_CHECK();
}

hipError_t launch_void_stored(Ctl *ctl, int max_slots, hipStream_t s)
{
    hipLaunchKernelGGL(k_void_stored, dim3((max_slots + 255) / 256), dim3(256), 0, s, ctl, max_slots);
    LAUNCH_CHECK();
}

hipError_t launch_poke(int *p, int v, hipStream_t s)
{
    hipLaunchKernelGGL(k_poke, dim3(1), dim3(1), 0, s, p, v);
    LAUNCH_CHECK();
}
