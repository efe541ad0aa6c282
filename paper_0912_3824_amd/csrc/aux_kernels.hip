// Observables, velocity scaling, the double-single self-test and stream-
// ordered control writes, with their launchers.
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
