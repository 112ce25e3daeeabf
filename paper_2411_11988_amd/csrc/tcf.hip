// Ring-polymer molecular dynamics (RPMD) velocity correlation functions
// (arXiv 2411.11988, Sec. "Output and Analysis": real-time correlation functions
// from NVE ring-polymer trajectories; Kubo-transformed correlations of
// linear operators are estimated from the centroids).
//
// One sample at time t: the centroid velocity of every particle,
// v_i = (1/N_i) sum_j p_ij / m_f,i, goes into slot t mod L of a caller-owned
// ring of the last L samples; then for every lag tau < min(t + 1, L) and
// every system, sum_i v_i(t - tau) . v_i(t) is added to the accumulator of
// the particle's species.  One workgroup owns each (system, lag) entry, so
// the accumulation is deterministic and needs no atomics.
#include "device_common.h"
#include "mixpi_internal.h"

namespace mixpi {

namespace {

constexpr int kTcfThreads = 256;

__device__ __forceinline__ double wave_sum_d(double v) { return wsum(v); }

// one wave per particle: lanes stride over its beads
__global__ __launch_bounds__(kTcfThreads) void k_centroid_v(const PartDev *parts, int n_part,
                                                           const double *p, double *out)
{
    const int i = blockIdx.x * (kTcfThreads / 64) + ((int)threadIdx.x >> 6);
    if (i >= n_part) return;
    const int lane = threadIdx.x & 63;
    const PartDev pd = parts[i];
    double sx = 0, sy = 0, sz = 0;
    for (int j = lane; j < pd.nb; j += 64) {
        const long long r = pd.row0 + (long long)j * pd.stride;
        sx += p[3 * r];
        sy += p[3 * r + 1];
        sz += p[3 * r + 2];
    }
    sx = wave_sum_d(sx);
    sy = wave_sum_d(sy);
    sz = wave_sum_d(sz);
    if (lane == 0) {
        out[3LL * i] = sx * pd.inv_nm;
        out[3LL * i + 1] = sy * pd.inv_nm;
        out[3LL * i + 2] = sz * pd.inv_nm;
    }
}

// workgroup (lag, system): per-species sums over the system's particles
__global__ __launch_bounds__(kTcfThreads) void k_vacf(TcfLaunch a)
{
    const int tau = blockIdx.x % a.n_lag;
    const int s = blockIdx.x / a.n_lag;
    const double *cur = a.ring + 3LL * a.n_part * a.slot;
    const int prev_slot = (int)((a.t - tau) % a.L);
    const double *prv = a.ring + 3LL * a.n_part * prev_slot;
    double part[kMaxLjTypes + 1];
#pragma unroll
    for (int k = 0; k <= kMaxLjTypes; ++k) part[k] = 0.0;
    for (int i = a.sys_part[s] + threadIdx.x; i < a.sys_part[s + 1]; i += kTcfThreads) {
        const double d = prv[3LL * i] * cur[3LL * i] + prv[3LL * i + 1] * cur[3LL * i + 1] +
                         prv[3LL * i + 2] * cur[3LL * i + 2];
        const int sp = a.parts[i].spec;
#pragma unroll
        for (int k = 0; k <= kMaxLjTypes; ++k) part[k] += sp == k ? d : 0.0;
    }
    __shared__ double red[kTcfThreads / 64][kMaxLjTypes + 1];
    const int lane = threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k <= kMaxLjTypes; ++k) {
        const double v = wave_sum_d(part[k]);
        if (lane == 0) red[wv][k] = v;
    }
    __syncthreads();
    const int nt1 = a.sys[s].nt1;
    if ((int)threadIdx.x < nt1) {
        const int k = threadIdx.x;
        double v = 0.0;
        for (int w = 0; w < kTcfThreads / 64; ++w) v += red[w][k];
        a.acc[((long long)s * a.nspec + k) * a.L + tau] += v;
    }
}

}  // namespace

void launch_tcf(const TcfLaunch &a, const double *p, hipStream_t st)
{
    if (a.n_part <= 0) return;
    double *slot = a.ring + 3LL * a.n_part * a.slot;
    const int per = kTcfThreads / 64;
    hipLaunchKernelGGL(k_centroid_v, dim3((a.n_part + per - 1) / per), dim3(kTcfThreads), 0, st,
                       a.parts, a.n_part, p, slot);
    hipLaunchKernelGGL(k_vacf, dim3(a.n_lag * a.n_sys), dim3(kTcfThreads), 0, st, a);
}

}  // namespace mixpi
