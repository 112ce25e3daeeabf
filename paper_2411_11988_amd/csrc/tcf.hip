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
    // beads lane, lane + 64, ... added in that order; the loads of U beads
    // are in flight together
    constexpr int U = 8;
    for (int j0 = lane; j0 < pd.nb; j0 += 64 * U) {
        double v[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = j0 + 64 * u;
            const long long r = pd.row0 + (long long)(j < pd.nb ? j : 0) * pd.stride;
            v[u][0] = p[3 * r];
            v[u][1] = p[3 * r + 1];
            v[u][2] = p[3 * r + 2];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j0 + 64 * u < pd.nb) {
                sx += v[u][0];
                sy += v[u][1];
                sz += v[u][2];
            }
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
    // particles i, i + 256, ... of the system in that order; the loads of U
    // particles are in flight together
    constexpr int U = 8;
    const int i1 = a.sys_part[s + 1];
    for (int i0 = a.sys_part[s] + threadIdx.x; i0 < i1; i0 += kTcfThreads * U) {
        double pv[U][3], cv[U][3];
        int spv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + kTcfThreads * u < i1 ? i0 + kTcfThreads * u : i0;
            for (int c = 0; c < 3; ++c) {
                pv[u][c] = prv[3LL * i + c];
                cv[u][c] = cur[3LL * i + c];
            }
            spv[u] = a.spec[i];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (i0 + kTcfThreads * u >= i1) break;
            const double d = pv[u][0] * cv[u][0] + pv[u][1] * cv[u][1] + pv[u][2] * cv[u][2];
#pragma unroll
            for (int k = 0; k <= kMaxLjTypes; ++k) part[k] += spv[u] == k ? d : 0.0;
        }
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
