// Device helpers shared by the kernels: wave/workgroup sums, the bonded
// sweep of one workgroup and the energy reducer.
#pragma once

#include "mixpi.h"
#include "mixpi_internal.h"

namespace mixpi {

// Wave sums by DPP lane moves (VALU operations, no trip through the LDS
// unit as a shuffle takes).  dpp_d: lane i receives v from the lane that
// the DPP control CTRL selects within its row of 16; lanes of rows outside
// ROW_MASK receive 0.  The order of the additions is fixed, so the sums are
// reproducible bit for bit.  Callers run them with every lane of the rows
// involved active.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_d(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int l)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}

// Sum over each row of 16 lanes, in every lane of the row.
__device__ __forceinline__ double row16_sum(double v)
{
    v += dpp_d<0xB1, 0xF>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E, 0xF>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x124, 0xF>(v);   // row_ror:4
    v += dpp_d<0x128, 0xF>(v);   // row_ror:8
    return v;
}

// Sum over aligned groups of G lanes (16, 32 or 64), in every lane of the
// group.
template <int G>
__device__ __forceinline__ double group_sum(double v)
{
    v = row16_sum(v);
    if constexpr (G == 16) return v;
    v += dpp_d<0x142, 0xA>(v);   // row_bcast:15: rows 1 and 3 hold rows 0+1 and 2+3
    if constexpr (G == 32) {
        const double s0 = readlane_d(v, 31), s1 = readlane_d(v, 63);
        return (threadIdx.x & 32) ? s1 : s0;
    }
    v += dpp_d<0x143, 0xC>(v);   // row_bcast:31: row 3 holds the wave's sum
    return readlane_d(v, 63);
}

// Sum over the wave, in every lane.
__device__ __forceinline__ double wsum(double v) { return group_sum<64>(v); }

// Largest v over the wave, in every lane (the steps of group_sum<64> with
// max; rows that a broadcast step leaves out receive 0 there, but their
// values do not reach lane 63, whose result every lane reads).
__device__ __forceinline__ double wmax(double v)
{
    v = fmax(v, dpp_d<0xB1, 0xF>(v));
    v = fmax(v, dpp_d<0x4E, 0xF>(v));
    v = fmax(v, dpp_d<0x124, 0xF>(v));
    v = fmax(v, dpp_d<0x128, 0xF>(v));
    v = fmax(v, dpp_d<0x142, 0xA>(v));
    v = fmax(v, dpp_d<0x143, 0xC>(v));
    return readlane_d(v, 63);
}

// A value equal in every lane, moved to scalar registers (the first active
// lane's copy): frees vector registers and lets address arithmetic on it
// run in scalar instructions.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uni(long long v)
{
    const unsigned long long u = (unsigned long long)v;
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ double uni(double v)
{
    return __longlong_as_double(uni(__double_as_longlong(v)));
}

// The wave's lane mask of b (bit l: lane l is active and has b set), a
// wave-uniform value.  A mask of one compare is that compare's own result,
// and masks combine with scalar instructions.
__device__ __forceinline__ unsigned long long lanes(bool b)
{
    return __builtin_amdgcn_ballot_w64(b);
}

// Sum of v over the workgroup (blockDim.x a multiple of 64), valid in
// thread 0.  red: LDS scratch of blockDim.x / 64 doubles.
__device__ __forceinline__ double bsum(double v, double *red)
{
    v = wsum(v);
    if (blockDim.x == 64) return v;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    return s;
}

__device__ __forceinline__ void min_img(double &x, double L, double iL) { x -= L * rint(x * iL); }

// Bonds and angles of V_mix (Eq. mts-hamiltonian, 2- and 3-body terms) for
// the terms of one workgroup (a system-pure range of at most blockDim.x
// terms): one thread per (term, slice); the slice's beads were resolved on
// the host, so a thread sees plain bead rows and the weight 1/N_max.  FP64
// throughout: bonded terms are stiff and cheap.  Forces go to the term's own
// partial-force slots, stored at their row-contiguous positions (summed later
// by the per-row gather); the energy sums go to the workgroup's slot `e`.
template <bool THETA>
__device__ void bonded_block(const BondedLaunch &a, const BlockRange &br, double *e, double *red)
{
    const SysDev &S = a.sys[br.sys];
    const double *th = a.theta ? a.theta + 6 * br.sys : S.theta0;
    const int t = br.begin + threadIdx.x;
    double eb = 0, ea = 0, gb = 0, ga = 0;
    if ((int)threadIdx.x < br.count) {
        const BondedTerm bt = a.terms[t];
        const int *dst = a.dest + a.part_base + 3LL * t;
        if (bt.kind == 0) {
            const bool t0 = bt.type == S.bond_off;
            const double k = t0 ? th[4] : a.bond_k[bt.type];
            const double r0 = a.bond_r0[bt.type];
            double d[3];
            for (int c = 0; c < 3; ++c) {
                d[c] = a.q[3LL * bt.r[0] + c] - a.q[3LL * bt.r[1] + c];
                min_img(d[c], S.box[c], S.ibox[c]);
            }
            const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const double dr = r - r0;
            eb = bt.w * 0.5 * k * dr * dr;
            if (THETA && t0) gb = bt.w * 0.5 * dr * dr;
            const double g = -bt.w * k * dr / r;
            double *o0 = a.part + 3LL * dst[0], *o1 = a.part + 3LL * dst[1];
            for (int c = 0; c < 3; ++c) {
                o0[c] = g * d[c];
                o1[c] = -g * d[c];
            }
        } else {
            const bool t0 = bt.type == S.angle_off;
            const double k = t0 ? th[5] : a.angle_k[bt.type];
            const double th0 = a.angle_t0[bt.type];
            double r1[3], r2[3];
            for (int c = 0; c < 3; ++c) {
                r1[c] = a.q[3LL * bt.r[0] + c] - a.q[3LL * bt.r[1] + c];
                r2[c] = a.q[3LL * bt.r[2] + c] - a.q[3LL * bt.r[1] + c];
                min_img(r1[c], S.box[c], S.ibox[c]);
                min_img(r2[c], S.box[c], S.ibox[c]);
            }
            const double l1 = sqrt(r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
            const double l2 = sqrt(r2[0] * r2[0] + r2[1] * r2[1] + r2[2] * r2[2]);
            double c = (r1[0] * r2[0] + r1[1] * r2[1] + r1[2] * r2[2]) / (l1 * l2);
            c = fmin(1.0, fmax(-1.0, c));
            const double dth = acos(c) - th0;
            ea = bt.w * 0.5 * k * dth * dth;
            if (THETA && t0) ga = bt.w * 0.5 * dth * dth;
            const double s = sqrt(1.0 - c * c);
            const double pref = bt.w * k * dth / s;
            const double i12 = 1.0 / (l1 * l2), i11 = 1.0 / (l1 * l1), i22 = 1.0 / (l2 * l2);
            double *o0 = a.part + 3LL * dst[0], *o1 = a.part + 3LL * dst[1];
            double *o2 = a.part + 3LL * dst[2];
            for (int x = 0; x < 3; ++x) {
                const double fa = pref * (r2[x] * i12 - c * r1[x] * i11);
                const double fb = pref * (r1[x] * i12 - c * r2[x] * i22);
                o0[x] = fa;                // end a
                o1[x] = -(fa + fb);        // vertex
                o2[x] = fb;                // end b
            }
        }
    }
    eb = bsum(eb, red);
    ea = bsum(ea, red);
    if (THETA) {
        gb = bsum(gb, red);
        ga = bsum(ga, red);
    }
    if (threadIdx.x == 0) {
        for (int k = 0; k < A_N; ++k) e[k] = 0.0;
        e[A_BOND] = eb;
        e[A_ANGLE] = ea;
        e[A_TH4] = gb;
        e[A_TH5] = ga;
    }
}

// Energies of system s from its summed slot row r: writes the requested
// outputs and adds its pair-evaluation counts (exact integers in FP64).
__device__ inline void energy_outputs(const ReduceB &a, int s, const double *r)
{
    const SysDev &S = a.sys[s];
    double e[MIXPI_NE];
    e[MIXPI_E_LJ] = r[A_LJ];
    e[MIXPI_E_COUL] = r[A_COUL] + S.bg_energy;
    e[MIXPI_E_PP] = r[A_PP];
    e[MIXPI_E_BOND] = r[A_BOND];
    e[MIXPI_E_ANGLE] = r[A_ANGLE];
    e[MIXPI_E_VMIX] = e[1] + e[2] + e[3] + e[4] + e[5];
    e[MIXPI_E_SPRING] = r[A_SPRING];
    e[MIXPI_E_KIN] = r[A_KIN] / kKcal;
    e[MIXPI_E_KCV] = S.cv_const - 0.5 * r[A_VIR];
    e[MIXPI_E_KPRIM] = S.prim_const - r[A_SPRING];
    e[MIXPI_E_HAM] = e[MIXPI_E_KIN] + e[MIXPI_E_SPRING] + e[MIXPI_E_VMIX];
    if (a.e_out)
        for (int k = 0; k < MIXPI_NV; ++k) a.e_out[(long long)s * MIXPI_NV + k] = e[k];
    if (a.elog) {
        for (int k = 0; k < MIXPI_NE; ++k) a.elog[(long long)s * MIXPI_NE + k] = e[k];
        if (a.nonfinite && !isfinite(e[MIXPI_E_HAM])) atomicOr(a.nonfinite, 1);
    }
    if (a.dtheta) {
        const double g = a.grad_e ? a.grad_e[s] : 1.0;
        for (int k = 0; k < 6; ++k) a.dtheta[(long long)s * 6 + k] = g * r[A_TH0 + k];
    }
    if (a.npairs) {
        if (r[A_CNT_AA] > 0.0) atomicAdd(&a.npairs[0], (unsigned long long)r[A_CNT_AA]);
        if (r[A_CNT_EA] > 0.0) atomicAdd(&a.npairs[1], (unsigned long long)r[A_CNT_EA]);
    }
}

// Stage A, one workgroup (kReduceThreads threads) per chunk: thread t sums
// component t % A_N of the chunk's slots (A_N divides the block size), the
// A_N-strided partials are added in LDS.  lds: >= kReduceThreads doubles.
__device__ inline void reduce_a_part(const ReduceA &a, int c, double *lds)
{
    const int t = threadIdx.x;
    const double *base = a.eslot + (long long)a.chunk_begin[c] * A_N;
    const int n = a.chunk_len[c] * A_N;
    double acc = 0.0;
#pragma unroll 4
    for (int k = t; k < n; k += kReduceThreads) acc += base[k];
    lds[t] = acc;
    __syncthreads();
    if (t < A_N) {
        double v = 0.0;
        for (int x = t; x < kReduceThreads; x += A_N) v += lds[x];
        a.partial[(long long)c * A_N + t] = v;
    }
}

// Stage B, one workgroup (kReduceThreads threads) per system s: thread t
// adds component t % A_N over the chunks g, g + G, ... of the system
// (g = t / A_N, G = kReduceThreads / A_N), the G partials per component are
// added in LDS in order, and thread 0 writes the outputs.
// lds: >= kReduceThreads + A_N doubles.
__device__ inline void reduce_b_part(const ReduceB &a, int s, double *lds)
{
    const int t = threadIdx.x;
    const int comp = t % A_N, g = t / A_N;
    constexpr int G = kReduceThreads / A_N;
    double v = 0.0;
    for (int c = a.sys_chunk[s] + g; c < a.sys_chunk[s + 1]; c += G)
        v += a.partial[(long long)c * A_N + comp];
    lds[t] = v;
    __syncthreads();
    if (t < A_N) {
        double r = 0.0;
        for (int x = t; x < kReduceThreads; x += A_N) r += lds[x];
        lds[kReduceThreads + t] = r;
    }
    __syncthreads();
    if (t == 0) energy_outputs(a, s, lds + kReduceThreads);
}

}  // namespace mixpi
