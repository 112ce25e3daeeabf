// Force gather, half-kick/estimator epilogue, energy reducer and small
// bookkeeping kernels.
#include <mutex>

#include "mixpi.h"
#include "mixpi_internal.h"
#include "device_common.h"

namespace mixpi {

// ---------------------------------------------------------------------------
// Device scratch of mixpi_forces_static: the partial-force slots, energy
// slots and reducer partials of one force evaluation, in a fixed array that
// every GPU the library runs on holds until the process ends.  In host code
// the array's name is not a device address: the address is looked up once
// per device (with that device current) and kept; only that address is ever
// passed to kernels.
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

namespace {
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    double *p = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

double *static_scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

// ---------------------------------------------------------------------------
// F[row] = sum over the row's partial-force slots, a contiguous run in the
// fixed CSR order (so forces are reproducible bit for bit).
struct Vec3 {
    double x, y, z;
};
// LPR lanes per row (lanes sl = 0 .. LPR-1 of an aligned group of the
// wave; LPR = 64 is one wave per row): slots sl, sl + LPR, ...; the group's
// lanes then reduce by DPP moves that stay inside the group, in a fixed
// order, and every lane of the group receives the sum.
template <int LPR>
__device__ __forceinline__ Vec3 gather_row_group(const GatherArgs &g, long long row, int sl)
{
    double x = 0.0, y = 0.0, z = 0.0;
    const long long e = g.row_ptr[row + 1];
    for (long long k = g.row_ptr[row] + sl; k < e; k += LPR) {
        const double *p = g.part + 3 * k;
        x += p[0];
        y += p[1];
        z += p[2];
    }
    return Vec3{group_sum<LPR>(x), group_sum<LPR>(y), group_sum<LPR>(z)};
}

// RPW rows per wave, grouped exactly as in the step epilogue, so that a
// force call and a step sum each row's partials in the same order.
template <int RPW>
__global__ __launch_bounds__(256) void k_gather(GatherArgs g, long long rows, double *f)
{
    constexpr int LPR = 64 / RPW;
    const int lane = threadIdx.x & 63;
    const long long row = (((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6) * RPW +
                          lane / LPR;
    if (row >= rows) return;   // whole groups leave together
    const int sl = lane % LPR;
    const Vec3 v = gather_row_group<LPR>(g, row, sl);
    if (sl == 0) {
        f[3 * row] = v.x;
        f[3 * row + 1] = v.y;
        f[3 * row + 2] = v.z;
    }
}

void launch_gather(const GatherArgs &g, long long rows, double *f, hipStream_t st, int rpw)
{
    if (rows <= 0) return;
    const long long waves = (rows + rpw - 1) / rpw;
    const dim3 grid((unsigned)((waves + 3) / 4));
    switch (rpw) {
    case 4: hipLaunchKernelGGL(k_gather<4>, grid, dim3(256), 0, st, g, rows, f); break;
    case 2: hipLaunchKernelGGL(k_gather<2>, grid, dim3(256), 0, st, g, rows, f); break;
    default: hipLaunchKernelGGL(k_gather<1>, grid, dim3(256), 0, st, g, rows, f); break;
    }
}

// ---------------------------------------------------------------------------
// Second half-kick and per-step energies.  One wave per bead row (a
// workgroup covers up to 4 rows of one system): F gathered from its partial
// slots and stored, p += dt/2 F, then the kinetic energy p^2/(2 m_f) and the
// centroid-virial term (q - qbar) . F summed into the workgroup's slot.  In
// velocity-Verlet mode the kick also carries the ring's spring force at the
// new positions, and the spring energy is summed here.
template <int RPW>
__global__ __launch_bounds__(256) void k_finish(FinishLaunch a)
{
    if ((int)blockIdx.x >= a.n_blocks) {
        // the extra workgroups: energy reduction (stage B) of the previous step
        __shared__ double racc[kReduceThreads + A_N];
        reduce_b_part(a.reduce, blockIdx.x - a.n_blocks, racc);
        return;
    }
    // RPW rows per wave: row w * RPW + lane / LPR of the block, lane sl of it
    constexpr int LPR = 64 / RPW;
    BlockRange br;
    if (a.uniform) {
        const long long b0 = (long long)blockIdx.x * (4 * RPW);
        br = BlockRange{0, (int)b0, (int)min((long long)(4 * RPW), a.rows - b0), 0};
    } else {
        br = a.blocks[blockIdx.x];
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sl = lane % LPR, ri = w * RPW + lane / LPR;
    double ke = 0.0, vir = 0.0, esp = 0.0;
    if (ri < br.count) {
        const long long row = (long long)br.begin + ri;
        // the row's own state, loaded before the gather so both are in flight
        const long long x = 3 * row + (sl < 3 ? sl : 0);
        const double p0 = a.p[x], q0 = a.q[x], c0 = a.cent[x];
        const double hk = a.row_hk[row], fm = a.row_fm[row];
        const int st = a.row_stage[row];
        double fsp = 0.0;
        if (a.vv) {
            // spring force of the ring at the new positions, and the energy
            // of the step (row, next): k/2 (q - q_next)^2
            const double k = a.row_ksp[row];
            const double qp = a.q[3 * a.row_prev[row] + (x - 3 * row)];
            const double qn = a.q[3 * a.row_next[row] + (x - 3 * row)];
            fsp = -k * (2.0 * q0 - qp - qn);
            if (sl < 3) esp = 0.5 * k * (q0 - qn) * (q0 - qn);
        } else if (a.row_spw) {
            // rings propagated by matrix-core items: their spring energy here
            const double spw = a.row_spw[row];
            if (spw != 0.0 && sl < 3) {
                const double qn = a.q[3 * a.row_next[row] + sl];
                esp = spw * (q0 - qn) * (q0 - qn);
            }
        }
        const double few = a.ew_rowf && sl < 3 ? a.ew_rowf[x] : 0.0;
        const Vec3 fv = gather_row_group<LPR>(a.gather, row, sl);
        if (sl < 3) {
            double fx = sl == 0 ? fv.x : (sl == 1 ? fv.y : fv.z);
            if (a.ew_rowf) fx += few;
            a.f[x] = fx;
            const double pv = p0 + hk * (fx + fsp);
            a.p[x] = pv;
            if (st >= 0) {
                a.stage[6LL * st + sl] = q0;
                a.stage[6LL * st + 3 + sl] = pv + hk * fx;
            }
            ke = pv * pv / (2.0 * fm);
            vir = (q0 - c0) * fx;
        }
    }
    // the workgroup's three sums: wave sums, then one exchange through LDS
    // (waves added in order)
    __shared__ double red3[3][4];
    ke = wsum(ke);
    vir = wsum(vir);
    if (a.vv || a.row_spw) esp = wsum(esp);
    if (lane == 0) {
        red3[0][w] = ke;
        red3[1][w] = vir;
        red3[2][w] = esp;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[3] = {0.0, 0.0, 0.0};
        for (int v = 0; v < 3; ++v)
            for (int k = 0; k < 4; ++k) t[v] += red3[v][k];
        double *e = a.eslot + (long long)blockIdx.x * A_N;
        for (int k = 0; k < A_N; ++k) e[k] = 0.0;
        e[A_KIN] = t[0];
        e[A_VIR] = t[1];
        e[A_SPRING] = t[2];
    }
}

void launch_finish(const FinishLaunch &a, hipStream_t st)
{
    const int grid = a.n_blocks + (a.with_reduce ? a.reduce.n_wg : 0);
    if (grid <= 0) return;
    switch (a.rpw) {
    case 4: hipLaunchKernelGGL(k_finish<4>, dim3(grid), dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL(k_finish<2>, dim3(grid), dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL(k_finish<1>, dim3(grid), dim3(256), 0, st, a); break;
    }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_stage(StageLaunch a)
{
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= 3LL * a.n) return;
    const long long s = x / 3;
    const int c = (int)(x - 3 * s);
    const long long g = 3 * a.rows[s] + c;
    a.stage[6 * s + c] = a.q[g];
    a.stage[6 * s + 3 + c] = a.p[g] + a.row_hk[a.rows[s]] * a.f[g];
}

void launch_stage(const StageLaunch &a, hipStream_t st)
{
    if (a.n <= 0) return;
    hipLaunchKernelGGL(k_stage, dim3((unsigned)((3LL * a.n + 255) / 256)), dim3(256), 0, st, a);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kReduceThreads) void k_reduce_a(ReduceA a)
{
    __shared__ double acc[kReduceThreads];
    reduce_a_part(a, blockIdx.x, acc);
}

__global__ __launch_bounds__(kReduceThreads) void k_reduce_b(ReduceB b)
{
    __shared__ double acc[kReduceThreads + A_N];
    reduce_b_part(b, blockIdx.x, acc);
}

void launch_reduce(const ReduceA &a, const ReduceB &b, hipStream_t st)
{
    if (a.n_chunks > 0)
        hipLaunchKernelGGL(k_reduce_a, dim3(a.n_chunks), dim3(kReduceThreads), 0, st, a);
    hipLaunchKernelGGL(k_reduce_b, dim3(b.n_wg), dim3(kReduceThreads), 0, st, b);
}

// ---------------------------------------------------------------------------

__global__ void k_fill(double *x, long long n, double v)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        x[i] = v;
}

void launch_fill(double *x, long long n, double v, hipStream_t st)
{
    if (n <= 0) return;
    long long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, x, n, v);
}

// Holds the stream for `ticks` of the 100 MHz wall clock (bounded wait).
__global__ void k_delay(long long ticks)
{
    const long long t0 = wall_clock64();
    while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(16);
}

void launch_delay(long long ticks, hipStream_t st)
{
    hipLaunchKernelGGL(k_delay, dim3(1), dim3(1), 0, st, ticks);
}

// dq <- -grad_e[sys] * dq (dq holds F on entry).
__global__ void k_scale_rows(long long rows, const int *row_sys, const double *grad_e,
                             double *dq)
{
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= 3 * rows) return;
    const int s = row_sys[x / 3];
    const double g = grad_e ? grad_e[s] : 1.0;
    dq[x] = -g * dq[x];
}

void launch_scale_rows(long long rows, const int *row_sys, const double *grad_e, double *dq,
                       hipStream_t st)
{
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_scale_rows, dim3((unsigned)((3 * rows + 255) / 256)), dim3(256), 0, st,
                       rows, row_sys, grad_e, dq);
}

}  // namespace mixpi
