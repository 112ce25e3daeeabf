// Bonded sweep, half-kick/estimator epilogue and small bookkeeping kernels.
#include "mixpi.h"
#include "mixpi_internal.h"

namespace mixpi {

__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Adds v to slot of the accumulator row of `sys`: one atomic per wave when
// every lane of the wave belongs to the same system (work lists are sorted
// by system), one per lane otherwise.
__device__ __forceinline__ void acc_add(double *eacc, int sys, int slot, double v)
{
    const int s0 = __shfl(sys, 0, 64);
    const bool uniform = __all(sys == s0);
    if (uniform) {
        v = wsum(v);
        if ((threadIdx.x & 63) == 0 && s0 >= 0 && v != 0.0)
            unsafeAtomicAdd(&acc_row(eacc, s0, blockIdx.x)[slot], v);
    } else if (sys >= 0 && v != 0.0) {
        unsafeAtomicAdd(&acc_row(eacc, sys, blockIdx.x)[slot], v);
    }
}

__device__ __forceinline__ void min_img(double &x, double L, double iL) { x -= L * rint(x * iL); }

// Bonds and angles of V_mix (Eq. mts-hamiltonian, 2- and 3-body terms): one
// thread per (term, slice); the slice's beads were resolved on the host, so
// a thread sees plain bead rows and the weight 1/N_max.  FP64 throughout:
// bonded terms are stiff and cheap.
template <bool THETA>
__global__ __launch_bounds__(256) void k_bonded(BondedLaunch a)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int sys = -1;
    double eb = 0, ea = 0, gb = 0, ga = 0;
    if (t < a.n_bonds) {
        const BondTerm b = a.bonds[t];
        sys = b.sys;
        const SysDev &S = a.sys[sys];
        const double *th = a.theta ? a.theta + 6 * sys : S.theta0;
        const bool t0 = b.type == S.bond_off;
        const double k = t0 ? th[4] : a.bond_k[b.type];
        const double r0 = a.bond_r0[b.type];
        double d[3];
        for (int c = 0; c < 3; ++c) {
            d[c] = a.q[3LL * b.ra + c] - a.q[3LL * b.rb + c];
            min_img(d[c], S.box[c], S.ibox[c]);
        }
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double dr = r - r0;
        eb = b.w * 0.5 * k * dr * dr;
        if (THETA && t0) gb = b.w * 0.5 * dr * dr;
        const double g = -b.w * k * dr / r;
        for (int c = 0; c < 3; ++c) {
            unsafeAtomicAdd(&a.f[3LL * b.ra + c], g * d[c]);
            unsafeAtomicAdd(&a.f[3LL * b.rb + c], -g * d[c]);
        }
    } else if (t < (long long)a.n_bonds + a.n_angles) {
        const AngleTerm an = a.angles[t - a.n_bonds];
        sys = an.sys;
        const SysDev &S = a.sys[sys];
        const double *th = a.theta ? a.theta + 6 * sys : S.theta0;
        const bool t0 = an.type == S.angle_off;
        const double k = t0 ? th[5] : a.angle_k[an.type];
        const double th0 = a.angle_t0[an.type];
        double r1[3], r2[3];
        for (int c = 0; c < 3; ++c) {
            r1[c] = a.q[3LL * an.ra + c] - a.q[3LL * an.rv + c];
            r2[c] = a.q[3LL * an.rb + c] - a.q[3LL * an.rv + c];
            min_img(r1[c], S.box[c], S.ibox[c]);
            min_img(r2[c], S.box[c], S.ibox[c]);
        }
        const double l1 = sqrt(r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
        const double l2 = sqrt(r2[0] * r2[0] + r2[1] * r2[1] + r2[2] * r2[2]);
        double c = (r1[0] * r2[0] + r1[1] * r2[1] + r1[2] * r2[2]) / (l1 * l2);
        c = fmin(1.0, fmax(-1.0, c));
        const double dth = acos(c) - th0;
        ea = an.w * 0.5 * k * dth * dth;
        if (THETA && t0) ga = an.w * 0.5 * dth * dth;
        const double s = sqrt(1.0 - c * c);
        const double pref = an.w * k * dth / s;
        const double i12 = 1.0 / (l1 * l2), i11 = 1.0 / (l1 * l1), i22 = 1.0 / (l2 * l2);
        for (int x = 0; x < 3; ++x) {
            const double fa = pref * (r2[x] * i12 - c * r1[x] * i11);
            const double fb = pref * (r1[x] * i12 - c * r2[x] * i22);
            unsafeAtomicAdd(&a.f[3LL * an.ra + x], fa);
            unsafeAtomicAdd(&a.f[3LL * an.rb + x], fb);
            unsafeAtomicAdd(&a.f[3LL * an.rv + x], -(fa + fb));
        }
    }
    acc_add(a.eacc, sys, A_BOND, eb);
    acc_add(a.eacc, sys, A_ANGLE, ea);
    if (THETA) {
        acc_add(a.eacc, sys, A_TH4, gb);
        acc_add(a.eacc, sys, A_TH5, ga);
    }
}

void launch_bonded(const BondedLaunch &a, bool with_theta, hipStream_t st)
{
    const long long n = (long long)a.n_bonds + a.n_angles;
    if (n <= 0) return;
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (with_theta) hipLaunchKernelGGL((k_bonded<true>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_bonded<false>), grid, block, 0, st, a);
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

// Sums the accumulator copies of system s, slot k, and clears them.
__device__ __forceinline__ double take(double *eacc, int s, int k)
{
    double v = 0.0;
    for (int c = 0; c < kAccCopies; ++c) {
        double *p = eacc + ((long long)s * kAccCopies + c) * A_N + k;
        v += *p;
        *p = 0.0;
    }
    return v;
}

__global__ void k_write_energy(const SysDev *sys, int n_sys, double *eacc, double *e_out)
{
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n_sys; s += gridDim.x * blockDim.x) {
        double e[MIXPI_NV];
        e[MIXPI_E_LJ] = take(eacc, s, A_LJ);
        e[MIXPI_E_COUL] = take(eacc, s, A_COUL) + sys[s].bg_energy;
        e[MIXPI_E_PP] = take(eacc, s, A_PP);
        e[MIXPI_E_BOND] = take(eacc, s, A_BOND);
        e[MIXPI_E_ANGLE] = take(eacc, s, A_ANGLE);
        e[MIXPI_E_VMIX] = e[1] + e[2] + e[3] + e[4] + e[5];
        for (int k = A_SPRING; k < A_N; ++k) take(eacc, s, k);
        if (e_out)
            for (int k = 0; k < MIXPI_NV; ++k) e_out[(long long)s * MIXPI_NV + k] = e[k];
    }
}

void launch_write_energy(const SysDev *sys, int n_sys, double *eacc, double *e_out,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_write_energy, dim3((n_sys + 63) / 64), dim3(64), 0, st, sys, n_sys,
                       eacc, e_out);
}

// dq <- -grad_e[sys] * dq (dq holds F on entry); dtheta <- grad_e * dV/dtheta.
__global__ void k_adjoint_scale(long long rows, const int *row_part, const int *part_sys,
                                const double *grad_e, double *dq)
{
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= 3 * rows) return;
    const int s = part_sys[row_part[x / 3]];
    const double g = grad_e ? grad_e[s] : 1.0;
    dq[x] = -g * dq[x];
}

__global__ void k_adjoint_theta(int n_sys, double *eacc, const double *grad_e, double *dtheta)
{
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n_sys; s += gridDim.x * blockDim.x) {
        const double g = grad_e ? grad_e[s] : 1.0;
        for (int k = 0; k < 6; ++k) {
            const double v = take(eacc, s, A_TH0 + k);
            if (dtheta) dtheta[(long long)s * 6 + k] = g * v;
        }
        for (int k = 0; k < A_TH0; ++k) take(eacc, s, k);
        for (int k = A_TH5 + 1; k < A_N; ++k) take(eacc, s, k);
    }
}

void launch_adjoint_finish(const SysDev *sys, int n_sys, long long rows, const int *row_part,
                           const int *part_sys, const double *grad_e, double *dq,
                           double *eacc, double *dtheta, hipStream_t st)
{
    (void)sys;
    if (dq && rows > 0)
        hipLaunchKernelGGL(k_adjoint_scale, dim3((unsigned)((3 * rows + 255) / 256)), dim3(256),
                           0, st, rows, row_part, part_sys, grad_e, dq);
    hipLaunchKernelGGL(k_adjoint_theta, dim3((n_sys + 63) / 64), dim3(64), 0, st, n_sys, eacc,
                       grad_e, dtheta);
}

// ---------------------------------------------------------------------------
// Second half-kick and per-step energies.  One thread per bead component:
// p += dt/2 F, then the kinetic energy p^2/(2 m_f) and the centroid-virial
// term (q - qbar) . F are summed per system.  The last workgroup to finish
// (ticket) turns the accumulators into the energy-log row and clears them.
__global__ __launch_bounds__(256) void k_finish(FinishLaunch a)
{
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int sys = -1;
    double ke = 0.0, vir = 0.0;
    if (x < a.n3) {
        const long long row = x / 3;
        const int d = (int)(x - 3 * row);
        const int part = a.row_part[row];
        sys = a.part_sys[part];
        const double pv = a.p[x] + a.sys[sys].hkick * a.f[x];
        a.p[x] = pv;
        ke = pv * pv / (2.0 * a.fm[part]);
        vir = (a.q[x] - a.cent[3LL * part + d]) * a.f[x];
    }
    acc_add(a.eacc, sys, A_KIN, ke);
    acc_add(a.eacc, sys, A_VIR, vir);

    __shared__ bool last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned tk = atomicAdd(a.ticket, 1u);
        last = tk == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    for (int s = threadIdx.x; s < a.n_sys; s += blockDim.x) {
        const SysDev &S = a.sys[s];
        double v[A_N];
        for (int k = 0; k < A_N; ++k) {
            double sum = 0.0;
            for (int c = 0; c < kAccCopies; ++c) {
                double *pp = a.eacc + ((long long)s * kAccCopies + c) * A_N + k;
                unsigned long long old = atomicExch((unsigned long long *)pp, 0ull);
                sum += __longlong_as_double((long long)old);
            }
            v[k] = sum;
        }
        double e[MIXPI_NE];
        e[MIXPI_E_LJ] = v[A_LJ];
        e[MIXPI_E_COUL] = v[A_COUL] + S.bg_energy;
        e[MIXPI_E_PP] = v[A_PP];
        e[MIXPI_E_BOND] = v[A_BOND];
        e[MIXPI_E_ANGLE] = v[A_ANGLE];
        e[MIXPI_E_VMIX] = e[1] + e[2] + e[3] + e[4] + e[5];
        e[MIXPI_E_SPRING] = v[A_SPRING];
        e[MIXPI_E_KIN] = v[A_KIN] / kKcal;
        e[MIXPI_E_KCV] = S.cv_const - 0.5 * v[A_VIR];
        e[MIXPI_E_KPRIM] = S.prim_const - v[A_SPRING];
        e[MIXPI_E_HAM] = e[MIXPI_E_KIN] + e[MIXPI_E_SPRING] + e[MIXPI_E_VMIX];
        if (!isfinite(e[MIXPI_E_HAM])) atomicOr(a.nonfinite, 1);
        if (a.elog)
            for (int k = 0; k < MIXPI_NE; ++k) a.elog[(long long)s * MIXPI_NE + k] = e[k];
    }
    if (threadIdx.x == 0) atomicExch(a.ticket, 0u);
}

void launch_finish(const FinishLaunch &a, hipStream_t st)
{
    const long long blocks = (a.n3 + 255) / 256;
    hipLaunchKernelGGL(k_finish, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, st, a);
}

}  // namespace mixpi
