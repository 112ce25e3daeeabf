// Long-range electrostatics between ring-polymer centroids (arXiv
// 2411.11988, Sec. "Theory": the example systems' smooth-particle-mesh
// Ewald electrostatics, with the bead-bead energies and forces replaced by
// those between the centroids).  The Ewald sum of the atom charges z_i at
// the centroids c_i: a real-space erfc sum within r_cut, the erf
// correction of excluded (same-molecule) pairs, the reciprocal part by
// smooth particle-mesh Ewald (Essmann et al., J. Chem. Phys. 103, 8577
// (1995)), and the self and neutralising-background constants.  Each bead
// of particle i receives F_i / N_i.
//
// Launch sequence, every system of the handle at once:
//   k_ew_prep     centroids; zero the fixed-point charge grid
//   k_ew_spread   cardinal B-spline weights of order P; one lane per (x, y)
//                 spline point adds its P z-points with int64 atomics in
//                 fixed point (exact, so the grid is independent of order)
//   k_ew_fft x3   3D FFT, forward; the first pass converts fixed point to
//                 FP64 complex
//   k_ew_recip    multiply by the influence function G = B C, energy
//                 partials sum G |F(Q)|^2
//   k_ew_fft x3   inverse (unnormalised): the convolution (theta * Q)
//   k_ew_real     real-space and exclusion terms, one thread per particle
//                 against its system's particles staged in LDS
//   k_ew_gather   spline-derivative gather of the convolution, plus the
//                 real-space force; bead forces F_i / N_i
//   k_ew_reduce   per-system energies in a fixed order
#include "device_common.h"
#include "mixpi_internal.h"

namespace mixpi {

namespace {

constexpr int kEwThreads = 256;
constexpr int kFftLines = 16;   // lines per FFT workgroup

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Scaled fractional coordinate u = K frac(c / L), its grid base floor(u)
// and offset w = u - base in [0, 1).
__device__ __forceinline__ void grid_coord(double c, double L, int K, int &base, double &w)
{
    double f = c / L;
    f -= floor(f);
    const double u = K * f;
    const double b = floor(u);
    base = (int)b;
    w = u - b;
}

// Cardinal B-spline values v[j] = M_P(w + j) and derivatives d[j] =
// M_{P-1}(w + j) - M_{P-1}(w + j - 1), j = 0 .. P-1, by the recursion
// M_k(u) = (u M_{k-1}(u) + (k - u) M_{k-1}(u - 1)) / (k - 1) from
// M_2(w) = w, M_2(w + 1) = 1 - w.
template <int P>
__device__ __forceinline__ void bspline(double w, double v[P], double d[P])
{
    double m[P];
#pragma unroll
    for (int j = 0; j < P; ++j) m[j] = 0.0;
    m[0] = w;
    m[1] = 1.0 - w;
#pragma unroll
    for (int k = 3; k <= P; ++k) {
        const double inv = 1.0 / (k - 1);
        if (k == P) {
#pragma unroll
            for (int j = 0; j < P; ++j) d[j] = m[j] - (j > 0 ? m[j - 1] : 0.0);
        }
#pragma unroll
        for (int j = k - 1; j >= 0; --j) {
            const double a = (w + j) * m[j];
            const double b = j > 0 ? (k - w - j) * m[j - 1] : 0.0;
            m[j] = (a + b) * inv;
        }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) v[j] = m[j];
}

__device__ __forceinline__ int wrap(int i, int K)
{
    i %= K;
    return i < 0 ? i + K : i;
}

// ---- centroids, grid clear --------------------------------------------------
__global__ __launch_bounds__(kEwThreads) void k_ew_prep(EwaldLaunch a)
{
    const long long gid = (long long)blockIdx.x * kEwThreads + threadIdx.x;
    const long long ngrid = (long long)a.n_sys * a.K * a.K * a.K;
    for (long long k = gid; k < ngrid; k += (long long)gridDim.x * kEwThreads) a.grid_i[k] = 0;
    // one wave per particle
    const int wid = (int)(gid >> 6);
    const int lane = threadIdx.x & 63;
    for (int i = wid; i < a.n_part; i += (int)((long long)gridDim.x * kEwThreads / 64)) {
        const PartDev pd = a.parts[i];
        double sx = 0, sy = 0, sz = 0;
        for (int j = lane; j < pd.nb; j += 64) {
            const long long r = pd.row0 + (long long)j * pd.stride;
            sx += a.q[3 * r];
            sy += a.q[3 * r + 1];
            sz += a.q[3 * r + 2];
        }
        sx = wave_sum(sx);
        sy = wave_sum(sy);
        sz = wave_sum(sz);
        if (lane == 0) {
            a.cpos[3LL * i] = sx / pd.nb;
            a.cpos[3LL * i + 1] = sy / pd.nb;
            a.cpos[3LL * i + 2] = sz / pd.nb;
        }
    }
}

// ---- charge spreading -------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kEwThreads) void k_ew_spread(EwaldLaunch a)
{
    const int i = blockIdx.x * (kEwThreads / 64) + ((int)threadIdx.x >> 6);
    if (i >= a.n_part) return;
    const double z = a.z[i];
    if (z == 0.0) return;
    const int lane = threadIdx.x & 63;
    const int s = a.parts[i].sys;
    const SysDev &S = a.sys[s];
    const int K = a.K;
    int b[3];
    double v[3][P], dv[P];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double w;
        grid_coord(a.cpos[3LL * i + c], S.box[c], K, b[c], w);
        bspline<P>(w, v[c], dv);
    }
    if (lane >= P * P) return;
    const int ja = lane / P, jb = lane % P;
    double vx = 0, vy = 0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
        vx = j == ja ? v[0][j] : vx;
        vy = j == jb ? v[1][j] : vy;
    }
    const double zxy = z * vx * vy * a.scale;
    unsigned long long *g = (unsigned long long *)a.grid_i + (long long)s * K * K * K +
                            ((long long)wrap(b[0] - ja, K) * K + wrap(b[1] - jb, K)) * K;
#pragma unroll
    for (int jc = 0; jc < P; ++jc) {
        const long long fx = (long long)rint(zxy * v[2][jc]);
        atomicAdd(&g[wrap(b[2] - jc, K)], (unsigned long long)fx);
    }
}

// ---- 3D FFT: kFftLines lines of K points per workgroup ------------------------
// axis 2 (z): lines (x, y), contiguous; axis 1 (y): lines (x, z), stride K;
// axis 0 (x): lines (y, z), stride K^2.  For axes 0 and 1 the workgroup's
// lines are kFftLines consecutive z, so every point row is one contiguous
// 256-byte run.  Radix-2 decimation in time from bit-reversed LDS order;
// sign -1 forward (exp(-2 pi i jk / K)), +1 inverse (unnormalised).
__global__ __launch_bounds__(kEwThreads) void k_ew_fft(EwaldLaunch a, int axis, int sign,
                                                       int from_fixed)
{
    extern __shared__ double2 lds_fft[];
    const int K = a.K, logK = a.logK;
    const long long K2 = (long long)K * K;
    const int groups = (int)(K2 / kFftLines);
    const int s = blockIdx.x / groups;
    const int g = blockIdx.x % groups;
    double2 *data = a.grid_c + (long long)s * K2 * K;
    const long long *fixed = a.grid_i + (long long)s * K2 * K;
    long long base0;
    long long lstep, stride;
    if (axis == 2) {
        base0 = (long long)g * kFftLines * K;
        lstep = K;
        stride = 1;
    } else {
        const int outer = g / (K / kFftLines), z0 = (g % (K / kFftLines)) * kFftLines;
        base0 = (axis == 1 ? (long long)outer * K2 : (long long)outer * K) + z0;
        lstep = 1;
        stride = axis == 1 ? K : K2;
    }
    const int tot = kFftLines * K;
    for (int e = threadIdx.x; e < tot; e += kEwThreads) {
        int li, pt;
        if (axis == 2) {
            li = e / K;
            pt = e % K;
        } else {
            li = e % kFftLines;
            pt = e / kFftLines;
        }
        const long long addr = base0 + li * lstep + pt * stride;
        double2 x;
        if (from_fixed) {
            x.x = (double)fixed[addr] * a.inv_scale;
            x.y = 0.0;
        } else {
            x = data[addr];
        }
        const int rev = (int)(__builtin_bitreverse32((unsigned)pt) >> (32 - logK));
        lds_fft[li * K + rev] = x;
    }
    __syncthreads();
    const int half_tot = tot / 2;
    for (int st = 1; st <= logK; ++st) {
        const int m = 1 << st, h = m >> 1;
        for (int bfly = threadIdx.x; bfly < half_tot; bfly += kEwThreads) {
            const int li = bfly / (K / 2), bb = bfly % (K / 2);
            const int grp = bb / h, pos = bb % h;
            const int i0 = li * K + grp * m + pos, i1 = i0 + h;
            double2 w = a.tw[pos * (K / m)];
            w.y *= sign == -1 ? 1.0 : -1.0;   // table holds exp(-2 pi i j / K)
            const double2 u = lds_fft[i0], v = lds_fft[i1];
            const double tr = w.x * v.x - w.y * v.y, ti = w.x * v.y + w.y * v.x;
            lds_fft[i0] = make_double2(u.x + tr, u.y + ti);
            lds_fft[i1] = make_double2(u.x - tr, u.y - ti);
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < tot; e += kEwThreads) {
        int li, pt;
        if (axis == 2) {
            li = e / K;
            pt = e % K;
        } else {
            li = e % kFftLines;
            pt = e / kFftLines;
        }
        data[base0 + li * lstep + pt * stride] = lds_fft[li * K + pt];
    }
}

// ---- influence function and reciprocal energy ----------------------------------
__global__ __launch_bounds__(kEwThreads) void k_ew_recip(EwaldLaunch a)
{
    const long long K3 = (long long)a.K * a.K * a.K;
    const int s = blockIdx.x / a.recip_wg;
    const int w = blockIdx.x % a.recip_wg;
    const long long per = K3 / a.recip_wg;
    double2 *data = a.grid_c + (long long)s * K3;
    const double *G = a.G + (long long)s * K3;
    double e = 0.0;
    for (long long k = w * per + threadIdx.x; k < (w + 1) * per; k += kEwThreads) {
        const double2 f = data[k];
        const double gk = G[k];
        e += gk * (f.x * f.x + f.y * f.y);
        data[k] = make_double2(gk * f.x, gk * f.y);
    }
    __shared__ double red[kEwThreads / 64];
    e = wave_sum(e);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kEwThreads / 64; ++k) t += red[k];
        a.e_recip_part[blockIdx.x] = 0.5 * kCoulombKcal * t;
    }
}

// ---- real space ---------------------------------------------------------------
__global__ __launch_bounds__(kEwThreads) void k_ew_real(EwaldLaunch a)
{
    const BlockRange rg = a.real_ranges[blockIdx.x];
    const SysDev &S = a.sys[rg.sys];
    const int p0 = a.sys_part[rg.sys], p1 = a.sys_part[rg.sys + 1];
    const int i = rg.begin + (int)threadIdx.x;
    const bool vi = (int)threadIdx.x < rg.count;
    double xi = 0, yi = 0, zi = 0, qi = 0;
    int mi = -1;
    if (vi) {
        xi = a.cpos[3LL * i];
        yi = a.cpos[3LL * i + 1];
        zi = a.cpos[3LL * i + 2];
        qi = a.z[i];
        mi = a.mol[i];
    }
    __shared__ double sx[kEwThreads], sy[kEwThreads], sz[kEwThreads], sq[kEwThreads];
    __shared__ int sm[kEwThreads];
    const double alpha = a.alpha, rc2 = a.r_cut * a.r_cut;
    const double two_a_rpi = 2.0 * alpha / sqrt(kPi);
    double fx = 0, fy = 0, fz = 0, e = 0;
    for (int j0 = p0; j0 < p1; j0 += kEwThreads) {
        const int j = j0 + (int)threadIdx.x;
        __syncthreads();
        if (j < p1) {
            sx[threadIdx.x] = a.cpos[3LL * j];
            sy[threadIdx.x] = a.cpos[3LL * j + 1];
            sz[threadIdx.x] = a.cpos[3LL * j + 2];
            sq[threadIdx.x] = a.z[j];
            sm[threadIdx.x] = a.mol[j];
        }
        __syncthreads();
        const int jn = min(kEwThreads, p1 - j0);
        if (!vi || qi == 0.0) continue;
        for (int t = 0; t < jn; ++t) {
            const double qq = qi * sq[t];
            if (qq == 0.0 || j0 + t == i) continue;
            double dx = xi - sx[t], dy = yi - sy[t], dz = zi - sz[t];
            dx -= S.box[0] * rint(dx * S.ibox[0]);
            dy -= S.box[1] * rint(dy * S.ibox[1]);
            dz -= S.box[2] * rint(dz * S.ibox[2]);
            const double r2 = dx * dx + dy * dy + dz * dz;
            const bool excl = sm[t] == mi;
            if (!excl && !(r2 < rc2)) continue;
            const double r = sqrt(r2);
            const double gauss = two_a_rpi * exp(-alpha * alpha * r2);
            double v, g;
            if (excl) {
                const double ef = erf(alpha * r);
                v = -ef / r;
                g = kCoulombKcal * qq * (gauss * r - ef) / (r2 * r);
            } else {
                const double ec = erfc(alpha * r);
                v = ec / r;
                g = kCoulombKcal * qq * (gauss * r + ec) / (r2 * r);
            }
            e += 0.5 * kCoulombKcal * qq * v;
            fx += g * dx;
            fy += g * dy;
            fz += g * dz;
        }
    }
    if (vi) {
        a.freal[3LL * i] = fx;
        a.freal[3LL * i + 1] = fy;
        a.freal[3LL * i + 2] = fz;
    }
    __shared__ double red[kEwThreads / 64];
    e = wave_sum(e);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kEwThreads / 64; ++k) t += red[k];
        a.e_real_part[blockIdx.x] = t;
    }
}

// ---- force gather and bead forces ---------------------------------------------
template <int P>
__global__ __launch_bounds__(kEwThreads) void k_ew_gather(EwaldLaunch a)
{
    const int i = blockIdx.x * (kEwThreads / 64) + ((int)threadIdx.x >> 6);
    if (i >= a.n_part) return;
    const int lane = threadIdx.x & 63;
    const PartDev pd = a.parts[i];
    const double z = a.z[i];
    double F[3] = {a.freal[3LL * i], a.freal[3LL * i + 1], a.freal[3LL * i + 2]};
    if (z != 0.0) {
        const SysDev &S = a.sys[pd.sys];
        const int K = a.K;
        int b[3];
        double v[3][P], d[3][P];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double w;
            grid_coord(a.cpos[3LL * i + c], S.box[c], K, b[c], w);
            bspline<P>(w, v[c], d[c]);
        }
        double gx = 0, gy = 0, gz = 0;
        if (lane < P * P) {
            const int ja = lane / P, jb = lane % P;
            double vx = 0, vy = 0, dx = 0, dy = 0;
#pragma unroll
            for (int j = 0; j < P; ++j) {
                vx = j == ja ? v[0][j] : vx;
                dx = j == ja ? d[0][j] : dx;
                vy = j == jb ? v[1][j] : vy;
                dy = j == jb ? d[1][j] : dy;
            }
            const double2 *row = a.grid_c + (long long)pd.sys * K * K * K +
                                 ((long long)wrap(b[0] - ja, K) * K + wrap(b[1] - jb, K)) * K;
#pragma unroll
            for (int jc = 0; jc < P; ++jc) {
                const double cv = row[wrap(b[2] - jc, K)].x;
                gx += cv * dx * vy * v[2][jc];
                gy += cv * vx * dy * v[2][jc];
                gz += cv * vx * vy * d[2][jc];
            }
        }
        gx = wave_sum(gx);
        gy = wave_sum(gy);
        gz = wave_sum(gz);
        F[0] -= kCoulombKcal * z * gx * K / S.box[0];
        F[1] -= kCoulombKcal * z * gy * K / S.box[1];
        F[2] -= kCoulombKcal * z * gz * K / S.box[2];
    }
    if (lane == 0) {
        a.fcent[3LL * i] = F[0];
        a.fcent[3LL * i + 1] = F[1];
        a.fcent[3LL * i + 2] = F[2];
    }
    if (a.f) {
        const double inv = 1.0 / pd.nb;
        for (int j = lane; j < pd.nb; j += 64) {
            const long long r = pd.row0 + (long long)j * pd.stride;
            a.f[3 * r] += F[0] * inv;
            a.f[3 * r + 1] += F[1] * inv;
            a.f[3 * r + 2] += F[2] * inv;
        }
    }
}

// ---- per-system energies ------------------------------------------------------
__global__ __launch_bounds__(64) void k_ew_reduce(EwaldLaunch a)
{
    const int s = blockIdx.x;
    const int lane = threadIdx.x;
    double er = 0.0, ek = 0.0;
    for (int k = a.real_first[s] + lane; k < a.real_first[s + 1]; k += 64) er += a.e_real_part[k];
    for (int k = lane; k < a.recip_wg; k += 64) ek += a.e_recip_part[(long long)s * a.recip_wg + k];
    er = wave_sum(er);
    ek = wave_sum(ek);
    if (lane == 0) {
        a.e_out[3 * s] = er;
        a.e_out[3 * s + 1] = ek;
        a.e_out[3 * s + 2] = a.e_const[s];
    }
}

template <int P>
void launch_order(const EwaldLaunch &a, hipStream_t st)
{
    const int per = kEwThreads / 64;
    const int pblocks = (a.n_part + per - 1) / per;
    hipLaunchKernelGGL(k_ew_spread<P>, dim3(pblocks), dim3(kEwThreads), 0, st, a);
    const int groups = a.K * a.K / kFftLines * a.n_sys;
    const size_t lds = sizeof(double2) * kFftLines * a.K;
    hipLaunchKernelGGL(k_ew_fft, dim3(groups), dim3(kEwThreads), lds, st, a, 2, -1, 1);
    hipLaunchKernelGGL(k_ew_fft, dim3(groups), dim3(kEwThreads), lds, st, a, 1, -1, 0);
    hipLaunchKernelGGL(k_ew_fft, dim3(groups), dim3(kEwThreads), lds, st, a, 0, -1, 0);
    hipLaunchKernelGGL(k_ew_recip, dim3(a.n_sys * a.recip_wg), dim3(kEwThreads), 0, st, a);
    hipLaunchKernelGGL(k_ew_fft, dim3(groups), dim3(kEwThreads), lds, st, a, 0, 1, 0);
    hipLaunchKernelGGL(k_ew_fft, dim3(groups), dim3(kEwThreads), lds, st, a, 1, 1, 0);
    hipLaunchKernelGGL(k_ew_fft, dim3(groups), dim3(kEwThreads), lds, st, a, 2, 1, 0);
    hipLaunchKernelGGL(k_ew_real, dim3(a.n_real), dim3(kEwThreads), 0, st, a);
    hipLaunchKernelGGL(k_ew_gather<P>, dim3(pblocks), dim3(kEwThreads), 0, st, a);
    hipLaunchKernelGGL(k_ew_reduce, dim3(a.n_sys), dim3(64), 0, st, a);
}

}  // namespace

void launch_ewald(const EwaldLaunch &a, hipStream_t st)
{
    if (a.n_part <= 0) return;
    const long long ngrid = (long long)a.n_sys * a.K * a.K * a.K;
    const long long want = std::max<long long>((ngrid + kEwThreads - 1) / kEwThreads,
                                               ((long long)a.n_part * 64 + kEwThreads - 1) / kEwThreads);
    const int blocks = (int)std::min<long long>(want, 16384);
    hipLaunchKernelGGL(k_ew_prep, dim3(blocks), dim3(kEwThreads), 0, st, a);
    switch (a.order) {
    case 4: launch_order<4>(a, st); break;
    case 6: launch_order<6>(a, st); break;
    default: launch_order<8>(a, st); break;
    }
}

}  // namespace mixpi
