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
// Five launches, every system of the handle at once:
//   k_ew_prep     one wave per particle: its centroid, then the grid bases
//                 and cardinal B-spline weights of order P of each axis
//   k_ew_plane    per x-plane: spread the charges whose x-support holds the
//                 plane into LDS as int64 fixed point (exact, so the grid
//                 does not depend on the order of the adds), then the
//                 forward 2D FFT (z, then y) in LDS
//   k_ew_xline    per 16 x-lines: forward FFT along x, multiply by the
//                 influence function G = B C with the energy partial
//                 sum G |F(Q)|^2, inverse FFT along x; the same grid runs
//                 the real-space workgroups: erfc terms within r_cut and the
//                 erf correction of excluded pairs, (64 i) x (kEwChunk j) tiles
//   k_ew_plane    inverse 2D FFT (y, then z): the convolution (theta * Q)
//   k_ew_gather   spline-derivative gather of the convolution plus the
//                 real-space partials, bead forces F_i / N_i; one extra
//                 workgroup per system sums its energies in a fixed order
// FFTs are radix-2 decimation in time from bit-reversed order, sign -1
// forward (exp(-2 pi i jk / K)), +1 inverse, unnormalised.
#include "device_common.h"
#include "mixpi_internal.h"

namespace mixpi {

namespace {

constexpr int kEwThreads = 256;
constexpr int kFftLines = 16;   // lines per FFT workgroup

__device__ __forceinline__ double wave_sum(double v) { return wsum(v); }

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

// ---- centroids and spline tables --------------------------------------------
// One wave per particle: its centroid, and for a charged particle the grid
// bases floor(u) and the order-P weights M_P(w + j) of the three axes.
template <int P>
__global__ __launch_bounds__(kEwThreads) void k_ew_prep(EwaldLaunch a)
{
    const int i = blockIdx.x * (kEwThreads / 64) + ((int)threadIdx.x >> 6);
    if (i >= a.n_part) return;
    const int lane = threadIdx.x & 63;
    const PartDev pd = a.parts[i];
    double c[3] = {0.0, 0.0, 0.0};
    for (int j = lane; j < pd.nb; j += 64) {
        const long long r = pd.row0 + (long long)j * pd.stride;
        c[0] += a.q[3 * r];
        c[1] += a.q[3 * r + 1];
        c[2] += a.q[3 * r + 2];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) c[k] = wave_sum(c[k]) / pd.nb;
    if (lane == 0) {
        a.cpos[3LL * i] = c[0];
        a.cpos[3LL * i + 1] = c[1];
        a.cpos[3LL * i + 2] = c[2];
    }
    if (a.z[i] == 0.0) return;
    const SysDev &S = a.sys[pd.sys];
    int b[3];
    double v[3][P], dv[P];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double w;
        grid_coord(c[k], S.box[k], a.K, b[k], w);
        bspline<P>(w, v[k], dv);
    }
    if (lane < 3) a.spl_base[4LL * i + lane] = b[lane];
    if (lane < 3 * P) {
        const int k = lane / P, j = lane % P;
        double x = 0.0;
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
#pragma unroll
            for (int jj = 0; jj < P; ++jj) x = (kk == k && jj == j) ? v[kk][jj] : x;
        a.spl_w[(long long)i * 3 * kMaxOrder + k * kMaxOrder + j] = x;
    }
}

// ---- FFT building blocks in LDS ------------------------------------------------
__device__ __forceinline__ int bitrev(int x, int logK)
{
    return (int)(__builtin_bitreverse32((unsigned)x) >> (32 - logK));
}

__device__ __forceinline__ void butterfly(double2 *x0, double2 *x1, double2 w)
{
    const double2 u = *x0, v = *x1;
    const double tr = w.x * v.x - w.y * v.y, ti = w.x * v.y + w.y * v.x;
    *x0 = make_double2(u.x + tr, u.y + ti);
    *x1 = make_double2(u.x - tr, u.y - ti);
}

// twiddle exp(sign 2 pi i pos / m) from the table exp(-2 pi i j / K)
__device__ __forceinline__ double2 twiddle(const double2 *tw, int pos, int m, int K, int sign)
{
    double2 w = tw[pos * (K / m)];
    if (sign > 0) w.y = -w.y;
    return w;
}

// Radix-2 passes over `lines` lines of K points held in bit-reversed order:
// point p of line l at buf[l * lstride + p * pstride].  With line_fast the
// threads of a wave take consecutive lines at one butterfly position (use
// when lstride is 1), otherwise consecutive positions of one line (use when
// pstride is 1), so a wave's LDS accesses stay contiguous.
__device__ void fft_lines(double2 *buf, int lines, int lstride, int pstride, bool line_fast,
                          int K, int logK, const double2 *tw, int sign)
{
    const int half = K / 2, nb = lines * half;
    for (int st = 1; st <= logK; ++st) {
        const int m = 1 << st, h = m >> 1;
        for (int t = threadIdx.x; t < nb; t += blockDim.x) {
            const int l = line_fast ? t % lines : t / half;
            const int bb = line_fast ? t / lines : t % half;
            const int grp = bb / h, pos = bb % h;
            const int p0 = grp * m + pos;
            double2 *x0 = buf + l * lstride + p0 * pstride;
            butterfly(x0, x0 + h * pstride, twiddle(tw, pos, m, K, sign));
        }
        __syncthreads();
    }
}

// In-place bit-reversal of every line (pairs p < rev(p) swapped).
__device__ void bitrev_lines(double2 *buf, int lines, int lstride, int pstride, bool line_fast,
                             int K, int logK)
{
    for (int t = threadIdx.x; t < lines * K; t += blockDim.x) {
        const int l = line_fast ? t % lines : t / K;
        const int p = line_fast ? t / lines : t % K;
        const int r = bitrev(p, logK);
        if (p < r) {
            double2 *a = buf + l * lstride + p * pstride, *b = buf + l * lstride + r * pstride;
            const double2 x = *a;
            *a = *b;
            *b = x;
        }
    }
    __syncthreads();
}

__device__ void real_space(const EwaldLaunch &a, const RealItem &it, int slot);

// ---- 2D FFT of x-planes (and the real-space workgroups) -------------------------
// Plane x of system s as P[y][z] (row stride K).  Forward: from the
// fixed-point grid (cleared for the next call), FFT along z then y.
// Inverse: y then z.
template <int P, int NT>
__global__ __launch_bounds__(NT) void k_ew_plane(EwaldLaunch a, int sign)
{
    extern __shared__ double2 plane[];
    const int K = a.K, logK = a.logK;
    const int s = blockIdx.x / K, x = blockIdx.x % K;
    const long long off = (long long)s * K * K * K + (long long)x * K * K;
    double2 *data = a.grid_c + off;
    const int ld = K;
    // the twiddle table follows the plane in LDS when the launch made room
    const double2 *tw = a.tw;
    if (a.tw_in_lds) {
        double2 *t = plane + K * K;
        for (int j = threadIdx.x; j < K / 2; j += NT) t[j] = a.tw[j];
        tw = t;
    }
    if (sign < 0) {
        // charge spreading of this plane: every charged particle of the
        // system whose x-support holds the plane adds z M(x) M(y) M(z) in
        // fixed point (int64 in the real words, z at its bit-reversed
        // place).  Batches of particles: the matching ones are listed in the
        // plane's imaginary words (free until the conversion), then the
        // (particle, y-point) items are shared out, P adds each.
        unsigned long long *acc = (unsigned long long *)plane;   // real words 2e, free 2e + 1
        __shared__ int n_match;
        for (int e = threadIdx.x; e < K * K; e += NT) plane[e] = make_double2(0.0, 0.0);
        const int batch = K * K < 1024 ? K * K : 1024;
        for (int i0 = a.sys_part[s]; i0 < a.sys_part[s + 1]; i0 += batch) {
            if (threadIdx.x == 0) n_match = 0;
            __syncthreads();
            const int i1 = min(i0 + batch, a.sys_part[s + 1]);
            for (int i = i0 + threadIdx.x; i < i1; i += NT) {
                if (a.z[i] == 0.0) continue;
                const int ja = wrap(a.spl_base[4LL * i] - x, K);
                if (ja >= P) continue;
                const int m = atomicAdd(&n_match, 1);
                acc[2 * m + 1] = (unsigned long long)i | ((unsigned long long)ja << 32);
            }
            __syncthreads();
            const int items = n_match * P;
            for (int it = threadIdx.x; it < items; it += NT) {
                const unsigned long long e = acc[2 * (it / P) + 1];
                const int i = (int)(e & 0xffffffffu), ja = (int)(e >> 32), jb = it % P;
                const double *w = a.spl_w + (long long)i * 3 * kMaxOrder;
                const int row = wrap(a.spl_base[4LL * i + 1] - jb, K) * ld;
                const int bz = a.spl_base[4LL * i + 2];
                const double zxy = a.z[i] * w[ja] * a.scale * w[kMaxOrder + jb];
#pragma unroll
                for (int jc = 0; jc < P; ++jc) {
                    const long long fx = (long long)rint(zxy * w[2 * kMaxOrder + jc]);
                    atomicAdd(&acc[2 * (row + bitrev(wrap(bz - jc, K), logK))],
                              (unsigned long long)fx);
                }
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < K * K; e += NT) {
            const long long fx = (long long)acc[2 * e];
            plane[e] = make_double2((double)fx * a.inv_scale, 0.0);
        }
        __syncthreads();
        fft_lines(plane, K, ld, 1, false, K, logK, tw, sign);     // along z
        bitrev_lines(plane, K, 1, ld, true, K, logK);
        fft_lines(plane, K, 1, ld, true, K, logK, tw, sign);      // along y
    } else {
        for (int e = threadIdx.x; e < K * K; e += NT) {
            const int y = e / K, z = e % K;
            plane[bitrev(y, logK) * ld + z] = data[e];
        }
        __syncthreads();
        fft_lines(plane, K, 1, ld, true, K, logK, tw, sign);      // along y
        bitrev_lines(plane, K, ld, 1, false, K, logK);
        fft_lines(plane, K, ld, 1, false, K, logK, tw, sign);     // along z
    }
    for (int e = threadIdx.x; e < K * K; e += NT) {
        const int y = e / K, z = e % K;
        data[e] = plane[y * ld + z];
    }
}

// ---- x-lines: forward FFT, influence function and energy, inverse FFT ---------
__global__ __launch_bounds__(kEwThreads) void k_ew_xline(EwaldLaunch a)
{
    extern __shared__ double2 xl[];
    const int K = a.K, logK = a.logK;
    const int groups = K * K / kFftLines;
    if ((int)blockIdx.x >= a.n_sys * groups) {
        const int k = blockIdx.x - a.n_sys * groups;
        real_space(a, a.real_items[k], k);
        return;
    }
    const int s = blockIdx.x / groups, g = blockIdx.x % groups;
    const int y = g / (K / kFftLines), z0 = (g % (K / kFftLines)) * kFftLines;
    const long long K2 = (long long)K * K;
    const long long base = (long long)s * K2 * K + (long long)y * K + z0;
    double2 *data = a.grid_c + base;
    const double *G = a.G + base;
    double2 *tw = xl + kFftLines * K;
    for (int j = threadIdx.x; j < K / 2; j += kEwThreads) tw[j] = a.tw[j];
    // xl[l][x], line l = z0 + l, row stride K
    for (int e = threadIdx.x; e < kFftLines * K; e += kEwThreads) {
        const int l = e % kFftLines, x = e / kFftLines;
        xl[l * K + bitrev(x, logK)] = data[x * K2 + l];
    }
    __syncthreads();
    fft_lines(xl, kFftLines, K, 1, false, K, logK, tw, -1);
    double en = 0.0;
    for (int e = threadIdx.x; e < kFftLines * K; e += kEwThreads) {
        const int l = e % kFftLines, x = e / kFftLines;
        const double gk = G[x * K2 + l];
        const double2 f = xl[l * K + x];
        en += gk * (f.x * f.x + f.y * f.y);
        xl[l * K + x] = make_double2(gk * f.x, gk * f.y);
    }
    __syncthreads();
    bitrev_lines(xl, kFftLines, K, 1, false, K, logK);
    fft_lines(xl, kFftLines, K, 1, false, K, logK, tw, 1);
    for (int e = threadIdx.x; e < kFftLines * K; e += kEwThreads) {
        const int l = e % kFftLines, x = e / kFftLines;
        data[x * K2 + l] = xl[l * K + x];
    }
    __shared__ double red[kEwThreads / 64];
    en = wave_sum(en);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = en;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kEwThreads / 64; ++k) t += red[k];
        a.e_recip_part[blockIdx.x] = 0.5 * kCoulombKcal * t;
    }
}

// ---- real space ---------------------------------------------------------------
// Workgroup = (64-particle i-tile, kEwChunk-particle j-chunk) of one system;
// wave w takes j-slots [w, w + 4, ...) of the chunk against its lane's i.
// Partial forces go to part[chunk][i]; the gather sums the chunks in order.
__device__ void real_space(const EwaldLaunch &a, const RealItem &it, int slot)
{
    const SysDev &S = a.sys[it.sys];
    const int lane = threadIdx.x & 63, wv = (int)threadIdx.x >> 6;
    const int i = it.i0 + lane;
    const bool vi = lane < it.ni;
    __shared__ double sx[kEwChunk], sy[kEwChunk], sz[kEwChunk], sq[kEwChunk];
    __shared__ int sm[kEwChunk];
    for (int t = threadIdx.x; t < it.nj; t += kEwThreads) {
        const int j = it.j0 + t;
        sx[t] = a.cpos[3LL * j];
        sy[t] = a.cpos[3LL * j + 1];
        sz[t] = a.cpos[3LL * j + 2];
        sq[t] = a.z[j];
        sm[t] = a.mol[j];
    }
    double xi = 0, yi = 0, zi = 0, qi = 0;
    int mi = -1;
    if (vi) {
        xi = a.cpos[3LL * i];
        yi = a.cpos[3LL * i + 1];
        zi = a.cpos[3LL * i + 2];
        qi = a.z[i];
        mi = a.mol[i];
    }
    __syncthreads();
    const double alpha = a.alpha, rc2 = a.r_cut * a.r_cut;
    const double two_a_rpi = 2.0 * alpha / sqrt(kPi);
    double fx = 0, fy = 0, fz = 0, e = 0;
    if (vi && qi != 0.0) {
        // wave wv takes j = wv, wv + 4, ...  A distance pass marks, in bit k
        // of a per-lane mask, the k-th of them that interacts (inside r_cut,
        // or of the same molecule: the erf correction); then each lane
        // evaluates only its marked pairs, in the same order, so the lanes
        // no longer all run erfc for every j while a fifth of them need it.
        constexpr int NW = kEwThreads / 64;
        static_assert(kEwChunk / NW <= 32, "one 32-bit mask per lane");
        const int nk = (it.nj - wv + NW - 1) / NW;
        auto sep = [&](int t, double &dx, double &dy, double &dz) {
            dx = xi - sx[t];
            dy = yi - sy[t];
            dz = zi - sz[t];
            dx -= S.box[0] * rint(dx * S.ibox[0]);
            dy -= S.box[1] * rint(dy * S.ibox[1]);
            dz -= S.box[2] * rint(dz * S.ibox[2]);
            return dx * dx + dy * dy + dz * dz;
        };
        unsigned m = 0;
        for (int k = 0; k < nk; ++k) {
            const int t = wv + NW * k;
            double dx, dy, dz;
            const double r2 = sep(t, dx, dy, dz);
            const bool on = (qi * sq[t] != 0.0) & (it.j0 + t != i) & ((sm[t] == mi) | (r2 < rc2));
            m |= on ? (1u << k) : 0u;
        }
        while (m != 0) {
            const int t = wv + NW * __builtin_ctz(m);
            m &= m - 1;
            const double qq = qi * sq[t];
            double dx, dy, dz;
            const double r2 = sep(t, dx, dy, dz);
            const bool excl = sm[t] == mi;
            const double r = sqrt(r2);
            const double ir = 1.0 / r;
            const double gauss = two_a_rpi * exp(-alpha * alpha * r2);
            double v, g;
            if (excl) {
                const double ef = erf(alpha * r);
                v = -ef * ir;
                g = kCoulombKcal * qq * (gauss * r - ef) * (ir * ir * ir);
            } else {
                const double ec = erfc(alpha * r);
                v = ec * ir;
                g = kCoulombKcal * qq * (gauss * r + ec) * (ir * ir * ir);
            }
            e += 0.5 * kCoulombKcal * qq * v;
            fx += g * dx;
            fy += g * dy;
            fz += g * dz;
        }
    }
    // the four waves' partial forces in a fixed order
    __shared__ double pf[kEwThreads / 64 - 1][64][3];
    if (wv > 0) {
        pf[wv - 1][lane][0] = fx;
        pf[wv - 1][lane][1] = fy;
        pf[wv - 1][lane][2] = fz;
    }
    __shared__ double red[kEwThreads / 64];
    e = wave_sum(e);
    if (lane == 0) red[wv] = e;
    __syncthreads();
    if (wv == 0) {
        for (int w = 0; w < kEwThreads / 64 - 1; ++w) {
            fx += pf[w][lane][0];
            fy += pf[w][lane][1];
            fz += pf[w][lane][2];
        }
        if (vi) {
            double *dst = a.freal + ((long long)it.chunk * a.n_part + i) * 3;
            dst[0] = fx;
            dst[1] = fy;
            dst[2] = fz;
        }
        if (lane == 0) {
            double t = 0.0;
            for (int k = 0; k < kEwThreads / 64; ++k) t += red[k];
            a.e_real_part[slot] = t;
        }
    }
}

// ---- force gather and bead forces ---------------------------------------------
__device__ void reduce_energies(const EwaldLaunch &a, int s);

template <int P>
__global__ __launch_bounds__(kEwThreads) void k_ew_gather(EwaldLaunch a)
{
    const int per = kEwThreads / 64;
    const int pblocks = (a.n_part + per - 1) / per;
    if ((int)blockIdx.x >= pblocks) {
        if (threadIdx.x < 64) reduce_energies(a, blockIdx.x - pblocks);
        return;
    }
    const int i = blockIdx.x * per + ((int)threadIdx.x >> 6);
    if (i >= a.n_part) return;
    const int lane = threadIdx.x & 63;
    const PartDev pd = a.parts[i];
    const double z = a.z[i];
    // real-space chunk partials: lane c takes chunks c, c + 64, ...; the
    // wave tree then adds the lanes in a fixed order
    double F[3] = {0.0, 0.0, 0.0};
    const int ns = a.sys_part[pd.sys + 1] - a.sys_part[pd.sys];
    const int nch = (ns + kEwChunk - 1) / kEwChunk;
    for (int c = lane; c < nch; c += 64) {
        const double *src = a.freal + ((long long)c * a.n_part + i) * 3;
        F[0] += src[0];
        F[1] += src[1];
        F[2] += src[2];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) F[k] = wave_sum(F[k]);
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
    if (a.f || a.rowf) {
        const double inv = 1.0 / pd.nb;
        for (int j = lane; j < pd.nb; j += 64) {
            const long long r = pd.row0 + (long long)j * pd.stride;
            if (a.f) {
                a.f[3 * r] += F[0] * inv;
                a.f[3 * r + 1] += F[1] * inv;
                a.f[3 * r + 2] += F[2] * inv;
            } else {
                a.rowf[3 * r] = F[0] * inv;
                a.rowf[3 * r + 1] = F[1] * inv;
                a.rowf[3 * r + 2] = F[2] * inv;
            }
        }
    }
}

// ---- per-system energies (first wave of an extra gather workgroup) --------------
__device__ void reduce_energies(const EwaldLaunch &a, int s)
{
    const int lane = threadIdx.x;
    double er = 0.0, ek = 0.0;
    for (int k = a.real_first[s] + lane; k < a.real_first[s + 1]; k += 64) er += a.e_real_part[k];
    for (int k = lane; k < a.recip_wg; k += 64) ek += a.e_recip_part[(long long)s * a.recip_wg + k];
    er = wave_sum(er);
    ek = wave_sum(ek);
    if (lane == 0 && a.e_out) {
        a.e_out[3 * s] = er;
        a.e_out[3 * s + 1] = ek;
        a.e_out[3 * s + 2] = a.e_const[s];
    }
    if (a.eslot_out && lane < A_N) {
        // the system's energy slot: the whole Ewald energy as Coulomb energy
        a.eslot_out[(long long)s * A_N + lane] = lane == A_COUL ? er + ek + a.e_const[s] : 0.0;
    }
}

template <int P>
void launch_order(const EwaldLaunch &a, hipStream_t st)
{
    const int per = kEwThreads / 64;
    const int pblocks = (a.n_part + per - 1) / per;
    const int K = a.K;
    hipLaunchKernelGGL(k_ew_prep<P>, dim3(pblocks), dim3(kEwThreads), 0, st, a);
    // the plane plus (when it stays within 64 KB) the twiddle table
    EwaldLaunch b = a;
    size_t plane_lds = sizeof(double2) * K * K;
    b.tw_in_lds = plane_lds + sizeof(double2) * (K / 2) <= 65536 ? 1 : 0;
    if (b.tw_in_lds) plane_lds += sizeof(double2) * (K / 2);
    // few planes (one system): 1024 threads each, so that spreading and the
    // plane FFTs use more of the chip; many planes: 256
    const bool wide = a.n_sys * K < 1024;
    if (wide)
        hipLaunchKernelGGL((k_ew_plane<P, 1024>), dim3(a.n_sys * K), dim3(1024), plane_lds, st, b, -1);
    else
        hipLaunchKernelGGL((k_ew_plane<P, kEwThreads>), dim3(a.n_sys * K), dim3(kEwThreads), plane_lds, st, b, -1);
    const int xgroups = a.n_sys * (K * K / kFftLines);
    hipLaunchKernelGGL(k_ew_xline, dim3(xgroups + a.n_real), dim3(kEwThreads),
                       sizeof(double2) * (kFftLines * K + K / 2), st, a);
    if (wide)
        hipLaunchKernelGGL((k_ew_plane<P, 1024>), dim3(a.n_sys * K), dim3(1024), plane_lds, st, b, 1);
    else
        hipLaunchKernelGGL((k_ew_plane<P, kEwThreads>), dim3(a.n_sys * K), dim3(kEwThreads), plane_lds, st, b, 1);
    hipLaunchKernelGGL(k_ew_gather<P>, dim3(pblocks + a.n_sys), dim3(kEwThreads), 0, st, a);
}

}  // namespace

void launch_ewald(const EwaldLaunch &a, hipStream_t st)
{
    if (a.n_part <= 0) return;
    switch (a.order) {
    case 4: launch_order<4>(a, st); break;
    case 6: launch_order<6>(a, st); break;
    default: launch_order<8>(a, st); break;
    }
}

}  // namespace mixpi
