// Free ring polymers in normal modes (arXiv 2411.11988, Sec. "Evaluation":
// the free ring-polymer part of the split propagator is integrated exactly
// in the ring-polymer normal modes; Eq. mts-hamiltonian-b gives each
// particle its own bead count N_i and spring constant N_i m_i/(beta hbar)^2).
//
// One launch processes every group of every system:
//   * groups with N <= 64: "dense" items.  A workgroup holds 256/N columns
//     (particle x Cartesian component) of the [N][n][3] block in LDS with the
//     orthonormal basis C and C^T; thread (column, mode) forms the mode,
//     propagates it, and thread (column, bead) transforms back.  Global
//     loads and stores run column-fastest (coalesced).
//   * groups with N > 64 (a many-bead electron): one workgroup per column,
//     a radix-2 FP64 FFT in LDS.  q and p are packed as one complex signal
//     q + i p; the real basis C follows from the FFT of a real signal
//     (mode 0 and N/2 from the real parts, cos mode m from Re Z_m, sin mode
//     N - m from Im Z_m, scaled by sqrt(2/N)), so the result equals the dense
//     transform up to rounding with O(N log N) work instead of O(N^2).
//
//   * rings with N > 64 and few columns (up to a work budget): in the step,
//     "circulant" items that propagate in bead space (rp_circ below) with
//     many workgroups per column; the transforms still use the FFT items.
//
// OP_STEP fuses: first half-kick p += dt/2 F on load, forward transform,
// exact propagation of every mode with tabulated coefficients
// (xi, pi) <- (a xi + b pi, c xi + d pi), spring energy sum_k k lambda_k/2
// xi_k^2 and the centroid of the new positions (mode 0 / sqrt N, stored for
// every bead row), backward transform, store of q and p, and zeroing of F for
// the force accumulation that follows.
#include <type_traits>

#include "device_common.h"
#include "mixpi_internal.h"

namespace mixpi {

__device__ __forceinline__ double bsum256(double v, double *red)
{
    v = wsum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    return s;
}

// Global -> LDS copy of n elements; thread t takes t, t + 256, ...  The
// loads of U consecutive rounds are issued before their LDS stores, so a
// thread waits on memory once per U rounds instead of once per element
// (a plain copy loop waits for each load before its store).
template <int U, typename Get, typename Put>
__device__ __forceinline__ void lds_fill(int n, Get get, Put put)
{
    using T = decltype(get(0));
    for (int b = threadIdx.x; b < n; b += U * 256) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (b + u * 256 < n) v[u] = get(b + u * 256);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (b + u * 256 < n) put(b + u * 256, v[u]);
    }
}

__device__ void rp_dense(const RpLaunch &a, const RpItem &it, double *smem, double *red)
{
    const int N = it.N, n = it.n;
    const int CB = 256 / N;
    const int tid = threadIdx.x;
    double *sC = smem;              // C[j*N + k]
    double *sCT = sC + N * N;       // C^T[k*N + j]
    double *s0 = sCT + N * N;       // [N][CB]
    double *s1 = s0 + 256;
    double *s2 = s1 + 256;
    double *s3 = s2 + 256;
    const double *Cg = a.basis + it.basis_off;
    const double hk = a.sys[it.sys].hkick;
    {   // stage: column fastest; the state loads go out before the basis
        const int r = tid / CB, cl = tid % CB;
        double v0 = 0.0, v1 = 0.0;
        if (cl < it.ncols) {
            const long long g = (it.row + (long long)r * n) * 3 + it.c0 + cl;
            v0 = a.in_q[g];
            if (a.op == OP_STEP) v1 = a.p[g] + hk * a.f[g];
        }
        lds_fill<8>(2 * N * N, [&](int x) { return Cg[x]; }, [&](int x, double v) { sC[x] = v; });
        if (a.op == OP_BWD) s2[r * CB + cl] = v0;
        else { s0[r * CB + cl] = v0; s1[r * CB + cl] = v1; }
    }
    __syncthreads();

    const int cl = tid % CB, k = tid / CB;
    const bool valid = cl < it.ncols;
    const int c = it.c0 + cl;
    double esp = 0.0;
    if (a.op != OP_BWD) {
        double xi = 0.0, pi = 0.0;
        for (int j = 0; j < N; ++j) {
            const double cjk = sC[j * N + k];
            xi += cjk * s0[j * CB + cl];
            pi += cjk * s1[j * CB + cl];
        }
        if (a.op == OP_FWD) {
            if (valid) a.out_q[(it.row + (long long)k * n) * 3 + c] = xi;
            return;
        }
        if (valid) {
            const int i = c / 3;
            const double *pr = a.prop + 5 * (it.row + (long long)k * n + i);
            const double x2 = pr[0] * xi + pr[1] * pi;
            const double p2 = pr[2] * xi + pr[3] * pi;
            xi = x2;
            pi = p2;
            esp = pr[4] * x2 * x2;
        }
        s2[k * CB + cl] = xi;
        s3[k * CB + cl] = pi;
        __syncthreads();
    }
    // backward: thread (column, bead j = k)
    const int j = k;
    double qn = 0.0, pn = 0.0;
    for (int m = 0; m < N; ++m) {
        const double cjm = sCT[m * N + j];
        qn += cjm * s2[m * CB + cl];
        if (a.op == OP_STEP) pn += cjm * s3[m * CB + cl];
    }
    if (valid) {
        const long long g = (it.row + (long long)j * n) * 3 + c;
        a.out_q[g] = qn;
        if (a.op == OP_STEP) {
            a.p[g] = pn;
            a.cent[g] = s2[cl] / sqrt((double)N);   // propagated mode 0 / sqrt(N)
        }
    }
    if (a.op == OP_STEP) {
        const double s = bsum256(esp, red);
        if (tid == 0) {
            double *e = a.eslot + (long long)blockIdx.x * A_N;
            for (int k = 0; k < A_N; ++k) e[k] = 0.0;
            e[A_SPRING] = s;
        }
    }
}

__device__ __forceinline__ double2 cmul(double2 x, double2 y)
{
    return make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
}

// In-place decimation-in-time FFT (exp(-2 pi i jk/N)) of a bit-reversed
// input held in LDS.  Radix-2 stages are fused into passes over LDS: a
// radix-4 pass (each thread loads 4 points, applies stages s and s+1 in
// registers, stores 4 points) or, where N/8 still gives every thread of the
// workgroup a group (N >= 2048 at 256 threads), a radix-8 pass over stages
// s..s+2.  Leading stages that the pass width does not divide form one
// radix-2 or radix-4 pass.  Fewer passes mean fewer LDS round trips and
// barriers; below that size the radix-8 pass leaves threads idle and ran
// slower.  R8 = false keeps radix-4 passes at every size: the Langevin items
// use it, since radix-8 code there raised the launch's register count (152
// to 169 VGPRs) and slowed the thermostatted step.  Twiddles are stage-major
// (stage s at offset 2^(s-1) - 1, entries exp(-2 pi i pos / 2^s)), so the
// lanes of a pass read consecutive entries.
__device__ __forceinline__ void bfly(double2 &a, double2 &b, double2 w)
{
    const double2 t = cmul(b, w);
    b = make_double2(a.x - t.x, a.y - t.y);
    a = make_double2(a.x + t.x, a.y + t.y);
}

// stages s and s+1 (half-lengths h and 2h)
__device__ __forceinline__ void fft_pass4(double2 *z, const double2 *tw, int N, int s)
{
    const int h = 1 << (s - 1);
    __syncthreads();
    for (int b = threadIdx.x; b < N / 4; b += blockDim.x) {
        const int pos = b & (h - 1);
        const int i0 = ((b >> (s - 1)) << (s + 1)) + pos;
        double2 x0 = z[i0], x1 = z[i0 + h], x2 = z[i0 + 2 * h], x3 = z[i0 + 3 * h];
        const double2 w1 = tw[h - 1 + pos];                  // stage s
        bfly(x0, x1, w1);
        bfly(x2, x3, w1);
        bfly(x0, x2, tw[2 * h - 1 + pos]);                   // stage s+1
        bfly(x1, x3, tw[2 * h - 1 + pos + h]);
        z[i0] = x0;
        z[i0 + h] = x1;
        z[i0 + 2 * h] = x2;
        z[i0 + 3 * h] = x3;
    }
}

// stages s, s+1 and s+2
__device__ __forceinline__ void fft_pass8(double2 *z, const double2 *tw, int N, int s)
{
    const int h = 1 << (s - 1);
    __syncthreads();
    for (int b = threadIdx.x; b < N / 8; b += blockDim.x) {
        const int pos = b & (h - 1);
        const int i0 = ((b >> (s - 1)) << (s + 2)) + pos;
        double2 x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = z[i0 + k * h];
        const double2 w1 = tw[h - 1 + pos];                  // stage s
        bfly(x[0], x[1], w1);
        bfly(x[2], x[3], w1);
        bfly(x[4], x[5], w1);
        bfly(x[6], x[7], w1);
        const double2 u0 = tw[2 * h - 1 + pos], u1 = tw[2 * h - 1 + pos + h];
        bfly(x[0], x[2], u0);                                // stage s+1
        bfly(x[1], x[3], u1);
        bfly(x[4], x[6], u0);
        bfly(x[5], x[7], u1);
#pragma unroll
        for (int j = 0; j < 4; ++j) bfly(x[j], x[j + 4], tw[4 * h - 1 + pos + j * h]);  // stage s+2
#pragma unroll
        for (int k = 0; k < 8; ++k) z[i0 + k * h] = x[k];
    }
}

template <bool R8>
__device__ void fft_stages(double2 *z, const double2 *tw, int N, int L)
{
    const int r = R8 && N >= 8 * (int)blockDim.x ? 3 : 2;
    int s = 1;
    const int lead = L % r;
    if (lead == 1) {
        __syncthreads();
        for (int b = threadIdx.x; b < N / 2; b += blockDim.x) {
            const double2 u = z[2 * b], v = z[2 * b + 1];
            z[2 * b] = make_double2(u.x + v.x, u.y + v.y);
            z[2 * b + 1] = make_double2(u.x - v.x, u.y - v.y);
        }
        s = 2;
    } else if (lead == 2) {
        fft_pass4(z, tw, N, 1);
        s = 3;
    }
    for (; s < L; s += r) {
        if (r == 3) fft_pass8(z, tw, N, s);
        else fft_pass4(z, tw, N, s);
    }
    __syncthreads();
}

__device__ __forceinline__ int brev(int j, int L) { return (int)(__brev((unsigned)j) >> (32 - L)); }

__device__ void rp_fft(const RpLaunch &a, const RpItem &it, double2 *z, double *red)
{
    const int N = it.N, L = it.logN, n = it.n;
    const int col = it.c0, i = col / 3;
    // stage-major twiddles (N - 1 entries) staged in LDS behind the signal
    double2 *tw = z + N;
    const double2 *twg = a.twiddle + it.tw_off;
    const int tid = threadIdx.x;
    const double rN = sqrt((double)N), r2N = sqrt(2.0 / N), rN2 = sqrt(0.5 * N);
    const double hk = a.sys[it.sys].hkick;
    auto gaddr = [&](int j) { return (it.row + (long long)j * n) * 3 + col; };

    if (a.op == OP_BWD) {
        lds_fill<4>(N - 1, [&](int m) { return twg[m]; }, [&](int m, double2 v) { tw[m] = v; });
        // modes -> Hermitian spectrum Z; load conj(Z) in bit-reversed order
        auto lone = [&](int m) { return m == 0 || 2 * m == N; };
        lds_fill<4>(
            N / 2 + 1,
            [&](int m) {
                return make_double2(a.in_q[gaddr(m)], lone(m) ? 0.0 : a.in_q[gaddr(N - m)]);
            },
            [&](int m, double2 x) {
                if (lone(m)) {
                    z[brev(m, L)] = make_double2(rN * x.x, 0.0);
                } else {
                    // Z_m = sqrt(N/2) (xi_m + i xi_{N-m}), Z_{N-m} = conj(Z_m)
                    z[brev(m, L)] = make_double2(rN2 * x.x, -rN2 * x.y);       // conj(Z_m)
                    z[brev(N - m, L)] = make_double2(rN2 * x.x, rN2 * x.y);    // conj(Z_{N-m})
                }
            });
        fft_stages<true>(z, tw, N, L);
        for (int j = tid; j < N; j += blockDim.x) a.out_q[gaddr(j)] = z[j].x / N;
        return;
    }

    // modes m and N - m share lambda_m, hence one coefficient set; the
    // first two sets of this thread are fetched before the transform
    const double *prop = a.prop;
    auto prow = [&](int k) { return prop + 5 * (it.row + (long long)k * n + i); };
    double pre[2][5];
    if (a.op == OP_STEP)
        for (int r = 0; r < 2; ++r) {
            const int m = tid + r * (int)blockDim.x;
            for (int c = 0; c < 5; ++c) pre[r][c] = m <= N / 2 ? prow(m)[c] : 0.0;
        }
    // the signal and the twiddles in one fill: one wait on memory per 4 rounds
    struct In {
        double2 z, t;
    };
    lds_fill<4>(
        N,
        [&](int j) {
            const long long g = gaddr(j);
            In v;
            v.z = make_double2(a.in_q[g], a.op == OP_STEP ? a.p[g] + hk * a.f[g] : 0.0);
            v.t = j < N - 1 ? twg[j] : make_double2(0.0, 0.0);
            return v;
        },
        [&](int j, const In &v) {
            z[brev(j, L)] = v.z;
            if (j < N - 1) tw[j] = v.t;
        });
    fft_stages<true>(z, tw, N, L);

    if (a.op == OP_FWD) {
        for (int m = tid; m <= N / 2; m += blockDim.x) {
            const double2 Z = z[m];
            if (m == 0 || 2 * m == N) {
                a.out_q[gaddr(m)] = Z.x / rN;
            } else {
                a.out_q[gaddr(m)] = r2N * Z.x;
                a.out_q[gaddr(N - m)] = r2N * Z.y;
            }
        }
        return;
    }

    // OP_STEP: unpack q and p modes, propagate, repack z = Zq' + i Zp'
    double esp = 0.0;
    __shared__ double cent_s;
    for (int m = tid, r = 0; m <= N / 2; m += blockDim.x, ++r) {
        double pc[5];
        for (int c = 0; c < 5; ++c) pc[c] = r < 2 ? pre[r][c] : prow(m)[c];
        const double2 Zm = z[m];
        const double2 Zc = make_double2(z[(N - m) & (N - 1)].x, -z[(N - m) & (N - 1)].y);
        const double Qr = 0.5 * (Zm.x + Zc.x), Qi = 0.5 * (Zm.y + Zc.y);
        const double Dr = Zm.x - Zc.x, Di = Zm.y - Zc.y;
        const double Pr = 0.5 * Di, Pi = -0.5 * Dr;        // (Zm - Zc) / (2i)
        if (m == 0 || 2 * m == N) {
            const double x = Qr / rN, y = Pr / rN;
            const double x2 = pc[0] * x + pc[1] * y, y2 = pc[2] * x + pc[3] * y;
            esp += pc[4] * x2 * x2;
            if (m == 0) cent_s = x2 / rN;
            z[m] = make_double2(rN * x2, rN * y2);
        } else {
            const double x1 = r2N * Qr, x2 = r2N * Qi;
            const double y1 = r2N * Pr, y2 = r2N * Pi;
            const double x1n = pc[0] * x1 + pc[1] * y1, y1n = pc[2] * x1 + pc[3] * y1;
            const double x2n = pc[0] * x2 + pc[1] * y2, y2n = pc[2] * x2 + pc[3] * y2;
            esp += pc[4] * (x1n * x1n + x2n * x2n);
            // Zq' = sqrt(N/2) (x1 + i x2), Zp' = sqrt(N/2) (y1 + i y2); z = Zq' + i Zp'
            z[m] = make_double2(rN2 * (x1n - y2n), rN2 * (x2n + y1n));
            z[N - m] = make_double2(rN2 * (x1n + y2n), rN2 * (y1n - x2n));
        }
    }
    __syncthreads();
    // inverse transform as conj(FFT(conj(z))) / N: conjugate and bit-reverse
    for (int j = tid; j < N; j += blockDim.x) {
        const int r = brev(j, L);
        if (j < r) {
            const double2 u = z[j], v = z[r];
            z[j] = make_double2(v.x, -v.y);
            z[r] = make_double2(u.x, -u.y);
        } else if (j == r) {
            z[j].y = -z[j].y;
        }
    }
    fft_stages<true>(z, tw, N, L);
    const double iN = 1.0 / N;
    const double cq = cent_s;
    for (int j = tid; j < N; j += blockDim.x) {
        const long long g = gaddr(j);
        a.out_q[g] = z[j].x * iN;
        a.p[g] = -z[j].y * iN;
        a.cent[g] = cq;
    }
    const double s = bsum256(esp, red);
    if (tid == 0) {
        double *e = a.eslot + (long long)blockIdx.x * A_N;
        for (int k = 0; k < A_N; ++k) e[k] = 0.0;
        e[A_SPRING] = s;
    }
}

// Free ring-polymer step in bead space for a many-bead ring with few
// columns.  The exact free propagator C diag(f_k) C^T of each of the maps
// (q <- a q + b p, p <- c q + a p) depends on the bead index only through
// j - j' (every f_k depends on lambda_k, shared by modes k and N - k), so
// it is circulant: a_d = (1/N) sum_k f_k cos(2 pi k d / N), tabulated per
// particle on the host.  An item computes kCircOut consecutive bead outputs
// of one column from the whole ring: the centroid parts move exactly
// (q_bar' = q_bar + dt/m_f p_bar, p_bar' = p_bar, as sum_d a_d = 1,
// sum_d b_d = dt/m_f, sum_d c_d = 0), the rest is the convolution of the
// centroid-free ring with a, b, c.
//
// Inputs (q and the half-kicked p) come from the ring's stage rows, since
// the items of a column write q and p in place.  All global loads of a
// thread are issued before its first LDS store.  Thread (og, jg) sums 4
// consecutive outputs over a contiguous 1/64 of the ring, sliding its
// coefficient window by one bead per step; wave og holds the 64 j-groups of
// one output group.  LDS rows are padded by one double per 1/64 of the ring,
// so a wave's 64 bead reads and its 64 coefficient reads are 17 doubles
// apart (distinct banks); the 64 j-group sums of each output are then a
// wave sum, with no LDS round trip.
// The spring energy of the item's bead steps (j, j+1) needs the output
// after the item; it is the dot product of raw (q, p) with the coefficients
// minus the centroid parts, accumulated with the loads.
__device__ void rp_circ(const RpLaunch &a, const RpItem &it, double *smem, double *red)
{
    const int N = it.N, n = it.n, L = it.logN;
    const int col = it.c0, i = col / 3, d = col - 3 * i;
    const int tid = threadIdx.x;
    const int lpad = L - 6;                      // one pad double per N/64 (a j-group)
    const int CS = N + 64;                       // row stride: q, p, a, b, c rows (N + pad)
    auto pad = [&](int x) { return x + (x >> lpad); };
    double *sq = smem, *sp = sq + CS, *ca = sp + CS, *cb = ca + CS, *cc = cb + CS;
    __shared__ double s_sum[3][4];
    __shared__ double s_out[kCircOut + 1];
    const double *coef = a.circ + it.circ_off;
    const int inext = (it.o0 + kCircOut) & (N - 1);

    // loads: up to kCircMaxN / 256 beads per thread, all issued first
    constexpr int KB = kCircMaxN / 256;
    double vq[KB], vp[KB], va[KB], vb[KB], vc[KB], na[KB], nb[KB];
    const int per = N >> 8;
#pragma unroll
    for (int u = 0; u < KB; ++u)
        if (u < per) {
            const int j = tid + (u << 8);
            const double *sr = a.stage + 6LL * (it.stage0 + (long long)j * n + i);
            vq[u] = sr[d];
            vp[u] = sr[3 + d];
            va[u] = coef[j];
            vb[u] = coef[N + j];
            vc[u] = coef[2 * N + j];
            const int jn = (inext - j) & (N - 1);
            na[u] = coef[jn];
            nb[u] = coef[N + jn];
        }
    double sum_q = 0.0, sum_p = 0.0, nx = 0.0;
#pragma unroll
    for (int u = 0; u < KB; ++u)
        if (u < per) {
            const int x = pad(tid + (u << 8));
            sq[x] = vq[u];
            sp[x] = vp[u];
            ca[x] = va[u];
            cb[x] = vb[u];
            cc[x] = vc[u];
            sum_q += vq[u];
            sum_p += vp[u];
            nx += na[u] * vq[u] + nb[u] * vp[u];
        }
    // one block reduction of the three sums
    sum_q = wsum(sum_q);
    sum_p = wsum(sum_p);
    nx = wsum(nx);
    if ((tid & 63) == 0) {
        s_sum[0][tid >> 6] = sum_q;
        s_sum[1][tid >> 6] = sum_p;
        s_sum[2][tid >> 6] = nx;
    }
    __syncthreads();
    const double qbar = (s_sum[0][0] + s_sum[0][1] + s_sum[0][2] + s_sum[0][3]) / N;
    const double pbar = (s_sum[1][0] + s_sum[1][1] + s_sum[1][2] + s_sum[1][3]) / N;
    const double dtm = a.prop[5 * (it.row + i) + 1];   // mode 0: dt / m_f
    const double qc = qbar + dtm * pbar;               // new centroid
#pragma unroll
    for (int u = 0; u < KB; ++u)
        if (u < per) {
            const int x = pad(tid + (u << 8));
            sq[x] = vq[u] - qbar;
            sp[x] = vp[u] - pbar;
        }
    __syncthreads();

    // thread (og, jg): outputs o0 + 4 og + r, beads jg*seg .. jg*seg + seg - 1
    static_assert(kCircOut / 4 * kCircJg == 256, "one wave per output group");
    const int og = tid / kCircJg, jg = tid % kCircJg;
    const int seg = N / kCircJg;
    const int i0 = it.o0 + 4 * og;
    const int jb = jg * seg;
    double wa[4], wb[4], wc[4], dq[4], dp[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int x = pad((i0 + r - jb) & (N - 1));
        wa[r] = ca[x];
        wb[r] = cb[x];
        wc[r] = cc[x];
        dq[r] = 0.0;
        dp[r] = 0.0;
    }
    // this thread's beads lie in one pad segment: pad(j) = j + jg
    const double *qrow = sq + jb + jg;
    int dn = (i0 - jb - 1) & (N - 1);            // next coefficient index
#pragma unroll 8
    for (int t = 0; t < seg; ++t) {
        const double qj = qrow[t], pj = qrow[t + CS];
        const int x = dn + (dn >> lpad);
        const double na0 = ca[x], nb0 = ca[x + CS], nc0 = ca[x + 2 * CS];
        dn = (dn - 1) & (N - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            dq[r] = fma(wa[r], qj, dq[r]);
            dq[r] = fma(wb[r], pj, dq[r]);
            dp[r] = fma(wc[r], qj, dp[r]);
            dp[r] = fma(wa[r], pj, dp[r]);
        }
#pragma unroll
        for (int r = 3; r > 0; --r) {
            wa[r] = wa[r - 1];
            wb[r] = wb[r - 1];
            wc[r] = wc[r - 1];
        }
        wa[0] = na0;
        wb[0] = nb0;
        wc[0] = nc0;
    }
    // the j-groups of output group og are the lanes of wave og: eight wave
    // sums (fixed order) give its four outputs
    double oq[4], op[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        oq[r] = wsum(dq[r]);
        op[r] = wsum(dp[r]);
    }
    const int lane = tid & 63;
    if (lane < 4) {
        double vq2 = oq[0], vp2 = op[0];
#pragma unroll
        for (int r = 1; r < 4; ++r) {
            vq2 = lane == r ? oq[r] : vq2;
            vp2 = lane == r ? op[r] : vp2;
        }
        const int o = 4 * og + lane;
        s_out[o] = vq2;
        const long long gq = (it.row + (long long)(it.o0 + o) * n) * 3 + col;
        a.out_q[gq] = qc + vq2;
        a.p[gq] = pbar + vp2;
        a.cent[gq] = qc;
    }
    if (tid == 0) {
        // the centroid-free part of the output after the item
        const double nraw = s_sum[2][0] + s_sum[2][1] + s_sum[2][2] + s_sum[2][3];
        s_out[kCircOut] = nraw - qc;
    }
    __syncthreads();
    // the spring energy of the item's bead steps, by the first wave
    if (tid >= 64) return;
    double esp = 0.0;
    if (tid < kCircOut) {
        const double dlt = s_out[tid] - s_out[tid + 1];
        esp = it.wsp * dlt * dlt;
    }
    esp = wsum(esp);
    if (tid == 0) {
        double *e = a.eslot + (long long)blockIdx.x * A_N;
        for (int k = 0; k < A_N; ++k) e[k] = 0.0;
        e[A_SPRING] = esp;
    }
}

// ---------------------------------------------------------------------------
// Matrix-core (MFMA) items.  A ring's exact free propagator and its normal-
// mode transform are dense N x N matrices applied to the ring's columns:
//   transform (mixpi_nm_transform): xi = C^T x and x = C xi with the
//     orthonormal basis C, generated from a table of cos(2 pi m / N) at
//     m = (j k) mod N (a sine mode at m - N/4);
//   step: q' = a * q + b * p, p' = c * q + a * p with the circulant rows
//     a_d, b_d, c_d of the propagator C diag(f) C^T (see rp_circ), generated
//     at d = (j - j') mod N; the transform, the per-mode propagation and the
//     back transform in one product, with nothing in between to keep.
// One item: 16 output rows of up to 16 columns that share the matrix (the
// columns of every ring of one propagator class, across the systems of a
// batch), so one 16x16x4 matrix instruction covers every column.  The four
// waves each take a quarter of the K range (beads) and add their 16x16
// results in LDS in a fixed order.  The step uses FP64 matrix instructions
// in both forms: FP32 ones drift the conserved energy.  Transforms: FP64 in
// the FP64 form; in the FP32 form FP32 matrix instructions on columns
// shifted by their bead 0 (restored in FP64; a transform's mode 0 in FP64),
// FP32 sums over 64 beads added into FP64 accumulators.  The shift is exact
// algebra for the step too (the matrices' row sums are exact: sum a = 1,
// sum b = dt/m_f, sum c = 0), so both forms share the code.
typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));
template <typename T> struct Mfma;
template <> struct Mfma<double> {
    using V = mf_d4;
    static __device__ __forceinline__ V mma(double x, double y, V c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
    }
    // A: lane l holds A[l % 16][l / 16]; B: lane l holds B[l / 16][l % 16];
    // result register r of lane l holds row (l / 16) + 4 r, column l % 16
    static __device__ __forceinline__ int row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
    using V = mf_f4;
    static __device__ __forceinline__ V mma(float x, float y, V c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
    }
    // as above, but result register r of lane l holds row 4 (l / 16) + r
    static __device__ __forceinline__ int row(int l, int r) { return 4 * (l >> 4) + r; }
};

template <typename T>
__device__ void rp_mfma(const RpLaunch &a, const RpItem &it, double *smem)
{
    using M = Mfma<T>;
    using V = typename M::V;
    const int N = it.N, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const bool prop = a.op == OP_STEP, bwd = a.op == OP_BWD;
    constexpr int tprec = std::is_same<T, float>::value ? 1 : 0;   // table layout of T
    T *tab = reinterpret_cast<T *>(smem);
    double *red = smem + mfma_tab_doubles(N, a.op, tprec);
    double *csum = red + 4 * 2 * 4 * 64;
    const int ntab = (prop ? 3 : 1) * N;
    const double *tg = a.mf_tab + it.circ_off;
    lds_fill<8>(ntab, [&](int x) { return tg[x]; }, [&](int x, double v) { tab[x] = (T)v; });

    // this lane's column (l % 16) and its reference values (bead 0)
    const int c = lane & 15;
    const bool cv = c < it.ncols;
    const MfmaCol col = a.mf_cols[it.c0 + (cv ? c : 0)];
    const double rsN = 1.0 / sqrt((double)N), r2N = sqrt(2.0 / N);
    double ref0 = 0.0, ref1 = 0.0;
    if (cv) {
        if (prop) {
            const double *sr = a.stage + 6 * col.srow0;
            ref0 = sr[col.d];
            ref1 = sr[3 + col.d];
        } else {
            ref0 = a.in_q[3 * col.row0 + col.d];   // bead 0 (forward) or mode 0 (backward)
        }
    }
    __syncthreads();

    // the output row of this lane's A operand, and its fixed sine shift and
    // scale in the forward transform
    const int m = it.o0 + c;
    const int ph_m = 2 * m > N ? N / 4 : 0;
    const int mask = N - 1;
    V d0 = {}, d1 = {};          // q' (or the transform) and p'
    double h0[4] = {0, 0, 0, 0}, h1[4] = {0, 0, 0, 0};   // FP64 sums (FP32 form)
    double sx = 0.0, sy = 0.0;   // column sums of the shifted inputs (propagation)
    const int kq = N >> 2;       // beads of each wave
    const int kb = w * kq;
    // the loads of KU bead steps go out together, then their matrix
    // instructions (a loop that waited for each step's loads would be bound
    // by memory latency)
    constexpr int KU = 8;
    int chunk = 0;
    for (int s0 = kb; s0 < kb + kq; s0 += 4 * KU) {
        double xs[KU], ys[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int kk = s0 + 4 * u + (lane >> 4);   // this lane's bead (or mode) of the B operand
            double x = 0.0, y = 0.0;
            if (cv && kk < kb + kq) {
                if (prop) {
                    const double *sr = a.stage + 6 * (col.srow0 + (long long)kk * col.stride);
                    x = sr[col.d] - ref0;
                    y = sr[3 + col.d] - ref1;
                } else {
                    const double v = a.in_q[3 * (col.row0 + (long long)kk * col.stride) + col.d];
                    if (bwd) x = kk == 0 ? 0.0 : (2 * kk == N ? rsN : r2N) * v;
                    else x = v - ref0;
                }
            }
            xs[u] = x;
            ys[u] = y;
        }
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            const int kk = s0 + 4 * u + (lane >> 4);
            if (s0 + 4 * u >= kb + kq) break;            // wave-uniform
            const double x = xs[u], y = ys[u];
            if (prop) {
                sx += x;
                sy += y;
                const int idx = (m - kk) & mask;
                const T ga = tab[idx], gb = tab[N + idx], gc = tab[2 * N + idx];
                const T bx = (T)x, by = (T)y;
                d0 = M::mma(ga, bx, d0);
                d0 = M::mma(gb, by, d0);
                d1 = M::mma(gc, bx, d1);
                d1 = M::mma(ga, by, d1);
            } else {
                // forward: row m is the mode, kk the bead; backward: the reverse
                const int idx = bwd ? ((m * kk - (2 * kk > N ? N / 4 : 0)) & mask)
                                    : ((kk * m - ph_m) & mask);
                d0 = M::mma(tab[idx], (T)x, d0);
            }
            if constexpr (std::is_same<T, float>::value) {
                if (++chunk == 16) {     // 64 beads summed in FP32: move them to FP64
                    chunk = 0;
                    for (int r = 0; r < 4; ++r) {
                        h0[r] += (double)d0[r];
                        h1[r] += (double)d1[r];
                    }
                    d0 = V{};
                    d1 = V{};
                }
            }
        }
    }
    double o0[4], o1[4];
    for (int r = 0; r < 4; ++r) {
        o0[r] = h0[r] + (double)d0[r];
        o1[r] = h1[r] + (double)d1[r];
    }
    // the four waves' partial results and column sums, added by wave 0 in order
    for (int r = 0; r < 4; ++r) {
        red[((w * 2 + 0) * 4 + r) * 64 + lane] = o0[r];
        red[((w * 2 + 1) * 4 + r) * 64 + lane] = o1[r];
    }
    csum[(w * 2 + 0) * 64 + lane] = sx;
    csum[(w * 2 + 1) * 64 + lane] = sy;
    __syncthreads();
    if (w != 0) return;
    for (int r = 0; r < 4; ++r) {
        for (int v = 1; v < 4; ++v) {
            o0[r] += red[((v * 2 + 0) * 4 + r) * 64 + lane];
            o1[r] += red[((v * 2 + 1) * 4 + r) * 64 + lane];
        }
    }
    if (prop) {
        double tx = 0.0, ty = 0.0;
        for (int v = 0; v < 4; ++v)
            for (int g = 0; g < 4; ++g) {
                tx += csum[(v * 2 + 0) * 64 + 16 * g + c];
                ty += csum[(v * 2 + 1) * 64 + 16 * g + c];
            }
        const double pbar = ref1 + ty / N;
        const double qc = ref0 + tx / N + it.dtm * pbar;     // the propagated centroid
        const double q0 = ref0 + it.dtm * ref1;
        if (cv)
            for (int r = 0; r < 4; ++r) {
                const int mr = it.o0 + M::row(lane, r);
                const long long g = 3 * (col.row0 + (long long)mr * col.stride) + col.d;
                a.out_q[g] = q0 + o0[r];
                a.p[g] = ref1 + o1[r];
                a.cent[g] = qc;
            }
        if (lane == 0) {
            // the spring energy of these rows is summed by the epilogue
            double *e = a.eslot + (long long)blockIdx.x * A_N;
            for (int k = 0; k < A_N; ++k) e[k] = 0.0;
        }
    } else if (cv) {
        for (int r = 0; r < 4; ++r) {
            const int mr = it.o0 + M::row(lane, r);
            const long long g = 3 * (col.row0 + (long long)mr * col.stride) + col.d;
            double v = o0[r];
            if (bwd) v += ref0 * rsN;                           // mode 0
            else v = (mr == 0 || 2 * mr == N ? rsN : r2N) * v + (mr == 0 ? ref0 * sqrt((double)N) : 0.0);
            a.out_q[g] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// Path-integral Langevin thermostat (the PILE thermostat of the paper's NVT
// runs): each ring's momenta are projected onto the normal modes, every mode
// takes one or two Ornstein-Uhlenbeck half steps pi <- c1 pi + c2 eta
// (c1 = exp(-gamma_k dt/2), c2 = sqrt(1 - c1^2) sqrt(m_f k_B T), friction
// 1/tau0 on the centroid and 2 omega_k on mode k), and projected back.  The
// noise is an input, indexed by mode like the mode coordinates.  Rows of
// circulant rings also get their stage rows (q, p + dt/2 F) for the next
// step, since p changed after the epilogue wrote them.
// The thermostat terms of mode row r (coefficients and noise), and the
// stage inputs of output row `row`, are loaded before an item's transforms,
// together with its momenta, so that their memory latency is paid once.
struct OTerms {
    double c1, c2, n1, n2;
};
__device__ __forceinline__ OTerms o_load(const RpLaunch &a, long long r, int d)
{
    OTerms t;
    t.c1 = a.lang[2 * r];
    t.c2 = a.lang[2 * r + 1];
    t.n1 = a.noise1 ? a.noise1[3 * r + d] : 0.0;
    t.n2 = a.noise2 ? a.noise2[3 * r + d] : 0.0;
    return t;
}
__device__ __forceinline__ double o_apply(const RpLaunch &a, const OTerms &t, double x)
{
    if (a.noise1) x = t.c1 * x + t.c2 * t.n1;
    if (a.noise2) x = t.c1 * x + t.c2 * t.n2;
    return x;
}

struct StageTerms {
    int st;
    double q, hk, f;
};
__device__ __forceinline__ StageTerms stage_load(const RpLaunch &a, long long row, long long g)
{
    StageTerms s{a.row_stage[row], 0.0, 0.0, 0.0};
    if (s.st >= 0) {
        s.q = a.in_q[g];
        s.hk = a.row_hk[row];
        s.f = a.f[g];
    }
    return s;
}
__device__ __forceinline__ void stage_store(const RpLaunch &a, const StageTerms &s, long long g,
                                            int d, double pn)
{
    a.p[g] = pn;
    if (s.st >= 0) {
        a.stage[6LL * s.st + d] = s.q;
        a.stage[6LL * s.st + 3 + d] = pn + s.hk * s.f;
    }
}

__device__ void rp_lang_dense(const RpLaunch &a, const RpItem &it, double *smem)
{
    const int N = it.N, n = it.n;
    const int CB = 256 / N;
    const int tid = threadIdx.x;
    double *sC = smem;              // C[j*N + k]
    double *sCT = sC + N * N;       // C^T[k*N + j]
    double *s0 = sCT + N * N;       // [N][CB] momenta
    double *s2 = s0 + 256;          // [N][CB] modes
    const double *Cg = a.basis + it.basis_off;
    const int cl = tid % CB, k = tid / CB;
    const bool valid = cl < it.ncols;
    const int c = it.c0 + cl, i = c / 3, d = c - 3 * i;
    // thread (k, cl) owns mode row k and bead row k of column cl
    const long long rowk = it.row + (long long)k * n + i;
    OTerms t{};
    StageTerms sg{-1, 0.0, 0.0, 0.0};
    double p0 = 0.0;
    if (valid) {
        p0 = a.p[rowk * 3 + d];
        t = o_load(a, rowk, d);
        sg = stage_load(a, rowk, rowk * 3 + d);
    }
    lds_fill<8>(2 * N * N, [&](int x) { return Cg[x]; }, [&](int x, double v) { sC[x] = v; });
    s0[k * CB + cl] = p0;
    __syncthreads();
    double pi = 0.0;
    for (int j = 0; j < N; ++j) pi += sC[j * N + k] * s0[j * CB + cl];
    if (valid) pi = o_apply(a, t, pi);
    s2[k * CB + cl] = pi;
    __syncthreads();
    double pn = 0.0;
    for (int m = 0; m < N; ++m) pn += sCT[m * N + k] * s2[m * CB + cl];
    if (valid) stage_store(a, sg, rowk * 3 + d, d, pn);
}

constexpr int kLangKeep = (kMaxBeads / 2 + 1 + 255) / 256;
constexpr int kLangPre = 3;     // mode slots with terms prefetched (all for N <= 1024)
constexpr int kLangOutPre = 4;  // output slots with stage inputs prefetched
__device__ void rp_lang_fft(const RpLaunch &a, const RpItem &it, double2 *z)
{
    const int N = it.N, L = it.logN, n = it.n;
    const int col = it.c0, i = col / 3, d = col - 3 * i;
    double2 *tw = z + N;
    const int tid = threadIdx.x;
    const double rN = sqrt((double)N), r2N = sqrt(2.0 / N), rN2 = sqrt(0.5 * N);
    auto rowm = [&](int k) { return it.row + (long long)k * n + i; };
    // modes m and N - m of slot r share a thread; m = 0 and m = N/2 are alone
    auto lone = [&](int m) { return m == 0 || 2 * m == N; };
    OTerms ot[kLangPre][2] = {};
#pragma unroll
    for (int r = 0; r < kLangPre; ++r) {
        const int m = tid + r * 256;
        if (m <= N / 2) {
            ot[r][0] = o_load(a, rowm(m), d);
            if (!lone(m)) ot[r][1] = o_load(a, rowm(N - m), d);
        }
    }
    // stage rows of the first outputs: their indices now, their inputs after
    // the fill (then used after the transforms)
    int sst[kLangOutPre];
#pragma unroll
    for (int r = 0; r < kLangOutPre; ++r) {
        const int j = tid + r * 256;
        sst[r] = j < N ? a.row_stage[rowm(j)] : -1;
    }
    // momenta and twiddles in one fill: one wait on memory per 4 rounds
    const double2 *twg = a.twiddle + it.tw_off;
    struct In {
        double p;
        double2 t;
    };
    lds_fill<4>(
        N,
        [&](int j) {
            In v;
            v.p = a.p[rowm(j) * 3 + d];
            v.t = j < N - 1 ? twg[j] : make_double2(0.0, 0.0);
            return v;
        },
        [&](int j, const In &v) {
            z[brev(j, L)] = make_double2(v.p, 0.0);
            if (j < N - 1) tw[j] = v.t;
        });
    StageTerms sg[kLangOutPre] = {};
#pragma unroll
    for (int r = 0; r < kLangOutPre; ++r) {
        const int j = tid + r * 256;
        sg[r].st = sst[r];
        if (sst[r] >= 0) {
            const long long row = rowm(j);
            sg[r].q = a.in_q[row * 3 + d];
            sg[r].hk = a.row_hk[row];
            sg[r].f = a.f[row * 3 + d];
        }
    }
    fft_stages<false>(z, tw, N, L);
    // modes of p (as the forward transform), thermostatted, then the
    // conjugated Hermitian spectrum of the new modes (as the backward one)
    double2 keep[kLangKeep];
#pragma unroll
    for (int r = 0; r < kLangKeep; ++r) {
        const int m = tid + r * 256;
        if (m > N / 2) break;
        OTerms t0, t1;
        if (r < kLangPre) {
            t0 = ot[r][0];
            t1 = ot[r][1];
        } else {
            t0 = o_load(a, rowm(m), d);
            t1 = lone(m) ? t0 : o_load(a, rowm(N - m), d);
        }
        const double2 Z = z[m];
        if (lone(m)) {
            const double x = o_apply(a, t0, Z.x / rN);
            keep[r] = make_double2(rN * x, 0.0);
        } else {
            const double x1 = o_apply(a, t0, r2N * Z.x);
            const double x2 = o_apply(a, t1, r2N * Z.y);
            keep[r] = make_double2(rN2 * x1, rN2 * x2);
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kLangKeep; ++r) {
        const int m = tid + r * 256;
        if (m > N / 2) break;
        if (lone(m)) {
            z[brev(m, L)] = keep[r];
        } else {
            z[brev(m, L)] = make_double2(keep[r].x, -keep[r].y);
            z[brev(N - m, L)] = make_double2(keep[r].x, keep[r].y);
        }
    }
    fft_stages<false>(z, tw, N, L);
#pragma unroll
    for (int r = 0; r < kMaxBeads / 256; ++r) {
        const int j = tid + r * 256;
        if (j >= N) break;
        const long long row = rowm(j);
        const StageTerms st = r < kLangOutPre ? sg[r] : stage_load(a, row, row * 3 + d);
        stage_store(a, st, row * 3 + d, d, z[j].x / N);
    }
}

// ---------------------------------------------------------------------------
// Velocity Verlet with the springs as forces (the paper's alternative to the
// exact normal-mode propagation), first half: for every bead of the item's
// whole columns, p += dt/2 (F + F_sp(q)) with F_sp = -k (2 q_j - q_{j-1} -
// q_{j+1}), then q += dt p / m_f; the centroid of the new ring is stored
// for the virial estimator.  Spring energies are summed in the epilogue.
__device__ void rp_vv(const RpLaunch &a, const RpItem &it, double *smem, double *red)
{
    const int N = it.N, n = it.n;
    const int nc = it.ncols;
    const int tid = threadIdx.x;
    double *sq = smem;                  // [N][nc] old q
    double *sn = smem + N * nc;         // [N][nc] new q
    const double hk = a.sys[it.sys].hkick;
    auto gaddr = [&](int j, int cl) { return (it.row + (long long)j * n) * 3 + it.c0 + cl; };
    lds_fill<8>(N * nc, [&](int e) { return a.in_q[gaddr(e / nc, e % nc)]; },
                [&](int e, double v) { sq[e] = v; });
    __syncthreads();
    const double s1 = sin(kPi / N), lam1 = 4.0 * s1 * s1;
    for (int e = tid; e < N * nc; e += 256) {
        const int j = e / nc, cl = e % nc;
        const int i = (it.c0 + cl) / 3;
        // k = 2 (k lambda_1 / 2) / lambda_1 from mode 1's spring entry; dt/m_f from mode 0
        const double k = N > 1 ? 2.0 * a.prop[5 * (it.row + (long long)n + i) + 4] / lam1 : 0.0;
        const double dtm = a.prop[5 * (it.row + i) + 1];
        const double qj = sq[e];
        const double qp = sq[((j + N - 1) % N) * nc + cl], qn = sq[((j + 1) % N) * nc + cl];
        const double fsp = -k * (2.0 * qj - qp - qn);
        const long long g = gaddr(j, cl);
        const double pn = a.p[g] + hk * (a.f[g] + fsp);
        const double qnew = qj + dtm * pn;
        a.p[g] = pn;
        a.out_q[g] = qnew;
        sn[e] = qnew;
    }
    __syncthreads();
    // centroids: one column per workgroup (many beads) by a block sum, else
    // a thread per column
    if (nc == 1) {
        double v = 0.0;
        for (int j = tid; j < N; j += 256) v += sn[j];
        v = bsum256(v, red);
        __shared__ double s_c;
        if (tid == 0) s_c = v / N;
        __syncthreads();
        for (int j = tid; j < N; j += 256) a.cent[gaddr(j, 0)] = s_c;
    } else {
        double *cs = sq;                // reuse: column centroids
        __syncthreads();
        if (tid < nc) {
            double v = 0.0;
            for (int j = 0; j < N; ++j) v += sn[j * nc + tid];
            cs[tid] = v / N;
        }
        __syncthreads();
        for (int e = tid; e < N * nc; e += 256) a.cent[gaddr(e / nc, e % nc)] = cs[e % nc];
    }
}

__global__ __launch_bounds__(256) void k_rp(RpLaunch a)
{
    extern __shared__ __align__(16) double smem[];
    __shared__ double red[4];
    if ((int)blockIdx.x >= a.n_items) {
        // the extra workgroups: energy reduction (stage A) of the previous
        // step (the dynamic LDS holds at least kReduceThreads doubles)
        reduce_a_part(a.reduce, blockIdx.x - a.n_items, smem);
        return;
    }
    const RpItem it = a.items[blockIdx.x];
    if (a.op == OP_LANG) {
        if (it.kind == RP_DENSE) rp_lang_dense(a, it, smem);
        else rp_lang_fft(a, it, reinterpret_cast<double2 *>(smem));
        return;
    }
    if (a.op == OP_VV) {
        rp_vv(a, it, smem, red);
        return;
    }
    if (it.kind == RP_MFMA) {
        // the step's propagation uses FP64 matrix instructions in both forms
        if (a.precision && a.op != OP_STEP) rp_mfma<float>(a, it, smem);
        else rp_mfma<double>(a, it, smem);
        return;
    }
    if (it.kind == RP_DENSE) rp_dense(a, it, smem, red);
    else if (it.kind == RP_CIRC) rp_circ(a, it, smem, red);
    else rp_fft(a, it, reinterpret_cast<double2 *>(smem), red);
}

const void *rp_kernel_symbol() { return (const void *)k_rp; }

void launch_rp(const RpLaunch &a, hipStream_t st)
{
    const int grid = a.n_items + (a.with_reduce ? a.reduce.n_chunks : 0);
    if (grid <= 0) return;
    hipLaunchKernelGGL(k_rp, dim3(grid), dim3(256), a.lds_bytes, st, a);
}

}  // namespace mixpi
