// Path-integral radial distribution functions (arXiv 2411.11988, the g(r)
// of Sec. "Examples and Discussion"): the bead average of a pair count is
// the same slice-mapped sum as V_mix of Eq. mts-hamiltonian -- every
// unordered, non-excluded particle pair on its N_max slices, particle p at
// bead floor(s * N_p / N_max), weight 1/N_max -- with the pair potential
// replaced by the indicator of a distance bin.
//
// The kernel walks the pair tiles of the force sweep (same blocks, same
// masks).  All slice-pairs of one block carry the weight 1/N_a and bead
// counts are powers of two, so a hit is counted as the integer N_top / N_a
// in units of 1/N_top (N_top: the largest bead count of the handle) in a
// uint32 LDS histogram per workgroup.  Each workgroup covers a run of tiles
// of one system and adds its nonzero bins to the FP64 histogram with
// atomics; every addend is a dyadic rational far inside the FP64 mantissa,
// so the sums are exact and independent of the order of the atomics.
//
// Distances: the nearest-image separation d - L * rint(d / L) and
// r = sqrt(dx^2 + dy^2 + dz^2) are evaluated in FP64 without contraction
// into fused multiply-adds; division and square root are correctly
// rounded, so the bin of every slice-pair is a deterministic function of
// the two positions.
#include "device_common.h"
#include "mixpi_internal.h"

namespace mixpi {

namespace {

struct alignas(16) RdfJ {
    double x, y, z;
    int spec, mol;
};

constexpr int kRdfWaves = 4;

__device__ __forceinline__ int pair_index(int a, int b, int nt1)
{
    // upper-triangle (a <= b) row-major index
    return a * nt1 - a * (a - 1) / 2 + (b - a);
}

__device__ __forceinline__ double nearest(double d, double L)
{
#pragma clang fp contract(off)
    return d - L * rint(d / L);
}

__global__ __launch_bounds__(64 * kRdfWaves) void k_rdf(RdfLaunch a)
{
    extern __shared__ unsigned int hist_lds[];
    __shared__ RdfJ sj[kRdfWaves][64];
    const BlockRange rg = a.ranges[blockIdx.x];
    const SysDev &S = a.sys[rg.sys];
    const int nt1 = S.nt1;
    const int nbins = a.nbins;
    const int nh = nt1 * (nt1 + 1) / 2 * nbins;
    for (int k = threadIdx.x; k < nh; k += blockDim.x) hist_lds[k] = 0u;
    __syncthreads();

    const int lane = threadIdx.x & 63;
    const int wv = (int)threadIdx.x >> 6;
    const double L[3] = {S.box[0], S.box[1], S.box[2]};
    const double iL[3] = {S.ibox[0], S.ibox[1], S.ibox[2]};
    const double rmax = a.rmax;
    const double screen2 = rmax * rmax * (1.0 + 1e-9);
    const double dr = a.rmax / nbins;
    for (int k = wv; k < rg.count; k += kRdfWaves) {
        const PairItem it = a.items[rg.begin + k];
        const PairBlock bk = a.blocks[it.block];
        const unsigned inc = (unsigned)(a.top / (bk.nbeads_b << bk.shift));
        const int jn = min(a.tj, bk.nb - it.j0);
        if (lane < jn) {
            const int j = it.j0 + lane;
            const long long rowj = bk.rowb + (long long)it.b * bk.nb + j;
            const int pj = bk.pb0 + j;
            RdfJ r;
            r.x = a.q[3 * rowj];
            r.y = a.q[3 * rowj + 1];
            r.z = a.q[3 * rowj + 2];
            r.spec = a.ljt[pj];
            r.mol = a.mol[pj];
            sj[wv][lane] = r;
        }
        const long long li = (long long)bk.na << bk.shift;
        const long long idx = (long long)it.i0 + lane;
        const bool vi = idx < li;
        double xi = 0, yi = 0, zi = 0;
        int ti = 0, mi = -1;
        if (vi) {
            const long long rowi = bk.rowa + ((long long)it.b << bk.shift) * bk.na + idx;
            const int pi = bk.pa0 + (int)(idx % bk.na);
            xi = a.q[3 * rowi];
            yi = a.q[3 * rowi + 1];
            zi = a.q[3 * rowi + 2];
            ti = a.ljt[pi];
            mi = a.mol[pi];
        }
        // the wave's own j records: written and read by this wave only
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // for a group with itself only j > i (slot index j0 + js > idx)
        const int jlo = bk.same ? (int)max(-1LL, min((long long)a.tj, idx - it.j0)) : -1;
        const int jhi = vi ? jn : 0;
        for (int js = jlo + 1; js < jhi; ++js) {
            const RdfJ r = sj[wv][js];
            if (r.mol == mi) continue;
            // cheap screen with multiplications by 1/L: a pair clearly
            // beyond r_max (margin 1e-9 relative, far above the few ulps the
            // screen can differ from the exact distance by) is skipped; the
            // rest take the exact, oracle-identical evaluation below
            {
                double ex = xi - r.x, ey = yi - r.y, ez = zi - r.z;
                ex -= L[0] * rint(ex * iL[0]);
                ey -= L[1] * rint(ey * iL[1]);
                ez -= L[2] * rint(ez * iL[2]);
                if (ex * ex + ey * ey + ez * ez > screen2) continue;
            }
            double dx = nearest(xi - r.x, L[0]);
            double dy = nearest(yi - r.y, L[1]);
            double dz = nearest(zi - r.z, L[2]);
            double rr;
            {
#pragma clang fp contract(off)
                rr = sqrt(dx * dx + dy * dy + dz * dz);
            }
            if (!(rr < rmax)) continue;
            int bin = (int)(rr / dr);
            if (bin >= nbins) bin = nbins - 1;
            const int sa = min(ti, r.spec), sb = max(ti, r.spec);
            atomicAdd(&hist_lds[pair_index(sa, sb, nt1) * nbins + bin], inc);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    __syncthreads();

    // flush: bin (sa <= sb, bin) of this system, in units of 1/N_top
    const int nspec = a.nspec;
    double *h = a.hist + (long long)rg.sys * nspec * nspec * nbins;
    for (int k = threadIdx.x; k < nt1 * nt1 * nbins; k += blockDim.x) {
        const int bin = k % nbins;
        const int sa = k / nbins / nt1, sb = k / nbins % nt1;
        if (sa > sb) continue;
        const unsigned c = hist_lds[pair_index(sa, sb, nt1) * nbins + bin];
        if (c) atomicAdd(&h[((long long)sa * nspec + sb) * nbins + bin], (double)c * a.unit);
    }
}

}  // namespace

void launch_rdf(const RdfLaunch &a, int n_ranges, int lds_bytes, hipStream_t st)
{
    if (n_ranges <= 0) return;
    hipLaunchKernelGGL(k_rdf, dim3(n_ranges), dim3(64 * kRdfWaves), lds_bytes, st, a);
}

}  // namespace mixpi
