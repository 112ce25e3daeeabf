// Slice-mapped nonbonded pair sweep of V_mix (arXiv 2411.11988,
// Eq. mts-hamiltonian): every unordered, non-excluded pair of particles is
// evaluated on N_max = max(N_i, N_j) slices, particle p at bead
// floor(s * N_p / N_max) in slice s, weight 1/N_max.
//
// Work decomposition.  Particles come in groups of equal bead count, and
// the state of group g is a [N_g][n_g][3] block.  For a group pair (a, b)
// with N_b = N_a >> shift, the slice-pairs that meet bead b of group b are
// exactly the rows [b << shift, (b + 1) << shift) of group a -- a contiguous
// run of n_a << shift beads.  One work item is a 64 IW x TJ tile of that
// rectangle (or of the upper triangle for a group with itself), TJ = 16, 32
// or 64 per system: one lane per i-bead, the TJ j-beads staged in LDS.
// With WAVES = 2 (IW = 1) two waves share a 64-bead i-tile, each taking half
// of the j-beads (more, shorter waves when a launch has few tiles per
// SIMD), and hand their i-forces to wave 0 at the end.  With IW = 2 or 4
// each of IW waves takes its own 64 i-beads against all TJ j-beads; each
// wave adds its j-reactions to its own LDS accumulator and the store sums
// them in wave order (one j-partial per IW i-tiles: fewer partial-force
// slots for large launches).  Lane l visits j-slot (l mod W) XOR t at step
// t, so the lanes spread over distinct j-beads and the Newton-3 reaction
// goes to a per-j LDS accumulator with a return-less LDS atomic add;
// i-forces stay in registers.  The loop body has no branches: cutoff,
// exclusion and padding are multiplicative masks, so consecutive steps
// overlap.  Electron-atom tiles of i-split waves in large boxes leave out
// the atoms no bead of the tile can reach (a box bound; see pair_tile).
// Each tile stores its i- and j-partial forces into slots of its own; a
// per-row gather in a fixed order sums them (no global atomics).
//
// Precision: separations and the nearest-image shift are FP64 (positions
// sit up to a box length from the origin).  The electron-atom
// pseudopotential is evaluated in R (double, or float for the FP32 form);
// atom-atom Lennard-Jones and Coulomb terms in FP64 from an R seed of 1/r.
// Every force, energy and theta term is summed in FP64 (per lane, then
// across lanes, waves and tiles).
#include <type_traits>

#include "device_common.h"
#include "mixpi_internal.h"

namespace mixpi {

// Reciprocal square root.  Hardware approximations: v_rsq_f32 in the FP32
// form, v_rsq_f64 in the FP64 form.  Atom-atom pairs refine either seed by
// one FP64 Newton step (y <- y (3 - r^2 y^2) / 2, which squares the seed's
// relative error), and take 1/r^2 as y^2; the electron-atom pseudopotential
// of the FP32 form uses the FP32 value as it is.  Used only where the
// argument is a positive, finite r^2 (or r^2 + a^2); masked candidates may
// produce non-finite values, which the masks select away.
template <typename R> __device__ __forceinline__ R rsqrt_r(R x);
template <> __device__ __forceinline__ double rsqrt_r<double>(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    return y * fma(-0.5 * x * y, y, 1.5);
}
template <> __device__ __forceinline__ float rsqrt_r<float>(float x) { return __builtin_amdgcn_rsqf(x); }

// 1/sqrt(x) in FP64 from the form's hardware seed and one FP64 Newton step.
template <typename R> __device__ __forceinline__ double rsqrt_fp64(double x)
{
    double y;
    if constexpr (std::is_same<R, float>::value) y = (double)__builtin_amdgcn_rsqf((float)x);
    else y = __builtin_amdgcn_rsq(x);
    return y * fma(-0.5 * x * y, y, 1.5);
}

// The j-beads of a tile in LDS as separate arrays of 8-byte elements, so
// that one byte offset (slot * 8) addresses every field of a slot and a
// wave's reads of consecutive slots are consecutive words (free of bank
// conflicts).  Fields: position; the FP64 charge (k_e q_j for an
// electron-atom block with the electron as i); the slot's molecule and
// index in its group (-1: padding); its LJ type as a byte offset into the
// type-pair table, and the R-rounded pseudopotential constant pp_q k_e q_j
// (FP32 form).
struct alignas(8) JMol {
    int mol, jg;
};
struct alignas(8) JTyp {
    int jt;        // LJ type * sizeof(LjPar)
    float kq;      // pp_q k_e q_j, FP32
};
template <typename R> struct JSlot {
    double x, y, z, qd;
    int mol, jg, jt;
    float kq;
};
// LDS of a pair workgroup with tiles up to TJM wide, WAVES j-split waves and
// IW i-split waves (the workgroups per CU are LDS-bound near 10 KB, so
// nothing unused is kept).
template <typename R, int TJM, int WAVES, int IW> struct PairLds {
    double sjx[TJM], sjy[TJM], sjz[TJM], sjq[TJM];
    JMol sjm[TJM];
    JTyp sjt[TJM];
    // j-reactions: one accumulator per i-split wave, summed in wave order at
    // the store (atomics of different waves would land in timing order)
    double fjx[IW][TJM], fjy[IW][TJM], fjz[IW][TJM];
    LjPar tlj[kLjTab];
    double xs[WAVES > 1 ? WAVES : 1][3][WAVES > 1 ? 64 : 1];   // i-forces handed to wave 0
    double es[WAVES > IW ? WAVES : IW][5];                      // the waves' sums
    double cbox[IW][6];   // culled tiles: each i-split wave's bead box
    int ncomp;            // culled tiles: slots the sweep visits
};

// Element at byte offset off of an LDS array.
template <typename T> __device__ __forceinline__ T &at(T *base, int off)
{
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off);
}

// One item of j-tile width TJ: its i-beads against it.nj consecutive
// j-tiles (a j-run), one after the other through the same LDS, the i-forces
// summed over the run and stored once.
// FIXED: every item of the launch has width TJ, so item k's natural slots
// start at k (64 IW + jrun TJ), known before the item is loaded.
template <typename R, bool THETA, int TJ, int WAVES, int IW, bool FIXED, int TJM>
__device__ __forceinline__ void pair_tile(const PairLaunch &a, const PairItem &it, const PairBlock &bk,
                                          PairLds<R, TJM, WAVES, IW> &L)
{
    const SysDev &S = a.sys[bk.sys];
    const double *th = a.theta ? a.theta + 6 * bk.sys : S.theta0;
    const int lane = threadIdx.x & 63;
    const int wv = WAVES > 1 ? (int)threadIdx.x >> 6 : 0;   // j-split wave: j-slots wv*TJ/WAVES ...
    const int iw = IW > 1 ? (int)threadIdx.x >> 6 : 0;      // i-split wave: i-beads i0 + 64 iw ...
    // output positions of this lane's slots, fetched early
    const long long si = FIXED ? (long long)blockIdx.x * (64 * IW + a.jrun * TJ) : it.islot;
    const long long sj = FIXED ? si + 64 * IW : it.jslot;
    const int di = a.dest[si + 64 * iw + lane];
    int dj = -1;

    double *const sjx = L.sjx, *const sjy = L.sjy, *const sjz = L.sjz, *const sjq = L.sjq;
    JMol *const sjm = L.sjm;
    JTyp *const sjt = L.sjt;
    double *const fjx = L.fjx[iw], *const fjy = L.fjy[iw], *const fjz = L.fjz[iw];
    LjPar *const tlj = L.tlj;
    // the j-slot at byte offset o (slot * 8) as read by the loops
    auto jload = [&](int o) {
        const JMol m = at(sjm, o);
        const JTyp t = at(sjt, o);
        return JSlot<R>{at(sjx, o), at(sjy, o), at(sjz, o), at(sjq, o), m.mol, m.jg, t.jt, t.kq};
    };

    const int nt1 = bk.nt1;
    const double rc_lj = S.rc_lj, rc_c = S.rc_c;
    if (bk.kind == PK_ATOM) {
        // the system's table, built at create time; with theta passed, the
        // pair (0, 0) takes its eps and sigma from it
        const LjPar *tab = a.ljpar + bk.lj_off;
        for (int tp = lane; tp < nt1 * nt1; tp += 64) {
            LjPar lp;
            if (tp == 0 && a.theta) {
                const double eps = th[2], sig = th[3];
                const double s2 = sig * sig;
                double c6 = s2 / (rc_lj * rc_lj);
                c6 = c6 * c6 * c6;
                const double c12 = c6 * c6;
                lp.e4 = 4.0 * eps;
                lp.s2 = s2;
                lp.c0 = 4.0 * eps * (c12 - c6);
                lp.c1 = 4.0 * eps * (-12.0 * c12 + 6.0 * c6) / (rc_lj * rc_lj);
            } else {
                lp = tab[tp];
            }
            tlj[tp] = lp;
        }
    }

    // Culled tiles (electron-atom blocks in boxes large against the
    // cutoff, one j-wave): the j-atoms that no i-bead of the item can reach
    // are left out of the sweep.  The item's i-beads lie in a box [lo, hi]
    // of minimum-image offsets from its first bead; a j-atom whose periodic
    // gap to that box is at least r_c (plus 1e-6 A against rounding) has
    // every pair distance at least r_c (triangle inequality of the
    // minimum-image distance), so all its terms would be masked.  The kept
    // atoms are staged first (in staging order), padded to a multiple of 4.
    // Only tiles of several i-split waves cull (their 128 or 256 beads
    // amortise the box; the one-wave kernels stay within their registers).
    constexpr bool CULLABLE = WAVES == 1 && IW > 1;
    const bool cull = CULLABLE && bk.cull != 0;
    double rx = 0, ry = 0, rz = 0, lox = 0, loy = 0, loz = 0, hix = 0, hiy = 0, hiz = 0;
    const double rcut = S.rc_pp + 1e-6, rcut2 = rcut * rcut;
    int jslot = -1;      // staging lane: its slot in the staged tile (-1: culled)

    // j-tile kj of the run: bead b of group b, particles j0 .. j0 + jn;
    // padding slots get harmless values and are masked out
    struct JLoad {
        double x, y, z, qd;
        JMol jm;
        JTyp jt;
    };
    auto stage_load = [&](int kj) {
        JLoad v{0.0, 0.0, 0.0, 0.0, JMol{-1, -1}, JTyp{0, 0.0f}};
        const int j0 = it.j0 + kj * TJ, jn = min(TJ, bk.nb - j0);
        const int js = threadIdx.x;
        if (js < TJ) dj = a.dest[sj + kj * TJ + js];
        if (js < jn) {
            const int j = j0 + js;
            const long long rowj = bk.rowb + (long long)it.b * bk.nb + j;
            const int pj = bk.pb0 + j;
            v.x = a.q[3 * rowj];
            v.y = a.q[3 * rowj + 1];
            v.z = a.q[3 * rowj + 2];
            // electron-atom blocks with the electron as i take k_e q_j as
            // their pseudopotential constant: scaled here, once per tile
            const double qc = a.charge[pj];
            v.qd = bk.kind == PK_E_ATOM ? kCoulombKcal * qc : qc;
            v.jm.mol = a.mol[pj];
            v.jm.jg = j;
            v.jt.jt = a.ljt[pj] * (int)sizeof(LjPar);
            v.jt.kq = (float)(th[0] * v.qd);
        }
        return v;
    };
    auto put = [&](int slot, const JLoad &v) {
        sjx[slot] = v.x;
        sjy[slot] = v.y;
        sjz[slot] = v.z;
        sjq[slot] = v.qd;
        sjm[slot] = v.jm;
        sjt[slot] = v.jt;
    };
    // periodic gap along one axis from offset d to the interval [lo, hi]
    // (offsets within half a box of the reference)
    auto gap = [](double d, double lo, double hi, double L) {
        double g = fmax(0.0, fmax(lo - d, d - hi));
        g = fmin(g, fmax(0.0, fmax(lo - (d + L), (d + L) - hi)));
        return fmin(g, fmax(0.0, fmax(lo - (d - L), (d - L) - hi)));
    };
    auto stage_write = [&](int kj, const JLoad &v) {
        const int js = threadIdx.x;
        if (js >= TJ) return;
        if (!cull) {
            jslot = js;
            put(js, v);
            for (int u = 0; u < IW; ++u) {
                L.fjx[u][js] = 0.0;
                L.fjy[u][js] = 0.0;
                L.fjz[u][js] = 0.0;
            }
            return;
        }
        const int jn = min(TJ, bk.nb - (it.j0 + kj * TJ));
        bool keep = false;
        if (js < jn) {
            double dx = v.x - rx, dy = v.y - ry, dz = v.z - rz;
            dx -= S.box[0] * rint(dx * S.ibox[0]);
            dy -= S.box[1] * rint(dy * S.ibox[1]);
            dz -= S.box[2] * rint(dz * S.ibox[2]);
            const double gx = gap(dx, lox, hix, S.box[0]);
            const double gy = gap(dy, loy, hiy, S.box[1]);
            const double gz = gap(dz, loz, hiz, S.box[2]);
            keep = gx * gx + gy * gy + gz * gz < rcut2;
        }
        // the staging lanes are the first TJ lanes of wave 0
        const unsigned long long km = lanes(keep);
        const int n = __builtin_popcountll(km);
        const int n4 = (n + 3) & ~3;
        jslot = keep ? (int)__builtin_amdgcn_mbcnt_hi((unsigned)(km >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((unsigned)km, 0u))
                     : -1;
        if (keep) put(jslot, v);
        if (js >= n && js < n4) put(js, JLoad{0.0, 0.0, 0.0, 0.0, JMol{-1, -1}, JTyp{0, 0.0f}});
        if (js < n4) {
            for (int u = 0; u < IW; ++u) {
                L.fjx[u][js] = 0.0;
                L.fjy[u][js] = 0.0;
                L.fjz[u][js] = 0.0;
            }
        }
        if (js == 0) L.ncomp = n4;
    };
    JLoad jv0 = stage_load(0);

    // i bead
    const long long li = (long long)bk.na << bk.shift;
    const long long idx = (long long)it.i0 + 64 * iw + lane;
    const bool vi = idx < li;
    const long long rowi = bk.rowa + ((long long)it.b << bk.shift) * bk.na + idx;
    double xi = 0, yi = 0, zi = 0, qi = 0;
    int ti = 0, mi = -1;
    if (vi) {
        // idx < na N_a: a 32-bit remainder
        const int pi = bk.pa0 + (int)((unsigned)idx % (unsigned)bk.na);
        xi = a.q[3 * rowi];
        yi = a.q[3 * rowi + 1];
        zi = a.q[3 * rowi + 2];
        qi = a.charge[pi];
        ti = a.ljt[pi];
        mi = a.mol[pi];
    }
    if (cull) {
        // the item's first i-bead is the reference; the box of the offsets
        // of every wave's beads
        const long long row0 = bk.rowa + ((long long)it.b << bk.shift) * bk.na + it.i0;
        rx = a.q[3 * row0];
        ry = a.q[3 * row0 + 1];
        rz = a.q[3 * row0 + 2];
        double dx = xi - rx, dy = yi - ry, dz = zi - rz;
        dx -= S.box[0] * rint(dx * S.ibox[0]);
        dy -= S.box[1] * rint(dy * S.ibox[1]);
        dz -= S.box[2] * rint(dz * S.ibox[2]);
        constexpr double kBig = 1e300;
        hix = wmax(vi ? dx : -kBig);
        hiy = wmax(vi ? dy : -kBig);
        hiz = wmax(vi ? dz : -kBig);
        lox = -wmax(vi ? -dx : -kBig);
        loy = -wmax(vi ? -dy : -kBig);
        loz = -wmax(vi ? -dz : -kBig);
        if constexpr (IW > 1) {
            if (lane == 0) {
                L.cbox[iw][0] = lox;
                L.cbox[iw][1] = loy;
                L.cbox[iw][2] = loz;
                L.cbox[iw][3] = hix;
                L.cbox[iw][4] = hiy;
                L.cbox[iw][5] = hiz;
            }
            __syncthreads();
            for (int u = 0; u < IW; ++u) {
                lox = fmin(lox, L.cbox[u][0]);
                loy = fmin(loy, L.cbox[u][1]);
                loz = fmin(loz, L.cbox[u][2]);
                hix = fmax(hix, L.cbox[u][3]);
                hiy = fmax(hiy, L.cbox[u][4]);
                hiz = fmax(hiz, L.cbox[u][5]);
            }
        }
    }
    stage_write(0, jv0);
    __syncthreads();

    const double Lx = S.box[0], Ly = S.box[1], Lz = S.box[2];
    const double iLx = S.ibox[0], iLy = S.ibox[1], iLz = S.ibox[2];
    double fxi = 0, fyi = 0, fzi = 0;
    // per-lane energy and theta sums in FP64 (each term converted once),
    // then FP64 across lanes, waves and tiles
    double e0r = 0, e1r = 0;          // atom: LJ, Coulomb; electron: pp
    double g0r = 0, g1r = 0;          // theta partials (pp: q_e, a; atom: eps, sigma)
    // in-cutoff slice-pairs of the wave: each candidate step adds the
    // population count of its lane mask (scalar instructions, wave-uniform)
    int cnt = 0;
    // slots that may interact: jg > key, i.e. real j (padding has jg = -1),
    // for a group with itself j > i, and none for a lane past the i-run
    const int key = !vi ? 0x7fffffff : (bk.same ? (int)idx : -1);
    // step t of a lane's sweep of its wave's W = TJ / WAVES slots takes slot
    // (lane mod W) XOR t (byte offset base ^ 8t, the wave's slot range in
    // the high bits of base): every lane visits each slot once, and at each
    // step the lanes mod W visit distinct slots, so the LDS reads and the
    // reaction adds spread over the slots
    const int base8 = ((lane & (TJ / WAVES - 1)) * 8) | (wv * (TJ / WAVES) * 8);
    // base8 made opaque to the optimiser where a sweep starts, so that
    // base8 ^ 8t stays one XOR per step (knowing base8 a multiple of 8, it
    // would shift (base ^ t) instead)
    auto opaque = [](int v) {
        asm volatile("" : "+v"(v));
        return v;
    };
    const double w = bk.w;
    // the j-tiles of the run: tile 0 is staged above; after each sweep its
    // j-reactions go to their slots, and the next tile replaces it
    const int nj = it.nj;
    auto run = [&](auto &&sweep_tile) {
        for (int kj = 0; kj < nj; ++kj) {
            if (kj > 0) {
                const JLoad jv = stage_load(kj);
                __syncthreads();      // the previous tile's reactions are stored
                stage_write(kj, jv);
                __syncthreads();
            }
            sweep_tile();
            __syncthreads();          // every wave's reactions are in
            const int jn = min(TJ, bk.nb - (it.j0 + kj * TJ));
            if ((int)threadIdx.x < jn) {
                // a culled atom's reaction is an exact 0
                double *o = a.part + 3LL * dj;
                const int t = jslot;
                double sx = 0.0, sy = 0.0, sz = 0.0;
                if (t >= 0) {
                    sx = L.fjx[0][t];
                    sy = L.fjy[0][t];
                    sz = L.fjz[0][t];
                    for (int v = 1; v < IW; ++v) {
                        sx += L.fjx[v][t];
                        sy += L.fjy[v][t];
                        sz += L.fjz[v][t];
                    }
                }
                o[0] = w * sx;
                o[1] = w * sy;
                o[2] = w * sz;
            }
        }
    };

    if (bk.kind == PK_ATOM) {
        // Atom-atom Lennard-Jones and Coulomb in FP64 in both forms, from
        // the form's 1/r seed refined by one FP64 Newton step: the forces on
        // a cation are small differences of large first-shell repulsions
        // and attractions, which FP32 arithmetic would leave about 1e-5 of
        // the RMS force off; without packed FP32 an FP64 multiply-add issues
        // at the FP32 rate on this chip, so only the seed is cheaper in FP32.
        const double rc2_lj = rc_lj * rc_lj, rc2_c = rc_c * rc_c;
        const double rc2max = fmax(rc2_lj, rc2_c);
        // rc_c = 0 (no bead-resolved Coulomb): finite stand-ins, every
        // Coulomb term is masked by r^2 < 0
        const double irc = S.irc, irc3 = S.irc3;
        const double hc = 0.5 * irc3;
        const double vc0 = irc + rc2_c * hc;   // Coulomb term: K (1/r + r^2 hc - vc0)
        const double kqi = kCoulombKcal * qi;
        const int trow = ti * nt1 * (int)sizeof(LjPar);   // byte offset of the i type's row
        const double th_eps = th[2], th_sig = th[3];
        // LJ: blocks whose type pairs all have eps = 0 (and cannot reach the
        // theta-overridden pair (0, 0)) run a loop without the LJ terms; the
        // masked LJ contribution there is an exact zero, so both loops give
        // the same bits.
        // SP (compacted): blocks where few candidates are inside the cutoff
        // first mark each lane's in-cutoff j-slots in a bit mask (distance
        // pass only), then run the pair math once per marked slot, all lanes
        // together until the fullest lane is done.  A lane visits its marked
        // slots in the same cyclic order as the masked loop visits all of
        // them; the j-reactions arrive in another order.
        auto sweep = [&](auto lj_tag, auto sp_tag) {
            constexpr bool LJ = decltype(lj_tag)::value;
            constexpr bool SP = decltype(sp_tag)::value;
            constexpr int W = TJ / WAVES;
            // candidate (this lane's i-bead, the j-slot at byte offset o);
            // with SP the distance pass has already established that it
            // interacts iff `live`
            auto body = [&](int o, bool live) {
                const JSlot<R> jr = jload(o);
                double dx = xi - jr.x, dy = yi - jr.y, dz = zi - jr.z;
                const int tp = trow + jr.jt;
                dx -= Lx * rint(dx * iLx);
                dy -= Ly * rint(dy * iLy);
                dz -= Lz * rint(dz * iLz);
                const double r2 = dx * dx + dy * dy + dz * dz;
                bool ok = live;
                // masks combine without short-circuit branches (straight-line
                // code); each term below also tests its own cutoff
                if constexpr (!SP) ok = (jr.jg > key) & (mi != jr.mol);
                // Masked terms are multiplied by 0 instead of selected away:
                // r^2 is clamped to 1e-20 A^2 (only coincident beads, all
                // masked, are below it), so every term is finite; a term kept
                // is multiplied by 1, exactly.
                const double K = kqi * jr.qd;
                const bool in_c = ok & (r2 < rc2_c) & (K != 0.0);
                const double Km = in_c ? K : 0.0;     // the Coulomb constant, 0 if masked
                const double ir = rsqrt_fp64<R>(fmax(r2, 1e-20));
                const double ir2 = ir * ir;
                const double vc = Km * (fma(r2, hc, ir) - vc0);
                const double gc = Km * fma(ir2, ir, -irc3);
                double g;
                // the in-cutoff count takes the same conditions as lane
                // masks (scalar instructions)
                unsigned long long hits = lanes(r2 < rc2_c) & lanes(K != 0.0);
                if constexpr (LJ) {
                    const LjPar lp = at(tlj, tp);
                    const double e4 = lp.e4, c1l = lp.c1;
                    const double s2 = lp.s2 * ir2;
                    const double s6 = s2 * s2 * s2;
                    const double s12 = s6 * s6;
                    const bool in_lj = ok & (r2 < rc2_lj) & (e4 != 0.0);
                    const double mlj = in_lj ? 1.0 : 0.0;
                    const double vlj = e4 * (s12 - s6) - lp.c0 - 0.5 * (r2 - rc2_lj) * c1l;
                    const double glj = e4 * (12.0 * s12 - 6.0 * s6) * ir2 + c1l;
                    g = fma(glj, mlj, gc);
                    e0r = fma(vlj, mlj, e0r);
                    hits |= lanes(r2 < rc2_lj) & lanes(e4 != 0.0);
                    if (THETA) {
                        // d/d eps and d/d sigma of the (0,0) LJ term
                        const bool on = in_lj & (tp == 0);   // type pair (0, 0)
                        const double c6 = tlj[0].s2 / rc2_lj;
                        const double c6c = c6 * c6 * c6, c12c = c6c * c6c;
                        const double fs = 4.0 * th_eps / th_sig;
                        const double dsg = fs * (12.0 * s12 - 6.0 * s6) -
                                           fs * (12.0 * c12c - 6.0 * c6c) -
                                           0.5 * (r2 - rc2_lj) * fs * (-144.0 * c12c + 36.0 * c6c) /
                                               rc2_lj;
                        g0r += on ? vlj / th_eps : 0.0;
                        g1r += on ? dsg : 0.0;
                    }
                } else {
                    g = gc;
                }
                e1r += vc;
                cnt += __builtin_popcountll(
                    hits & (SP ? lanes(live) : lanes(jr.jg > key) & lanes(mi != jr.mol)));
                fxi = fma(g, dx, fxi);
                fyi = fma(g, dy, fyi);
                fzi = fma(g, dz, fzi);
                if (SP && !live) return;   // nothing to add: spare the LDS
                const double ng = -g;
                atomicAdd(&at(fjx, o), ng * dx);
                atomicAdd(&at(fjy, o), ng * dy);
                atomicAdd(&at(fjz, o), ng * dz);
            };
            const int b8 = opaque(base8);
            if constexpr (!SP) {
#pragma unroll 4
                for (int t = 0; t < W; ++t) body(b8 ^ (8 * t), true);
            } else {
                using Mask = std::conditional_t<(W > 32), unsigned long long, unsigned>;
                Mask m = 0;
#pragma unroll 4
                for (int t = 0; t < W; ++t) {
                    const int o = b8 ^ (8 * t);
                    const JSlot<R> jr = jload(o);
                    double dx = xi - jr.x, dy = yi - jr.y, dz = zi - jr.z;
                    dx -= Lx * rint(dx * iLx);
                    dy -= Ly * rint(dy * iLy);
                    dz -= Lz * rint(dz * iLz);
                    const double r2d = dx * dx + dy * dy + dz * dz;
                    // non-short-circuit: no branch, so the unrolled steps' LDS
                    // reads are issued together
                    const bool ok = (jr.jg > key) & (mi != jr.mol) & (r2d < rc2max);
                    m |= ok ? (Mask(1) << t) : Mask(0);
                }
                // wave-uniform trip count: the most marked slots of any lane
                while (__ballot(m != 0)) {
                    const bool live = m != 0;
                    int t = 0;
                    if constexpr (W > 32) t = live ? __builtin_ctzll(m) : 0;
                    else t = live ? __builtin_ctz(m) : 0;
                    m &= m - 1;
                    body(b8 ^ (8 * t), live);
                }
            }
        };
        if (bk.lj) {
            if (bk.sparse) run([&] { sweep(std::true_type{}, std::true_type{}); });
            else run([&] { sweep(std::true_type{}, std::false_type{}); });
        } else {
            if (bk.sparse) run([&] { sweep(std::false_type{}, std::true_type{}); });
            else run([&] { sweep(std::false_type{}, std::false_type{}); });
        }
    } else {
        // electron-atom pseudopotential K / sqrt(r^2 + a^2), K = k_e pp_q q_atom,
        // in R; the theta partials (adjoint launches only) in FP64
        const double rc = S.rc_pp, rc2 = rc * rc;
        const double pa = th[1], a2 = pa * pa, pq = th[0];
        double phicd = S.pp_phic, psicd = S.pp_psic, chicd = S.pp_chic;
        if (a.theta) {
            const double u_c = rc2 + a2;
            phicd = 1.0 / sqrt(u_c);
            psicd = -1.0 / (u_c * sqrt(u_c));
            chicd = 1.0 / (u_c * u_c * sqrt(u_c));
        }
        const R phic = (R)phicd, psic = (R)psicd, hpsic = (R)(0.5 * psicd);
        const R ra2 = (R)a2, rrc2 = (R)rc2;
        const double kqid = kCoulombKcal * qi;
        // the constant pp_q k_e q_atom of an atom-i block (R)
        const R kqi = (R)(pq * kqid);
        // E_IS_I: the electron is the i side and the constant is the j
        // atom's pp_q k_e q_j (its slot's kq in the FP32 form); otherwise the
        // i atom's
        // MOL: some pair of the block may share a molecule id (else the
        // compare is left out; it would always pass)
        // CULL: the staged tile holds L.ncomp slots (a multiple of 4; the
        // kept atoms, then padding); lane l sweeps them from slot l mod
        // ncomp on, wrapping around
        auto sweep_e = [&](auto e_tag, auto mol_tag, auto cull_tag) {
            constexpr bool E_IS_I = decltype(e_tag)::value;
            constexpr bool MOL = decltype(mol_tag)::value;
            constexpr bool CULL = decltype(cull_tag)::value;
            auto step = [&](int o) {
                const JSlot<R> jr = jload(o);
                double dx = xi - jr.x, dy = yi - jr.y, dz = zi - jr.z;
                dx -= Lx * rint(dx * iLx);
                dy -= Ly * rint(dy * iLy);
                dz -= Lz * rint(dz * iLz);
                const double r2d = dx * dx + dy * dy + dz * dz;
                const bool ok = (jr.jg > key) & (!MOL || mi != jr.mol) & (r2d < rc2);
                const R r2 = (R)r2d;
                R kq = kqi;
                if constexpr (E_IS_I) {
                    if constexpr (std::is_same<R, float>::value) kq = jr.kq;
                    else kq = pq * jr.qd;
                }
                // a masked candidate gets the constant 0 (r^2 + a^2 > 0, so
                // its terms are finite zeros): no branch, no selects after
                const R kqm = ok ? kq : (R)0;
                const R ir = rsqrt_r<R>(r2 + ra2);
                const R ir3 = ir * ir * ir;
                const R vq = kqm * (ir - phic - (r2 - rrc2) * hpsic);
                const R gq = kqm * (ir3 + psic);
                e0r += (double)vq;
                cnt += __builtin_popcountll(lanes(jr.jg > key) & lanes(!MOL || mi != jr.mol) &
                                            lanes(r2d < rc2));
                if (THETA) {
                    const double kqd = E_IS_I ? jr.qd : kqid;
                    const double u = r2d + a2;
                    const double y = rsqrt_fp64<R>(u);
                    const double y3 = y * y * y;
                    const double vqd = kqd * (y - phicd - 0.5 * (r2d - rc2) * psicd);
                    g0r += ok ? vqd : 0.0;
                    g1r += ok ? pq * kqd * (-pa * y3 - pa * psicd - 1.5 * pa * (r2d - rc2) * chicd)
                              : 0.0;
                }
                const double gd = (double)gq, ngd = -gd;
                fxi = fma(gd, dx, fxi);
                fyi = fma(gd, dy, fyi);
                fzi = fma(gd, dz, fzi);
                atomicAdd(&at(fjx, o), ngd * dx);
                atomicAdd(&at(fjy, o), ngd * dy);
                atomicAdd(&at(fjz, o), ngd * dz);
            };
            if constexpr (CULL) {
                const int nc = uni(L.ncomp);
                if (nc == 0) return;
                int s = (int)((unsigned)lane % (unsigned)nc);
                for (int t = 0; t < nc; t += 4) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        step(s * 8);
                        s = s + 1 == nc ? 0 : s + 1;
                    }
                }
            } else {
                const int b8 = opaque(base8);
#pragma unroll 4
                for (int t = 0; t < TJ / WAVES; ++t) step(b8 ^ (8 * t));
            }
        };
        using T1 = std::true_type;
        using F0 = std::false_type;
        if (bk.kind == PK_E_ATOM) {
            if (cull) {
                if constexpr (CULLABLE) {
                    if (bk.mol) run([&] { sweep_e(T1{}, T1{}, T1{}); });
                    else run([&] { sweep_e(T1{}, F0{}, T1{}); });
                }
            } else {
                if (bk.mol) run([&] { sweep_e(T1{}, T1{}, F0{}); });
                else run([&] { sweep_e(T1{}, F0{}, F0{}); });
            }
        } else {
            if (bk.mol) run([&] { sweep_e(F0{}, T1{}, F0{}); });
            else run([&] { sweep_e(F0{}, F0{}, F0{}); });
        }
    }
    // e0: LJ (atom blocks with LJ) or pseudopotential; e1: Coulomb (atom
    // blocks); a sum that the block cannot have is an exact 0
    double e0 = (bk.kind != PK_ATOM || bk.lj) ? wsum(e0r) : 0.0;
    double e1 = bk.kind == PK_ATOM ? wsum(e1r) : 0.0;
    double g0 = 0.0, g1 = 0.0;

    if (THETA) {
        g0 = wsum(g0r);
        g1 = wsum(g1r);
    }
    if (WAVES > 1) {
        // the other waves hand their i-forces and sums to wave 0
        auto &xs = L.xs;
        auto &es = L.es;
        if (wv > 0) {
            xs[wv][0][lane] = fxi;
            xs[wv][1][lane] = fyi;
            xs[wv][2][lane] = fzi;
            if (lane == 0) {
                es[wv][0] = e0;
                es[wv][1] = e1;
                es[wv][2] = g0;
                es[wv][3] = g1;
                es[wv][4] = (double)cnt;
            }
        }
        __syncthreads();
        if (wv > 0) return;
        for (int v = 1; v < WAVES; ++v) {
            fxi += xs[v][0][lane];
            fyi += xs[v][1][lane];
            fzi += xs[v][2][lane];
            e0 += es[v][0];
            e1 += es[v][1];
            g0 += es[v][2];
            g1 += es[v][3];
            cnt += (int)es[v][4];
        }
    } else if (IW > 1) {
        // the i-split waves' sums meet in wave 0, in wave order
        auto &es = L.es;
        if (lane == 0) {
            es[iw][0] = e0;
            es[iw][1] = e1;
            es[iw][2] = g0;
            es[iw][3] = g1;
            es[iw][4] = (double)cnt;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int v = 1; v < IW; ++v) {
                e0 += es[v][0];
                e1 += es[v][1];
                g0 += es[v][2];
                g1 += es[v][3];
                cnt += (int)es[v][4];
            }
        }
    }

    // partial forces of this item go to its own slots (64 IW i-slots, then
    // TJ j-slots per j-tile, stored above), each at its row-contiguous
    // position; the per-row gather sums them, so no two workgroups write the
    // same address
    if (vi) {
        double *o = a.part + 3LL * di;
        o[0] = w * fxi;
        o[1] = w * fyi;
        o[2] = w * fzi;
    }
    if (threadIdx.x == 0) {
        double *e = a.eslot + (long long)blockIdx.x * A_N;
        for (int k = 0; k < A_N; ++k) e[k] = 0.0;
        if (bk.kind == PK_ATOM) {
            e[A_LJ] = w * e0;
            e[A_COUL] = w * e1;
            e[A_TH2] = w * g0;
            e[A_TH3] = w * g1;
            e[A_CNT_AA] = (double)cnt;
        } else {
            e[A_PP] = w * e0;
            e[A_TH0] = w * g0;
            e[A_TH1] = w * g1;
            e[A_CNT_EA] = (double)cnt;
        }
    }
}

// TJ > 0: every item of the launch has that width; TJ = 0: each item's own
// width (a batch whose systems differ; the widest body sets the registers).
// The fixed-width one-wave FP32-form force kernels are held to 96 VGPRs,
// five waves per SIMD (the compiler fits them without spills; left alone it
// takes a few more and drops to four; the FP64 form and the multi-wave
// tiles would spill).
template <typename R, bool THETA, int TJ, int WAVES, int IW>
__global__ __launch_bounds__(64 * WAVES * IW) __attribute__((amdgpu_waves_per_eu(TJ > 0 && !THETA && sizeof(R) == 4 && WAVES * IW == 1 ? 5 : 1)))
void k_pair(PairLaunch a, BondedLaunch bl)
{
    __shared__ double red[WAVES * IW];
    if ((int)blockIdx.x >= a.n_items) {
        // bonded workgroups of the same launch (64 terms each)
        const int bb = blockIdx.x - a.n_items;
        bonded_block<THETA>(bl, bl.blocks[bb], bl.eslot + (long long)bb * A_N, red);
        return;
    }
    // the item and its block are independent loads (the block is copied per
    // item), so everything after them is one dependent step away
    PairItem it = a.items[blockIdx.x];
    PairBlock bk = a.iblocks[blockIdx.x];
    // both are the same in every lane: scalar registers
    it = PairItem{uni(it.block), uni(it.b), uni(it.i0), uni(it.j0),
                  uni(it.tj), uni(it.islot), uni(it.jslot), uni(it.nj)};
    bk = PairBlock{uni(bk.sys), uni(bk.kind), uni(bk.same), uni(bk.shift), uni(bk.na),
                   uni(bk.nb), uni(bk.pa0), uni(bk.pb0), uni(bk.rowa), uni(bk.rowb),
                   uni(bk.w), uni(bk.nbeads_b), uni(bk.lj), uni(bk.sparse), uni(bk.lj_off),
                   uni(bk.nt1), uni(bk.mol), uni(bk.cull)};
    constexpr int TJM = TJ > 0 ? TJ : kMaxTj;
    __shared__ PairLds<R, TJM, WAVES, IW> L;
    if constexpr (TJ > 0) {
        pair_tile<R, THETA, TJ, WAVES, IW, true>(a, it, bk, L);
    } else {
        if (it.tj == 16) pair_tile<R, THETA, 16, WAVES, IW, false>(a, it, bk, L);
        else if (it.tj == 32) pair_tile<R, THETA, 32, WAVES, IW, false>(a, it, bk, L);
        else pair_tile<R, THETA, 64, WAVES, IW, false>(a, it, bk, L);
    }
}

template <int TJ, int WAVES, int IW>
void launch_pair_tj(const PairLaunch &a, const BondedLaunch &b, int precision, bool with_theta,
                    hipStream_t st)
{
    dim3 grid(a.n_items + b.n_blocks), block(64 * WAVES * IW);
    if (precision == 0) {
        if (with_theta) hipLaunchKernelGGL((k_pair<double, true, TJ, WAVES, IW>), grid, block, 0, st, a, b);
        else hipLaunchKernelGGL((k_pair<double, false, TJ, WAVES, IW>), grid, block, 0, st, a, b);
    } else {
        if (with_theta) hipLaunchKernelGGL((k_pair<float, true, TJ, WAVES, IW>), grid, block, 0, st, a, b);
        else hipLaunchKernelGGL((k_pair<float, false, TJ, WAVES, IW>), grid, block, 0, st, a, b);
    }
}

template <int WAVES, int IW>
void launch_pair_w(const PairLaunch &a, const BondedLaunch &b, int precision, bool with_theta,
                   hipStream_t st)
{
    switch (a.tj) {
    case 16: launch_pair_tj<16, WAVES, IW>(a, b, precision, with_theta, st); break;
    case 32: launch_pair_tj<32, WAVES, IW>(a, b, precision, with_theta, st); break;
    case 64: launch_pair_tj<64, WAVES, IW>(a, b, precision, with_theta, st); break;
    default: launch_pair_tj<0, WAVES, IW>(a, b, precision, with_theta, st); break;
    }
}

// The bonded workgroups alone (a system without pair work, and the
// per-kernel timing).
template <bool THETA>
__global__ __launch_bounds__(64) void k_bonded(BondedLaunch bl)
{
    bonded_block<THETA>(bl, bl.blocks[blockIdx.x], bl.eslot + (long long)blockIdx.x * A_N, nullptr);
}

void launch_bonded(const BondedLaunch &b, bool with_theta, hipStream_t st)
{
    if (b.n_blocks <= 0) return;
    if (with_theta) hipLaunchKernelGGL((k_bonded<true>), dim3(b.n_blocks), dim3(64), 0, st, b);
    else hipLaunchKernelGGL((k_bonded<false>), dim3(b.n_blocks), dim3(64), 0, st, b);
}

void launch_pair(const PairLaunch &a, const BondedLaunch &b, int precision, bool with_theta,
                 hipStream_t st)
{
    if (a.n_items <= 0) {
        launch_bonded(b, with_theta, st);
        return;
    }
    if (a.waves == 2) launch_pair_w<2, 1>(a, b, precision, with_theta, st);
    else if (a.iw == 2) launch_pair_w<1, 2>(a, b, precision, with_theta, st);
    else if (a.iw == 4) launch_pair_w<1, 4>(a, b, precision, with_theta, st);
    else launch_pair_w<1, 1>(a, b, precision, with_theta, st);
}

}  // namespace mixpi
