// Host side of the C-ABI: validation, layout, work lists, constant tables,
// launches and cached HIP graphs for the step loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "mixpi.h"
#include "mixpi_internal.h"

using namespace mixpi;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(MIXPI_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }
int ilog2(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

struct Group {
    int p0, n, N, ele;
    long long row;
};

struct GraphEntry {
    const void *q, *p, *f, *elog;
    int nsteps;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

template <typename T>
int upload(T **dst, const std::vector<T> &v)
{
    *dst = nullptr;
    if (v.empty()) return MIXPI_OK;
    HIP_TRY(hipMalloc((void **)dst, sizeof(T) * v.size()));
    HIP_TRY(hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
    return MIXPI_OK;
}

}  // namespace

struct mixpi_system {
    int device = 0;
    int n_sys = 0;
    int precision = 0, flags = 0;
    long long rows = 0;
    int n_part = 0;
    int n_groups = 0;
    long long candidates = 0;
    std::vector<long long> bead_index;

    SysDev *d_sys = nullptr;
    double *d_lj_eps = nullptr, *d_lj_sig = nullptr;
    double *d_charge = nullptr, *d_fm = nullptr;
    int *d_ljt = nullptr, *d_mol = nullptr, *d_part_sys = nullptr, *d_row_part = nullptr;
    PairBlock *d_blocks = nullptr;
    PairItem *d_items = nullptr;
    int n_items = 0;
    BondTerm *d_bonds = nullptr;
    int n_bonds = 0;
    AngleTerm *d_angles = nullptr;
    int n_angles = 0;
    double *d_bond_k = nullptr, *d_bond_r0 = nullptr, *d_angle_k = nullptr, *d_angle_t0 = nullptr;
    RpItem *d_rp = nullptr;
    int n_rp = 0;
    unsigned rp_lds = 0;
    double *d_basis = nullptr;
    double2 *d_tw = nullptr;
    double *d_prop = nullptr;
    double *d_eacc = nullptr;
    unsigned long long *d_npairs = nullptr;
    unsigned *d_ticket = nullptr;
    int *d_nonfinite = nullptr;
    double *d_cent = nullptr;
    double *d_scratch = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<GraphEntry> graphs;
};

namespace {

void release(mixpi_system *s)
{
    if (!s) return;
    for (auto &g : s->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    void *ptrs[] = {s->d_sys, s->d_lj_eps, s->d_lj_sig, s->d_charge, s->d_fm, s->d_ljt,
                    s->d_mol, s->d_part_sys, s->d_row_part, s->d_blocks, s->d_items,
                    s->d_bonds, s->d_angles, s->d_bond_k, s->d_bond_r0, s->d_angle_k,
                    s->d_angle_t0, s->d_rp, s->d_basis, s->d_tw, s->d_prop, s->d_eacc,
                    s->d_npairs, s->d_ticket, s->d_nonfinite, s->d_cent, s->d_scratch};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    delete s;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int validate(const mixpi_system_desc *d, int idx)
{
    if (!d) return fail(MIXPI_E_INVALID, "system %d: null description", idx);
    const int n = d->n_particles;
    if (n < 1) return fail(MIXPI_E_INVALID, "system %d: n_particles must be >= 1", idx);
    if (!d->n_beads || !d->mass || !d->fict_mass || !d->charge || !d->lj_type || !d->mol_id ||
        !d->is_electron)
        return fail(MIXPI_E_INVALID, "system %d: a per-particle array is null", idx);
    if (d->n_lj_types < 0 || d->n_lj_types > kMaxLjTypes)
        return fail(MIXPI_E_UNSUPPORTED, "system %d: n_lj_types must be in [0, %d]", idx,
                    kMaxLjTypes);
    if (d->n_lj_types > 0 && (!d->lj_eps || !d->lj_sigma))
        return fail(MIXPI_E_INVALID, "system %d: LJ tables are null", idx);
    for (int i = 0; i < n; ++i) {
        const int N = d->n_beads[i];
        if (!is_pow2(N))
            return fail(MIXPI_E_NOT_POW2, "system %d: particle %d has %d beads (not a power of two)",
                        idx, i, N);
        if (N > kMaxBeads)
            return fail(MIXPI_E_UNSUPPORTED, "system %d: particle %d has %d beads (max %d)", idx, i,
                        N, kMaxBeads);
        if (i > 0 && N > d->n_beads[i - 1])
            return fail(MIXPI_E_ORDER,
                        "system %d: bead counts must not increase along the particle list "
                        "(particle %d: %d after %d)",
                        idx, i, N, d->n_beads[i - 1]);
        if (!finite_pos(d->mass[i]) || !finite_pos(d->fict_mass[i]) || !std::isfinite(d->charge[i]))
            return fail(MIXPI_E_INVALID, "system %d: particle %d has a bad mass or charge", idx, i);
        if (d->lj_type[i] < -1 || d->lj_type[i] >= d->n_lj_types)
            return fail(MIXPI_E_INVALID, "system %d: particle %d has LJ type %d", idx, i,
                        d->lj_type[i]);
        if (d->is_electron[i] != 0 && d->is_electron[i] != 1)
            return fail(MIXPI_E_INVALID, "system %d: is_electron must be 0 or 1", idx);
    }
    const int nt = d->n_lj_types;
    for (int k = 0; k < nt * nt; ++k)
        if (!std::isfinite(d->lj_eps[k]) || !finite_pos(d->lj_sigma[k]) ||
            d->lj_eps[k] != d->lj_eps[(k % nt) * nt + k / nt] ||
            d->lj_sigma[k] != d->lj_sigma[(k % nt) * nt + k / nt])
            return fail(MIXPI_E_INVALID, "system %d: LJ tables must be finite and symmetric", idx);
    if (d->n_bonds < 0 || d->n_angles < 0 || d->n_bond_types < 0 || d->n_angle_types < 0)
        return fail(MIXPI_E_INVALID, "system %d: negative topology count", idx);
    if (d->n_bonds > 0 && (!d->bonds || !d->bond_type || !d->bond_k || !d->bond_r0))
        return fail(MIXPI_E_INVALID, "system %d: bond arrays are null", idx);
    if (d->n_angles > 0 && (!d->angles || !d->angle_type || !d->angle_k || !d->angle_t0))
        return fail(MIXPI_E_INVALID, "system %d: angle arrays are null", idx);
    for (int b = 0; b < d->n_bonds; ++b) {
        const int i = d->bonds[2 * b], j = d->bonds[2 * b + 1], t = d->bond_type[b];
        if (i < 0 || i >= n || j < 0 || j >= n || i == j || t < 0 || t >= d->n_bond_types)
            return fail(MIXPI_E_INVALID, "system %d: bond %d is malformed", idx, b);
    }
    for (int a = 0; a < d->n_angles; ++a) {
        const int i = d->angles[3 * a], v = d->angles[3 * a + 1], j = d->angles[3 * a + 2];
        const int t = d->angle_type[a];
        if (i < 0 || i >= n || v < 0 || v >= n || j < 0 || j >= n || i == v || j == v ||
            t < 0 || t >= d->n_angle_types)
            return fail(MIXPI_E_INVALID, "system %d: angle %d is malformed", idx, a);
    }
    for (int k = 0; k < d->n_bond_types; ++k)
        if (!std::isfinite(d->bond_k[k]) || !std::isfinite(d->bond_r0[k]))
            return fail(MIXPI_E_INVALID, "system %d: bond type %d is not finite", idx, k);
    for (int k = 0; k < d->n_angle_types; ++k)
        if (!std::isfinite(d->angle_k[k]) || !std::isfinite(d->angle_t0[k]))
            return fail(MIXPI_E_INVALID, "system %d: angle type %d is not finite", idx, k);
    if (!finite_pos(d->pp_a) || !std::isfinite(d->pp_q) || !finite_pos(d->rc_pp) ||
        !finite_pos(d->rc_coul) || !finite_pos(d->rc_lj))
        return fail(MIXPI_E_INVALID, "system %d: bad pseudopotential or cutoff", idx);
    for (int k = 0; k < 3; ++k)
        if (!finite_pos(d->box[k])) return fail(MIXPI_E_INVALID, "system %d: bad box", idx);
    if (!finite_pos(d->temperature) || !std::isfinite(d->dt))
        return fail(MIXPI_E_INVALID, "system %d: bad temperature or time step", idx);
    if (d->precision != MIXPI_FP64 && d->precision != MIXPI_FP32_ACC64)
        return fail(MIXPI_E_INVALID, "system %d: unknown precision %d", idx, d->precision);
    return MIXPI_OK;
}

// Host tables being assembled for all systems of a handle.
struct Build {
    std::vector<SysDev> sys;
    std::vector<double> lj_eps, lj_sig, charge, fm, bond_k, bond_r0, angle_k, angle_t0;
    std::vector<int> ljt, mol, part_sys, row_part;
    std::vector<PairBlock> blocks;
    std::vector<PairItem> items;
    std::vector<BondTerm> bonds;
    std::vector<AngleTerm> angles;
    std::vector<RpItem> rp_fft, rp_dense;
    std::vector<double> basis, prop;
    std::vector<double2> tw;
    std::map<int, int> basis_off, tw_off;
    std::vector<long long> bead_index;
    long long rows = 0;
    long long candidates = 0;
    int n_part = 0, n_groups = 0;
    unsigned rp_lds = 0;
};

// Orthonormal real normal-mode basis of an N-bead ring, C[j*N + k].
void nm_basis(int N, std::vector<double> &C)
{
    C.assign((size_t)N * N, 0.0);
    for (int j = 0; j < N; ++j)
        for (int k = 0; k < N; ++k) {
            double v;
            if (k == 0) v = 1.0 / std::sqrt((double)N);
            else if (2 * k < N) v = std::sqrt(2.0 / N) * std::cos(2.0 * kPi * ((long long)j * k % N) / N);
            else if (2 * k == N) v = (j % 2 ? -1.0 : 1.0) / std::sqrt((double)N);
            else v = std::sqrt(2.0 / N) * std::sin(2.0 * kPi * ((long long)j * k % N) / N);
            C[(size_t)j * N + k] = v;
        }
}

void add_system(Build &B, const mixpi_system_desc *d, int s)
{
    const int n = d->n_particles;
    const int p_base = B.n_part;
    const long long row_base = B.rows;
    const int nt = d->n_lj_types, nt1 = nt + 1;
    const double beta = 1.0 / (kBoltz * d->temperature);
    const double bh = beta * kHbar;
    const double kT = kBoltzKcal * d->temperature;

    SysDev S{};
    long long beads = 0;
    for (int i = 0; i < n; ++i) beads += d->n_beads[i];
    double Q = 0.0;
    for (int i = 0; i < n; ++i)
        if (!d->is_electron[i]) Q += d->charge[i];
    for (int k = 0; k < 3; ++k) {
        S.box[k] = d->box[k];
        S.ibox[k] = 1.0 / d->box[k];
    }
    S.rc_lj = d->rc_lj;
    S.rc_c = d->rc_coul;
    S.rc_pp = d->rc_pp;
    S.theta0[0] = d->pp_q;
    S.theta0[1] = d->pp_a;
    S.theta0[2] = nt > 0 ? d->lj_eps[0] : 0.0;
    S.theta0[3] = nt > 0 ? d->lj_sigma[0] : 1.0;
    S.theta0[4] = d->n_bond_types > 0 ? d->bond_k[0] : 0.0;
    S.theta0[5] = d->n_angle_types > 0 ? d->angle_k[0] : 0.0;
    const double V = d->box[0] * d->box[1] * d->box[2];
    S.bg_energy = d->background ? -kPi * kCoulombKcal * d->rc_coul * d->rc_coul * Q * Q / (5.0 * V)
                                : 0.0;
    S.kT = kT;
    S.cv_const = 1.5 * n * kT;
    S.prim_const = 1.5 * (double)beads * kT;
    S.hkick = 0.5 * d->dt * kKcal;
    S.lj_off = (int)B.lj_eps.size();
    S.nt1 = nt1;
    S.bond_off = (int)B.bond_k.size();
    S.angle_off = (int)B.angle_k.size();
    B.sys.push_back(S);

    for (int a = 0; a < nt1; ++a)
        for (int b = 0; b < nt1; ++b) {
            const bool real = a < nt && b < nt;
            B.lj_eps.push_back(real ? d->lj_eps[a * nt + b] : 0.0);
            B.lj_sig.push_back(real ? d->lj_sigma[a * nt + b] : 1.0);
        }
    for (int k = 0; k < d->n_bond_types; ++k) {
        B.bond_k.push_back(d->bond_k[k]);
        B.bond_r0.push_back(d->bond_r0[k]);
    }
    for (int k = 0; k < d->n_angle_types; ++k) {
        B.angle_k.push_back(d->angle_k[k]);
        B.angle_t0.push_back(d->angle_t0[k]);
    }
    for (int i = 0; i < n; ++i) {
        B.charge.push_back(d->charge[i]);
        B.fm.push_back(d->fict_mass[i]);
        B.ljt.push_back(d->lj_type[i] < 0 ? nt : d->lj_type[i]);
        B.mol.push_back(d->mol_id[i]);
        B.part_sys.push_back(s);
    }

    // groups: maximal runs of equal bead count and electron flag
    std::vector<Group> groups;
    long long row = row_base;
    for (int i = 0; i < n;) {
        int j = i;
        while (j < n && d->n_beads[j] == d->n_beads[i] && d->is_electron[j] == d->is_electron[i]) ++j;
        Group g{i, j - i, d->n_beads[i], d->is_electron[i], row};
        row += (long long)g.N * g.n;
        groups.push_back(g);
        i = j;
    }
    B.n_groups += (int)groups.size();

    // layout: bead index and row -> particle
    std::vector<long long> part_first(n);
    {
        long long acc = 0;
        for (int i = 0; i < n; ++i) {
            part_first[i] = acc;
            acc += d->n_beads[i];
        }
    }
    std::vector<long long> rows_of(beads);
    B.row_part.resize(row - 0, -1);
    for (const Group &g : groups)
        for (int a = 0; a < g.N; ++a)
            for (int i = 0; i < g.n; ++i) {
                const long long r = g.row + (long long)a * g.n + i;
                rows_of[part_first[g.p0 + i] + a] = r;
                B.row_part[r] = p_base + g.p0 + i;
            }
    B.bead_index.insert(B.bead_index.end(), rows_of.begin(), rows_of.end());
    auto bead_row = [&](int i, int a) { return rows_of[part_first[i] + a]; };

    // nonbonded pair blocks and 64 x 64 tiles
    for (size_t ga = 0; ga < groups.size(); ++ga)
        for (size_t gb = ga; gb < groups.size(); ++gb) {
            const Group &A = groups[ga], &Bg = groups[gb];
            if (A.ele && Bg.ele) continue;
            PairBlock pb{};
            pb.sys = s;
            pb.kind = (!A.ele && !Bg.ele) ? PK_ATOM : (A.ele ? PK_E_ATOM : PK_ATOM_E);
            pb.same = ga == gb;
            pb.shift = ilog2(A.N / Bg.N);
            pb.na = A.n;
            pb.nb = Bg.n;
            pb.pa0 = p_base + A.p0;
            pb.pb0 = p_base + Bg.p0;
            pb.rowa = A.row;
            pb.rowb = Bg.row;
            pb.w = 1.0 / A.N;
            const int bi = (int)B.blocks.size();
            B.blocks.push_back(pb);
            const long long li = (long long)A.n << pb.shift;
            for (int b = 0; b < Bg.N; ++b)
                for (long long i0 = 0; i0 < li; i0 += kPairTile)
                    for (int j0 = 0; j0 < Bg.n; j0 += kPairTile) {
                        if (pb.same && j0 < i0) continue;
                        B.items.push_back(PairItem{bi, b, (int)i0, j0});
                    }
            const long long pairs = pb.same ? (long long)A.n * (A.n - 1) / 2 : (long long)A.n * Bg.n;
            B.candidates += pairs * A.N;
        }
    {   // excluded pairs (equal mol id) do not count as candidates
        std::map<int, std::vector<int>> by_mol;
        for (int i = 0; i < n; ++i) by_mol[d->mol_id[i]].push_back(i);
        for (auto &kv : by_mol) {
            const auto &v = kv.second;
            for (size_t x = 0; x < v.size(); ++x)
                for (size_t y = x + 1; y < v.size(); ++y) {
                    if (d->is_electron[v[x]] && d->is_electron[v[y]]) continue;
                    B.candidates -= std::max(d->n_beads[v[x]], d->n_beads[v[y]]);
                }
        }
    }

    // bonded terms: one entry per (term, slice), beads resolved here
    for (int b = 0; b < d->n_bonds; ++b) {
        const int i = d->bonds[2 * b], j = d->bonds[2 * b + 1];
        const int Ni = d->n_beads[i], Nj = d->n_beads[j], Nm = std::max(Ni, Nj);
        for (int sl = 0; sl < Nm; ++sl)
            B.bonds.push_back(BondTerm{(int)bead_row(i, (int)((long long)sl * Ni / Nm)),
                                       (int)bead_row(j, (int)((long long)sl * Nj / Nm)),
                                       S.bond_off + d->bond_type[b], s, 1.0 / Nm});
    }
    for (int a = 0; a < d->n_angles; ++a) {
        const int i = d->angles[3 * a], v = d->angles[3 * a + 1], j = d->angles[3 * a + 2];
        const int Ni = d->n_beads[i], Nv = d->n_beads[v], Nj = d->n_beads[j];
        const int Nm = std::max(Ni, std::max(Nv, Nj));
        for (int sl = 0; sl < Nm; ++sl)
            B.angles.push_back(AngleTerm{(int)bead_row(i, (int)((long long)sl * Ni / Nm)),
                                         (int)bead_row(v, (int)((long long)sl * Nv / Nm)),
                                         (int)bead_row(j, (int)((long long)sl * Nj / Nm)),
                                         S.angle_off + d->angle_type[a], s, 0, 1.0 / Nm});
    }

    // normal modes: propagator coefficients per (mode row, particle)
    B.prop.resize((size_t)5 * row, 0.0);
    for (const Group &g : groups) {
        const int N = g.N;
        for (int i = 0; i < g.n; ++i) {
            const int p = g.p0 + i;
            const double ksp = N * d->mass[p] / (bh * bh);   // amu / fs^2
            const double mf = d->fict_mass[p];
            for (int k = 0; k < N; ++k) {
                const double sn = std::sin(kPi * k / N);
                const double lam = 4.0 * sn * sn;
                const double w = std::sqrt(ksp * lam / mf);
                double *pr = &B.prop[5 * (size_t)(g.row + (long long)k * g.n + i)];
                if (k == 0 || w == 0.0) {
                    pr[0] = 1.0;
                    pr[1] = d->dt / mf;
                    pr[2] = 0.0;
                    pr[3] = 1.0;
                } else {
                    const double c = std::cos(w * d->dt), sw = std::sin(w * d->dt);
                    pr[0] = c;
                    pr[1] = sw / (mf * w);
                    pr[2] = -mf * w * sw;
                    pr[3] = c;
                }
                pr[4] = 0.5 * ksp * lam / kKcal;
            }
        }
        if (N <= kDenseMaxN) {
            if (!B.basis_off.count(N)) {
                std::vector<double> C;
                nm_basis(N, C);
                B.basis_off[N] = (int)B.basis.size();
                B.basis.insert(B.basis.end(), C.begin(), C.end());
                for (int k = 0; k < N; ++k)
                    for (int j = 0; j < N; ++j) B.basis.push_back(C[(size_t)j * N + k]);
            }
            const int CB = 256 / N;
            for (int c0 = 0; c0 < 3 * g.n; c0 += CB) {
                RpItem it{};
                it.kind = RP_DENSE;
                it.sys = s;
                it.N = N;
                it.logN = ilog2(N);
                it.n = g.n;
                it.p0 = p_base + g.p0;
                it.row = g.row;
                it.c0 = c0;
                it.ncols = std::min(CB, 3 * g.n - c0);
                it.basis_off = B.basis_off[N];
                B.rp_dense.push_back(it);
            }
            B.rp_lds = std::max(B.rp_lds, (unsigned)((2 * N * N + 4 * 256) * sizeof(double)));
        } else {
            if (!B.tw_off.count(N)) {
                B.tw_off[N] = (int)B.tw.size();
                for (int m = 0; m < N / 2; ++m)
                    B.tw.push_back(make_double2(std::cos(2.0 * kPi * m / N), -std::sin(2.0 * kPi * m / N)));
            }
            for (int c = 0; c < 3 * g.n; ++c) {
                RpItem it{};
                it.kind = RP_FFT;
                it.sys = s;
                it.N = N;
                it.logN = ilog2(N);
                it.n = g.n;
                it.p0 = p_base + g.p0;
                it.row = g.row;
                it.c0 = c;
                it.ncols = 1;
                it.tw_off = B.tw_off[N];
                B.rp_fft.push_back(it);
            }
            B.rp_lds = std::max(B.rp_lds, (unsigned)(N * sizeof(double2)));
        }
    }
    B.rows = row;
    B.n_part += n;
}

int create_impl(const mixpi_system_desc *const *descs, int n_sys, mixpi_system **out)
{
    if (!out) return fail(MIXPI_E_INVALID, "out is null");
    *out = nullptr;
    if (!descs || n_sys < 1) return fail(MIXPI_E_INVALID, "need at least one system");
    for (int s = 0; s < n_sys; ++s) {
        int rc = validate(descs[s], s);
        if (rc) return rc;
        if (descs[s]->precision != descs[0]->precision || descs[s]->flags != descs[0]->flags)
            return fail(MIXPI_E_INVALID, "all systems of a batch must share precision and flags");
    }
    Build B;
    for (int s = 0; s < n_sys; ++s) add_system(B, descs[s], s);
    if (B.rows > (1LL << 31) / 3)
        return fail(MIXPI_E_UNSUPPORTED, "too many beads (%lld)", B.rows);

    mixpi_system *S = new mixpi_system();
    int rc = MIXPI_OK;
    auto T = [&](int r) {
        if (r && !rc) rc = r;
    };
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return fail(MIXPI_E_HIP, "hipGetDevice failed (no GPU?)");
    }
    S->n_sys = n_sys;
    S->precision = descs[0]->precision;
    S->flags = descs[0]->flags;
    S->rows = B.rows;
    S->n_part = B.n_part;
    S->n_groups = B.n_groups;
    S->candidates = B.candidates;
    S->bead_index = B.bead_index;
    S->n_items = (int)B.items.size();
    S->n_bonds = (int)B.bonds.size();
    S->n_angles = (int)B.angles.size();
    std::vector<RpItem> rp = B.rp_fft;
    rp.insert(rp.end(), B.rp_dense.begin(), B.rp_dense.end());
    S->n_rp = (int)rp.size();
    S->rp_lds = B.rp_lds;

    T(upload(&S->d_sys, B.sys));
    T(upload(&S->d_lj_eps, B.lj_eps));
    T(upload(&S->d_lj_sig, B.lj_sig));
    T(upload(&S->d_charge, B.charge));
    T(upload(&S->d_fm, B.fm));
    T(upload(&S->d_ljt, B.ljt));
    T(upload(&S->d_mol, B.mol));
    T(upload(&S->d_part_sys, B.part_sys));
    T(upload(&S->d_row_part, B.row_part));
    T(upload(&S->d_blocks, B.blocks));
    T(upload(&S->d_items, B.items));
    T(upload(&S->d_bonds, B.bonds));
    T(upload(&S->d_angles, B.angles));
    T(upload(&S->d_bond_k, B.bond_k));
    T(upload(&S->d_bond_r0, B.bond_r0));
    T(upload(&S->d_angle_k, B.angle_k));
    T(upload(&S->d_angle_t0, B.angle_t0));
    T(upload(&S->d_rp, rp));
    T(upload(&S->d_basis, B.basis));
    T(upload(&S->d_tw, B.tw));
    T(upload(&S->d_prop, B.prop));
    T(upload(&S->d_eacc, std::vector<double>((size_t)n_sys * kAccCopies * A_N, 0.0)));
    T(upload(&S->d_npairs, std::vector<unsigned long long>(2 * kAccCopies, 0ull)));
    T(upload(&S->d_ticket, std::vector<unsigned>(1, 0u)));
    T(upload(&S->d_nonfinite, std::vector<int>(1, 0)));
    T(upload(&S->d_cent, std::vector<double>((size_t)3 * B.n_part, 0.0)));
    T(upload(&S->d_scratch, std::vector<double>((size_t)9 * B.rows, 0.0)));
    if (!rc) {
        hipError_t e = hipStreamCreateWithFlags(&S->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) rc = fail(MIXPI_E_HIP, "hipStreamCreate: %s", hipGetErrorString(e));
    }
    if (!rc) {
        hipError_t e = hipFuncSetAttribute(rp_kernel_symbol(), hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)std::max<unsigned>(S->rp_lds, 1024));
        if (e != hipSuccess) rc = fail(MIXPI_E_HIP, "hipFuncSetAttribute: %s", hipGetErrorString(e));
    }
    if (rc) {
        std::string msg = g_err;
        release(S);
        g_err = msg;
        return rc;
    }
    *out = S;
    return MIXPI_OK;
}

int check_sys(const mixpi_system *s)
{
    if (!s) return fail(MIXPI_E_INVALID, "system handle is null");
    return MIXPI_OK;
}

PairLaunch pair_args(mixpi_system *s, const double *q, double *f, const double *theta)
{
    PairLaunch a{};
    a.items = s->d_items;
    a.n_items = s->n_items;
    a.blocks = s->d_blocks;
    a.sys = s->d_sys;
    a.lj_eps = s->d_lj_eps;
    a.lj_sig = s->d_lj_sig;
    a.charge = s->d_charge;
    a.ljt = s->d_ljt;
    a.mol = s->d_mol;
    a.q = q;
    a.f = f;
    a.theta = theta;
    a.eacc = s->d_eacc;
    a.npairs = s->d_npairs;
    return a;
}

BondedLaunch bonded_args(mixpi_system *s, const double *q, double *f, const double *theta)
{
    BondedLaunch b{};
    b.bonds = s->d_bonds;
    b.n_bonds = s->n_bonds;
    b.angles = s->d_angles;
    b.n_angles = s->n_angles;
    b.sys = s->d_sys;
    b.bond_k = s->d_bond_k;
    b.bond_r0 = s->d_bond_r0;
    b.angle_k = s->d_angle_k;
    b.angle_t0 = s->d_angle_t0;
    b.q = q;
    b.f = f;
    b.theta = theta;
    b.eacc = s->d_eacc;
    return b;
}

// Enqueues F(q) (zeroed first) and the potential accumulators.
void enqueue_forces(mixpi_system *s, const double *q, const double *theta, double *f,
                    bool with_theta, hipStream_t st)
{
    launch_fill(f, 3 * s->rows, 0.0, st);
    launch_pair(pair_args(s, q, f, theta), s->precision, with_theta, st);
    launch_bonded(bonded_args(s, q, f, theta), with_theta, st);
}

int last_launch_error()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MIXPI_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return MIXPI_OK;
}

RpLaunch rp_step_args(mixpi_system *s, double *q, double *p, double *f)
{
    RpLaunch r{};
    r.items = s->d_rp;
    r.n_items = s->n_rp;
    r.sys = s->d_sys;
    r.basis = s->d_basis;
    r.twiddle = s->d_tw;
    r.prop = s->d_prop;
    r.op = OP_STEP;
    r.in_q = q;
    r.out_q = q;
    r.p = p;
    r.f = f;
    r.cent = s->d_cent;
    r.eacc = s->d_eacc;
    r.lds_bytes = s->rp_lds;
    return r;
}

FinishLaunch finish_args(mixpi_system *s, double *q, double *p, double *f, double *elog_row)
{
    FinishLaunch fl{};
    fl.n3 = 3 * s->rows;
    fl.row_part = s->d_row_part;
    fl.part_sys = s->d_part_sys;
    fl.fm = s->d_fm;
    fl.sys = s->d_sys;
    fl.n_sys = s->n_sys;
    fl.p = p;
    fl.f = f;
    fl.q = q;
    fl.cent = s->d_cent;
    fl.eacc = s->d_eacc;
    fl.elog = elog_row;
    fl.ticket = s->d_ticket;
    fl.nonfinite = s->d_nonfinite;
    return fl;
}

// One step: free ring polymers (with the first half-kick and F := 0), pair
// and bonded forces, second half-kick with the energy-log row.
void enqueue_step(mixpi_system *s, double *q, double *p, double *f, double *elog_row,
                  hipStream_t st)
{
    launch_rp(rp_step_args(s, q, p, f), st);
    launch_pair(pair_args(s, q, f, nullptr), s->precision, false, st);
    launch_bonded(bonded_args(s, q, f, nullptr), false, st);
    launch_finish(finish_args(s, q, p, f, elog_row), st);
}

// Finds or captures the graph of nsteps steps for these pointers.
int step_graph(mixpi_system *sys, int nsteps, double *q, double *p, double *f, double *elog,
               GraphEntry **out)
{
    *out = nullptr;
    if (int rc = check_sys(sys)) return rc;
    if (nsteps < 0) return fail(MIXPI_E_INVALID, "nsteps must be >= 0");
    if (!q || !p || !f) return fail(MIXPI_E_INVALID, "q, p and f must be non-null");
    if (q == p || q == f || p == f) return fail(MIXPI_E_INVALID, "q, p and f must be distinct");
    if (nsteps == 0) return MIXPI_OK;
    HIP_TRY(hipSetDevice(sys->device));
    for (auto &g : sys->graphs)
        if (g.q == q && g.p == p && g.f == f && g.elog == elog && g.nsteps == nsteps) {
            *out = &g;
            return MIXPI_OK;
        }
    if (sys->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(sys->graphs.front().exec);
        (void)hipGraphDestroy(sys->graphs.front().graph);
        sys->graphs.erase(sys->graphs.begin());
    }
    GraphEntry g{q, p, f, elog, nsteps, nullptr, nullptr};
    HIP_TRY(hipStreamBeginCapture(sys->cap_stream, hipStreamCaptureModeRelaxed));
    for (int k = 0; k < nsteps; ++k)
        enqueue_step(sys, q, p, f, elog ? elog + (size_t)k * sys->n_sys * MIXPI_NE : nullptr,
                     sys->cap_stream);
    HIP_TRY(hipStreamEndCapture(sys->cap_stream, &g.graph));
    hipError_t e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g.graph);
        return fail(MIXPI_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    sys->graphs.push_back(g);
    *out = &sys->graphs.back();
    return MIXPI_OK;
}

}  // namespace

extern "C" {

const char *mixpi_last_error(void) { return g_err.c_str(); }

int mixpi_create(const mixpi_system_desc *desc, mixpi_system **out)
{
    const mixpi_system_desc *d[1] = {desc};
    return create_impl(d, 1, out);
}

int mixpi_batch_create(const mixpi_system_desc *const *descs, int32_t n, mixpi_system **out)
{
    return create_impl(descs, n, out);
}

int mixpi_destroy(mixpi_system *sys)
{
    if (!sys) return MIXPI_OK;
    (void)hipSetDevice(sys->device);
    (void)hipDeviceSynchronize();
    release(sys);
    return MIXPI_OK;
}

int mixpi_sizes(const mixpi_system *sys, int64_t *n_bead_rows, int32_t *n_particles,
                int32_t *n_groups, int32_t *n_systems)
{
    if (int rc = check_sys(sys)) return rc;
    if (n_bead_rows) *n_bead_rows = sys->rows;
    if (n_particles) *n_particles = sys->n_part;
    if (n_groups) *n_groups = sys->n_groups;
    if (n_systems) *n_systems = sys->n_sys;
    return MIXPI_OK;
}

int mixpi_bead_index(const mixpi_system *sys, int64_t *rows_out)
{
    if (int rc = check_sys(sys)) return rc;
    if (!rows_out) return fail(MIXPI_E_INVALID, "rows_out is null");
    std::copy(sys->bead_index.begin(), sys->bead_index.end(), rows_out);
    return MIXPI_OK;
}

int mixpi_forces(mixpi_system *sys, const double *q, const double *theta, double *f,
                 double *e_out, void *stream)
{
    if (int rc = check_sys(sys)) return rc;
    if (!q || !f) return fail(MIXPI_E_INVALID, "q and f must be non-null");
    if ((const void *)q == (const void *)f) return fail(MIXPI_E_INVALID, "f must not alias q");
    HIP_TRY(hipSetDevice(sys->device));
    hipStream_t st = (hipStream_t)stream;
    enqueue_forces(sys, q, theta, f, false, st);
    launch_write_energy(sys->d_sys, sys->n_sys, sys->d_eacc, e_out, st);
    return last_launch_error();
}

int mixpi_energy(mixpi_system *sys, const double *q, const double *theta, double *e_out,
                 void *stream)
{
    if (int rc = check_sys(sys)) return rc;
    if (!q || !e_out) return fail(MIXPI_E_INVALID, "q and e_out must be non-null");
    HIP_TRY(hipSetDevice(sys->device));
    hipStream_t st = (hipStream_t)stream;
    enqueue_forces(sys, q, theta, sys->d_scratch, false, st);
    launch_write_energy(sys->d_sys, sys->n_sys, sys->d_eacc, e_out, st);
    return last_launch_error();
}

int mixpi_energy_adjoint(mixpi_system *sys, const double *q, const double *theta,
                         const double *grad_e, double *dq, double *dtheta, void *stream)
{
    if (int rc = check_sys(sys)) return rc;
    if (!q) return fail(MIXPI_E_INVALID, "q must be non-null");
    if ((const void *)q == (const void *)dq) return fail(MIXPI_E_INVALID, "dq must not alias q");
    HIP_TRY(hipSetDevice(sys->device));
    hipStream_t st = (hipStream_t)stream;
    double *target = dq ? dq : sys->d_scratch;
    enqueue_forces(sys, q, theta, target, true, st);
    launch_adjoint_finish(sys->d_sys, sys->n_sys, sys->rows, sys->d_row_part, sys->d_part_sys,
                          grad_e, dq, sys->d_eacc, dtheta, st);
    return last_launch_error();
}

int mixpi_nm_transform(mixpi_system *sys, int32_t dir, const double *in, double *out,
                       void *stream)
{
    if (int rc = check_sys(sys)) return rc;
    if (dir != 1 && dir != -1) return fail(MIXPI_E_INVALID, "dir must be +1 or -1");
    if (!in || !out) return fail(MIXPI_E_INVALID, "in and out must be non-null");
    if ((const void *)in == (const void *)out) return fail(MIXPI_E_INVALID, "out must not alias in");
    HIP_TRY(hipSetDevice(sys->device));
    RpLaunch r{};
    r.items = sys->d_rp;
    r.n_items = sys->n_rp;
    r.sys = sys->d_sys;
    r.basis = sys->d_basis;
    r.twiddle = sys->d_tw;
    r.prop = sys->d_prop;
    r.op = dir > 0 ? OP_FWD : OP_BWD;
    r.in_q = in;
    r.out_q = out;
    r.lds_bytes = sys->rp_lds;
    launch_rp(r, (hipStream_t)stream);
    return last_launch_error();
}

int mixpi_step_prepare(mixpi_system *sys, int32_t nsteps, double *q, double *p, double *f,
                       double *elog)
{
    GraphEntry *ge = nullptr;
    return step_graph(sys, nsteps, q, p, f, elog, &ge);
}

int mixpi_step(mixpi_system *sys, int32_t nsteps, double *q, double *p, double *f, double *elog,
               void *stream)
{
    GraphEntry *ge = nullptr;
    if (int rc = step_graph(sys, nsteps, q, p, f, elog, &ge)) return rc;
    if (!ge) return MIXPI_OK;
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipGraphLaunch(ge->exec, st));
    if (sys->flags & MIXPI_FLAG_CHECK_FINITE) {
        int flag = 0;
        HIP_TRY(hipMemcpyAsync(&flag, sys->d_nonfinite, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (flag) {
            const int zero = 0;
            HIP_TRY(hipMemcpy(sys->d_nonfinite, &zero, sizeof(int), hipMemcpyHostToDevice));
            return fail(MIXPI_E_NONFINITE, "non-finite energy during mixpi_step");
        }
    }
    return MIXPI_OK;
}

int mixpi_kernel_time(mixpi_system *sys, int32_t which, int32_t reps, const double *q,
                      const double *p, double *avg_us, void *stream)
{
    if (int rc = check_sys(sys)) return rc;
    if (which < 0 || which > 3) return fail(MIXPI_E_INVALID, "which must be 0..3");
    if (reps < 1 || !q || !p || !avg_us) return fail(MIXPI_E_INVALID, "bad arguments");
    HIP_TRY(hipSetDevice(sys->device));
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = sizeof(double) * 3 * sys->rows;
    double *sq = sys->d_scratch, *sp = sq + 3 * sys->rows, *sf = sp + 3 * sys->rows;
    HIP_TRY(hipMemcpyAsync(sq, q, bytes, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(sp, p, bytes, hipMemcpyDeviceToDevice, st));
    enqueue_forces(sys, sq, nullptr, sf, false, st);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) {
        if (which == 0) launch_pair(pair_args(sys, sq, sf, nullptr), sys->precision, false, st);
        else if (which == 1) launch_bonded(bonded_args(sys, sq, sf, nullptr), false, st);
        else if (which == 2) launch_rp(rp_step_args(sys, sq, sp, sf), st);
        else launch_finish(finish_args(sys, sq, sp, sf, nullptr), st);
    }
    HIP_TRY(hipEventRecord(e1, st));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_us = 1000.0 * ms / reps;
    // leave the accumulators and counters as they were before the call
    launch_write_energy(sys->d_sys, sys->n_sys, sys->d_eacc, nullptr, st);
    HIP_TRY(hipStreamSynchronize(st));
    return last_launch_error();
}

int mixpi_pair_candidates(const mixpi_system *sys, int64_t *candidates)
{
    if (int rc = check_sys(sys)) return rc;
    if (!candidates) return fail(MIXPI_E_INVALID, "candidates is null");
    *candidates = sys->candidates;
    return MIXPI_OK;
}

int mixpi_pair_evals(mixpi_system *sys, int64_t *evals, int32_t reset, void *stream)
{
    if (int rc = check_sys(sys)) return rc;
    HIP_TRY(hipSetDevice(sys->device));
    hipStream_t st = (hipStream_t)stream;
    unsigned long long h[2 * kAccCopies];
    HIP_TRY(hipMemcpyAsync(h, sys->d_npairs, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    unsigned long long tot[2] = {0, 0};
    for (int c = 0; c < 2 * kAccCopies; ++c) tot[c / kAccCopies] += h[c];
    if (evals) {
        evals[0] = (int64_t)tot[0];
        evals[1] = (int64_t)tot[1];
    }
    if (reset) {
        HIP_TRY(hipMemsetAsync(sys->d_npairs, 0, sizeof h, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    return MIXPI_OK;
}

}  // extern "C"
