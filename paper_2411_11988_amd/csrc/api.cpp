// Host side of the C-ABI: validation, layout, work lists, constant tables,
// launches and cached HIP graphs for the step loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdlib>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "mixpi.h"
#include "mixpi_internal.h"

using namespace mixpi;

static_assert(kStaticScratchBytes == MIXPI_STATIC_SCRATCH_BYTES,
              "the static scratch size and its public constant must agree");

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
    const void *noise = nullptr;   // thermostatted sequences: their noise
    int mode = 0;                  // NVE split propagator, thermostatted, velocity Verlet
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

template <typename T>
int alloc(T **dst, size_t n)
{
    *dst = nullptr;
    if (n == 0) return MIXPI_OK;
    HIP_TRY(hipMalloc((void **)dst, sizeof(T) * n));
    return MIXPI_OK;
}

}  // namespace

struct mixpi_system {
    int device = 0;
    int n_sys = 0;
    int precision = 0, flags = 0;
    long long rows = 0;
    int n_part = 0, n_groups = 0;
    long long candidates = 0;
    std::vector<long long> bead_index;
    std::vector<long long> layout;              // per group: first row, N, n, first particle, system
    std::vector<long long> sys_row0;            // first row of each system, then the row count
    double *d_bstage = nullptr;                 // mixpi_batch_step staging: q, p, f [rows][3] each
    std::vector<int> pair_tj;                   // j-tile width of each system's items
    int pair_tj_all = 0;                        // their common width, 0 if they differ
    int pair_waves = 1;                         // j-split waves per pair tile
    int pair_iw = 1;                            // i-split waves per pair tile
    int pair_jrun = 1;                          // most j-tiles per pair item

    SysDev *d_sys = nullptr;
    LjPar *d_ljpar = nullptr;                   // LJ tables in the pair sweep's form
    double *d_charge = nullptr;
    int *d_ljt = nullptr, *d_mol = nullptr, *d_row_sys = nullptr;
    double *d_row_fm = nullptr, *d_row_hk = nullptr;
    // pair sweep: items in system and block order
    PairBlock *d_blocks = nullptr;
    PairItem *d_items = nullptr;
    PairBlock *d_iblocks = nullptr;             // the block of every item
    int n_items = 0;
    // radial distribution: the pair blocks' 64 x 64 tiles in system-pure runs,
    // largest bead count
    PairItem *d_rdf_items = nullptr;
    BlockRange *d_rdf_ranges = nullptr;
    int n_rdf_ranges = 0, top_beads = 1, max_nt1 = 1;
    // centroid quantities: particles in handle order, first particle per system
    PartDev *d_parts = nullptr;
    unsigned char *d_pspec = nullptr;          // species of every particle (correlation sums)
    int *d_sys_part = nullptr;
    std::vector<PartDev> h_parts;
    std::vector<int> h_sys_part;
    std::vector<double> h_ew_z;
    // centroid Ewald electrostatics (mixpi_set_ewald)
    struct Ewald {
        bool on = false;
        double alpha = 0, r_cut = 0, scale = 1;
        int K = 0, logK = 0, order = 0, recip_wg = 1, n_real = 0;
        double *z = nullptr, *cpos = nullptr, *freal = nullptr, *fcent = nullptr, *G = nullptr;
        double *rowf = nullptr;   // [rows][3] bead forces for the step's epilogue
        int *spl_base = nullptr;
        double *spl_w = nullptr;
        double2 *grid_c = nullptr, *tw = nullptr;
        double *e_real_part = nullptr, *e_recip_part = nullptr, *e_const = nullptr;
        RealItem *real_items = nullptr;
        int *real_first = nullptr;
    } ew;
    // bonded sweep: terms and system-pure blocks of 256 (fast blocks first)
    BondedTerm *d_bterms = nullptr;
    BlockRange *d_bblocks = nullptr;
    int n_bblocks = 0, n_bblocks_fast = 0;
    double *d_bond_k = nullptr, *d_bond_r0 = nullptr, *d_angle_k = nullptr, *d_angle_t0 = nullptr;
    // normal modes: dense items first, then FFT items
    RpItem *d_rp = nullptr;       // items of the step
    RpItem *d_rp_nm = nullptr;    // items of the normal-mode transforms
    RpItem *d_rp_lang = nullptr;  // items of the Langevin and velocity-Verlet launches
    int n_rp = 0, n_rp_fast = 0, n_rp_nm = 0, n_rp_lang = 0;
    // matrix-core items: columns, generator tables, step items; spring
    // weights of the rows they propagate (epilogue)
    MfmaCol *d_mf_cols = nullptr;
    double *d_mf_tab = nullptr;
    double *d_row_spw = nullptr;
    int n_mf_step = 0;
    double *d_circ = nullptr;
    // circulant rings' stage rows: q and p + dt/2 F of each of their bead rows
    double *d_stage = nullptr;
    int *d_row_stage = nullptr;
    long long *d_stage_rows = nullptr;
    int n_stage = 0;
    // thermostat: Langevin coefficients per mode row, and the host data to build them
    double *d_lang = nullptr;
    bool lang_set = false;
    std::vector<double> h_prop, h_row_fm;
    std::vector<int> h_row_sys;
    std::vector<SysDev> h_sys;
    // dynamic LDS: largest, step items, transform items, Langevin / VV items
    unsigned rp_lds = 0, rp_lds_step = 0, rp_lds_nm = 0, rp_lds_lang = 0;
    double *d_basis = nullptr;
    double2 *d_tw = nullptr;
    double *d_prop = nullptr;
    // partial forces and their per-row gather lists
    long long *d_row_ptr = nullptr;
    int *d_dest = nullptr;
    double *d_part = nullptr;
    long long n_slots = 0, part_bonded = 0;
    long long n_positions = 0;     // partial-force positions (CSR entries of all rows)
    // epilogue blocks (4 rows of one system)
    BlockRange *d_fblocks = nullptr;
    int n_fblocks = 0;
    int fin_rpw = 1;               // bead rows per wave in the epilogue
    // energy slots (two buffers, alternating by step): pair items | bonded
    // blocks | normal-mode items | epilogue blocks; per-system slot lists for
    // the force-only range and for the whole step
    double *d_eslot = nullptr;
    // reducer plans: the force-only slots [0, e_rp) and the whole step
    int *d_red_f = nullptr, *d_red_a = nullptr;   // packed chunk_begin | chunk_len | sys_chunk
    int *d_red_v = nullptr;                       // the same for velocity-Verlet steps
    int red_f_off[3] = {0, 0, 0}, red_a_off[3] = {0, 0, 0}, red_v_off[3] = {0, 0, 0};
    int nch_f = 0, nch_a = 0, nch_v = 0;          // chunks of each list
    // the same three lists with the centroid-Ewald slots (one per system)
    int *d_red_fE = nullptr, *d_red_aE = nullptr, *d_red_vE = nullptr;
    int red_fE_off[3] = {0, 0, 0}, red_aE_off[3] = {0, 0, 0}, red_vE_off[3] = {0, 0, 0};
    int nch_fE = 0, nch_aE = 0, nch_vE = 0;
    int e_ew = 0;                                 // first centroid-Ewald slot
    bool ew_use = false;                          // mixpi_use_ewald
    long long *d_row_prev = nullptr, *d_row_next = nullptr;
    double *d_row_ksp = nullptr;
    double *d_partial = nullptr;      // [max chunks][A_N] stage-A sums
    int n_eslots = 0, e_bonded = 0, e_rp = 0, e_fin = 0;

    unsigned long long *d_npairs = nullptr;
    int *d_nonfinite = nullptr;
    double *d_cent = nullptr;
    double *d_scratch = nullptr;
    hipStream_t cap_stream = nullptr;
    std::vector<GraphEntry> graphs;
};

namespace {

// Drops every captured step graph (their launches hold pointers and
// settings that are about to change).
void clear_graphs(mixpi_system *s)
{
    for (auto &g : s->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    s->graphs.clear();
}

void release_ewald(mixpi_system *s)
{
    auto &e = s->ew;
    void *ptrs[] = {e.z, e.cpos, e.freal, e.fcent, e.G, e.spl_base, e.spl_w, e.grid_c, e.tw, e.rowf,
                    e.e_real_part, e.e_recip_part, e.e_const, e.real_items, e.real_first};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    e = mixpi_system::Ewald{};
}

void release(mixpi_system *s)
{
    if (!s) return;
    release_ewald(s);
    for (auto &g : s->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    void *ptrs[] = {s->d_sys, s->d_ljpar, s->d_charge, s->d_ljt, s->d_mol,
                    s->d_row_sys, s->d_row_fm, s->d_row_hk, s->d_blocks, s->d_items, s->d_iblocks, s->d_rdf_items,
                    s->d_bterms, s->d_bblocks, s->d_bond_k, s->d_bond_r0, s->d_angle_k,
                    s->d_angle_t0, s->d_rp, s->d_rp_nm, s->d_rp_lang, s->d_mf_cols,
                    s->d_mf_tab, s->d_row_spw, s->d_circ, s->d_stage,
                    s->d_row_stage, s->d_stage_rows, s->d_lang, s->d_basis, s->d_tw,
                    s->d_prop, s->d_row_ptr,
                    s->d_dest, s->d_part, s->d_fblocks, s->d_eslot, s->d_red_f, s->d_red_a,
                    s->d_partial, s->d_red_v, s->d_row_prev, s->d_row_next, s->d_row_ksp,
                    s->d_npairs, s->d_nonfinite, s->d_cent, s->d_scratch,
                    s->d_rdf_ranges, s->d_parts, s->d_pspec, s->d_sys_part, s->d_red_fE,
                    s->d_red_aE, s->d_red_vE, s->d_bstage};
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
    {
        const int tjf = MIXPI_FLAG_TILE_J16 | MIXPI_FLAG_TILE_J32 | MIXPI_FLAG_TILE_J64;
        const int jobf = MIXPI_FLAG_TILE_WAVES1 | MIXPI_FLAG_TILE_WAVES2 | MIXPI_FLAG_TILE_I128 |
                         MIXPI_FLAG_TILE_I256;
        const int known = MIXPI_FLAG_CHECK_FINITE | tjf | jobf;
        const int f = d->flags;
        if ((f & ~known) || __builtin_popcount(f & tjf) > 1 || __builtin_popcount(f & jobf) > 1)
            return fail(MIXPI_E_INVALID, "system %d: bad flags 0x%x", idx, f);
    }
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
        if (d->mol_id[i] < 0 || d->mol_id[i] >= (1 << 27))
            return fail(MIXPI_E_INVALID, "system %d: particle %d has mol_id %d (range [0, 2^27))",
                        idx, i, d->mol_id[i]);
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
        !(std::isfinite(d->rc_coul) && d->rc_coul >= 0.0) || !finite_pos(d->rc_lj))
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
    std::vector<double> lj_eps, lj_sig, charge, bond_k, bond_r0, angle_k, angle_t0;
    std::vector<int> ljt, mol, row_part, row_sys;
    std::vector<double> row_fm, row_hk, row_ksp;
    std::vector<long long> row_prev, row_next;
    std::vector<PairBlock> blocks;
    std::vector<BondedTerm> bterms, bterms_slow;
    std::vector<RpItem> rp_fft, rp_dense;
    std::vector<RpItem> rings;                 // one per big ring column group (circulant candidates)
    std::vector<double> basis, prop, circ;
    std::vector<double2> tw;
    std::map<int, int> basis_off, tw_off;
    std::vector<long long> bead_index;
    std::vector<PartDev> parts;
    std::vector<double> ew_z;                  // Ewald charge per particle (0 for electrons)
    std::vector<int> sys_part;                 // first particle of each system
    std::vector<std::pair<long long, long long>> sys_rows;   // [begin, end) per system
    struct GroupRec {
        int sys;
        long long row;
        int N, n;
        int p;                                 // first particle (over the handle)
    };
    std::vector<GroupRec> groups;              // every group of every system, in row order
    std::vector<MfmaCol> mf_cols;              // columns of the matrix-core items
    std::vector<double> mf_tab;                // their generator tables
    long long rows = 0;
    long long candidates = 0;
    int n_part = 0, n_groups = 0;
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
    // the pair sweep's cutoff constants, formed once (launches that pass
    // theta form the theta-dependent ones in the kernel)
    S.irc = d->rc_coul > 0.0 ? 1.0 / d->rc_coul : 0.0;
    S.irc3 = d->rc_coul > 0.0 ? 1.0 / (d->rc_coul * d->rc_coul * d->rc_coul) : 0.0;
    {
        const double u_c = d->rc_pp * d->rc_pp + d->pp_a * d->pp_a;
        S.pp_phic = 1.0 / std::sqrt(u_c);
        S.pp_psic = -1.0 / (u_c * std::sqrt(u_c));
        S.pp_chic = 1.0 / (u_c * u_c * std::sqrt(u_c));
    }
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
        B.ljt.push_back(d->lj_type[i] < 0 ? nt : d->lj_type[i]);
        B.mol.push_back(d->mol_id[i]);
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
    for (const Group &g : groups)
        B.groups.push_back(Build::GroupRec{s, g.row, g.N, g.n, p_base + g.p0});
    B.sys_part.push_back(p_base);
    for (const Group &g : groups)
        for (int i = 0; i < g.n; ++i) {
            PartDev pd{};
            pd.row0 = g.row + i;
            pd.stride = g.n;
            pd.nb = g.N;
            pd.inv_nm = 1.0 / (g.N * d->fict_mass[g.p0 + i]);
            pd.spec = d->lj_type[g.p0 + i] < 0 ? nt : d->lj_type[g.p0 + i];
            pd.sys = s;
            B.parts.push_back(pd);
        }
    for (int i = 0; i < n; ++i) B.ew_z.push_back(d->is_electron[i] ? 0.0 : d->charge[i]);

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
    B.row_part.resize(row, -1);
    B.row_sys.resize(row, s);
    B.row_fm.resize(row, 0.0);
    B.row_hk.resize(row, S.hkick);
    B.row_ksp.resize(row, 0.0);
    B.row_prev.resize(row, 0);
    B.row_next.resize(row, 0);
    for (const Group &g : groups)
        for (int a = 0; a < g.N; ++a)
            for (int i = 0; i < g.n; ++i) {
                const long long r = g.row + (long long)a * g.n + i;
                rows_of[part_first[g.p0 + i] + a] = r;
                B.row_part[r] = p_base + g.p0 + i;
                B.row_fm[r] = d->fict_mass[g.p0 + i];
                // ring neighbours and spring constant N m / (beta hbar)^2 in kcal/mol/A^2
                B.row_prev[r] = g.row + (long long)((a + g.N - 1) % g.N) * g.n + i;
                B.row_next[r] = g.row + (long long)((a + 1) % g.N) * g.n + i;
                B.row_ksp[r] = g.N > 1 ? g.N * d->mass[g.p0 + i] / (bh * bh) / kKcal : 0.0;
            }
    B.bead_index.insert(B.bead_index.end(), rows_of.begin(), rows_of.end());
    auto bead_row = [&](int i, int a) { return rows_of[part_first[i] + a]; };

    // nonbonded pair blocks (tiles are cut later, once the tile width is known)
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
            pb.nbeads_b = Bg.N;
            pb.lj_off = S.lj_off;
            pb.nt1 = S.nt1;
            {
                // LJ can act between the groups if a type pair of them has
                // eps != 0, or both hold type 0 (its eps can be overridden)
                std::vector<char> ta(nt + 1, 0), tb(nt + 1, 0);
                for (int x = 0; x < A.n; ++x) ta[B.ljt[p_base + A.p0 + x]] = 1;
                for (int x = 0; x < Bg.n; ++x) tb[B.ljt[p_base + Bg.p0 + x]] = 1;
                pb.lj = 0;
                for (int a = 0; a < nt; ++a)
                    for (int b = 0; b < nt; ++b)
                        if (ta[a] && tb[b] && (d->lj_eps[a * nt + b] != 0.0 || (a == 0 && b == 0)))
                            pb.lj = 1;
            }
            {
                // the molecule compare can be left out where no two distinct
                // particles of the two groups share a molecule id
                std::map<int, int> ma;
                for (int x = 0; x < A.n; ++x) ++ma[d->mol_id[A.p0 + x]];
                pb.mol = 0;
                if (pb.same) {
                    for (auto &kv : ma) pb.mol |= kv.second > 1;
                } else {
                    for (int x = 0; x < Bg.n; ++x) pb.mol |= ma.count(d->mol_id[Bg.p0 + x]) > 0;
                }
            }
            {
                // electron (i) - atom (j) blocks in a box large against the
                // pseudopotential cutoff cull the j-atoms out of reach of a
                // tile's beads: a sphere of r_c + 3 A (the cutoff plus a
                // typical extent of 64 to 128 beads of an electron) under
                // 0.6 of the box volume; MIXPI_PAIR_CULL = 0 or 1 turns it
                // off or on for every such block
                const double rr = d->rc_pp + 3.0;
                const double vbox = d->box[0] * d->box[1] * d->box[2];
                pb.cull = pb.kind == PK_E_ATOM && 4.0 / 3.0 * kPi * rr * rr * rr < 0.6 * vbox;
                if (const char *env = getenv("MIXPI_PAIR_CULL")) {
                    const int v = atoi(env);
                    if (v == 0 || v == 1) pb.cull = pb.kind == PK_E_ATOM && v == 1;
                }
            }
            B.blocks.push_back(pb);
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

    // bonded terms: one entry per (term, slice), beads resolved here;
    // terms whose slices reach an FFT group go to the "slow" list
    for (int b = 0; b < d->n_bonds; ++b) {
        const int i = d->bonds[2 * b], j = d->bonds[2 * b + 1];
        const int Ni = d->n_beads[i], Nj = d->n_beads[j], Nm = std::max(Ni, Nj);
        auto &dst = Nm > kDenseMaxN ? B.bterms_slow : B.bterms;
        for (int sl = 0; sl < Nm; ++sl) {
            BondedTerm t{};
            t.r[0] = (int)bead_row(i, (int)((long long)sl * Ni / Nm));
            t.r[1] = (int)bead_row(j, (int)((long long)sl * Nj / Nm));
            t.r[2] = t.r[1];
            t.type = S.bond_off + d->bond_type[b];
            t.kind = 0;
            t.sys = s;
            t.w = 1.0 / Nm;
            dst.push_back(t);
        }
    }
    for (int a = 0; a < d->n_angles; ++a) {
        const int i = d->angles[3 * a], v = d->angles[3 * a + 1], j = d->angles[3 * a + 2];
        const int Ni = d->n_beads[i], Nv = d->n_beads[v], Nj = d->n_beads[j];
        const int Nm = std::max(Ni, std::max(Nv, Nj));
        auto &dst = Nm > kDenseMaxN ? B.bterms_slow : B.bterms;
        for (int sl = 0; sl < Nm; ++sl) {
            BondedTerm t{};
            t.r[0] = (int)bead_row(i, (int)((long long)sl * Ni / Nm));
            t.r[1] = (int)bead_row(v, (int)((long long)sl * Nv / Nm));
            t.r[2] = (int)bead_row(j, (int)((long long)sl * Nj / Nm));
            t.type = S.angle_off + d->angle_type[a];
            t.kind = 1;
            t.sys = s;
            t.w = 1.0 / Nm;
            dst.push_back(t);
        }
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
        } else {
            if (!B.tw_off.count(N)) {
                B.tw_off[N] = (int)B.tw.size();
                // stage-major: stage s (span 2^s) holds exp(-2 pi i pos / 2^s), pos < 2^(s-1)
                for (int span = 2; span <= N; span *= 2)
                    for (int pos = 0; pos < span / 2; ++pos)
                        B.tw.push_back(make_double2(std::cos(2.0 * kPi * pos / span),
                                                    -std::sin(2.0 * kPi * pos / span)));
            }
            {
                // a candidate for the bead-space (circulant) step
                RpItem rg{};
                rg.kind = RP_CIRC;
                rg.sys = s;
                rg.N = N;
                rg.logN = ilog2(N);
                rg.n = g.n;
                rg.p0 = p_base + g.p0;
                rg.row = g.row;
                rg.tw_off = B.tw_off[N];
                B.rings.push_back(rg);
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
        }
    }
    B.sys_rows.push_back({row_base, row});
    B.rows = row;
    B.n_part += n;
}

// LDS bytes a ring-polymer item needs: the dense basis and its transpose,
// the complex signal and its twiddles, or the circulant rows (q, p, a, b, c,
// each N plus its pad) and the partial outputs.  A launch takes the largest
// over its items, so items of small rings run more workgroups per CU.
unsigned rp_item_lds(const RpItem &it, int op = OP_STEP, int precision = 0)
{
    const long long N = it.N;
    if (it.kind == RP_MFMA) return mfma_lds_bytes(it.N, op, precision);
    if (it.kind == RP_DENSE) return (unsigned)((2 * N * N + 4 * 256) * sizeof(double));
    if (it.kind == RP_FFT) return (unsigned)((2 * N - 1) * sizeof(double2));
    return (unsigned)((5 * (N + 64)) * sizeof(double));
}

// Rings propagated in bead space (circulant items): the cheapest first,
// while the total multiply-adds stay within a budget of about two waves of
// items over the chip, where they beat one FFT workgroup per column in
// latency.  A ring needs N <= kCircMaxN.  Only handles with few ring
// columns (at most kCircMaxCols over all their rings) use them: with many
// columns the FFT workgroups already fill the chip, and the circulant
// items only add work beside them (measured on the 64-system batch: ring
// launch 30.1 us with circulant items for its smaller rings, 23.9 us with
// FFT items only; one 1024-bead ring: 6.4 against 11.4 us).
// MIXPI_RING_CIRC = 0 or 1 turns them off, or on whatever the column count.
constexpr int kCircMaxCols = 24;
std::vector<char> choose_circulant(const std::vector<RpItem> &rings)
{
    std::vector<char> use(rings.size(), 0);
    int force = -1;
    if (const char *env = getenv("MIXPI_RING_CIRC")) force = atoi(env);
    if (force == 0) return use;
    long long cols = 0;
    for (const RpItem &rg : rings) cols += 3LL * rg.n;
    if (force != 1 && cols > kCircMaxCols) return use;
    std::vector<size_t> order(rings.size());
    for (size_t r = 0; r < rings.size(); ++r) order[r] = r;
    auto cost = [&](size_t r) { return 12.0 * rings[r].n * (double)rings[r].N * rings[r].N; };
    std::sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost(x) < cost(y); });
    // MIXPI_RING_CIRC_MMAC: the budget in millions of multiply-adds
    double budget = 32.0 * 1024 * 1024;
    if (const char *env = getenv("MIXPI_RING_CIRC_MMAC")) {
        const double v = atof(env);
        if (v >= 0.0) budget = v * 1024 * 1024;
    }
    double used = 0.0;
    for (size_t r : order) {
        if (rings[r].N > kCircMaxN) continue;
        if (used + cost(r) > budget) break;
        used += cost(r);
        use[r] = 1;
    }
    return use;
}

// Circulant rows a_d, b_d, c_d (d = 0 .. N-1) of every particle of ring
// group rg, from the per-mode propagation coefficients: row_d =
// (1/N) sum_k f_k cos(2 pi k d / N), f = (cos w dt, sin(w dt)/(m w),
// -m w sin(w dt)); then the items of kCircOut outputs per column.
void add_circulant(Build &B, const RpItem &rg, int stage0, std::vector<RpItem> &items)
{
    const int N = rg.N, n = rg.n;
    std::vector<double> cs(N);
    for (int m = 0; m < N; ++m) cs[m] = std::cos(2.0 * kPi * m / N);
    for (int i = 0; i < n; ++i) {
        const int off = (int)B.circ.size();
        B.circ.resize(B.circ.size() + 3 * (size_t)N, 0.0);
        double *A = &B.circ[off], *Bq = A + N, *Cq = Bq + N;
        for (int d = 0; d < N; ++d) {
            double sa = 0.0, sb = 0.0, sc = 0.0;
            for (int k = 0; k < N; ++k) {
                const double *pr = &B.prop[5 * (size_t)(rg.row + (long long)k * n + i)];
                const double c = cs[(int)(((long long)k * d) % N)];
                sa += pr[0] * c;
                sb += pr[1] * c;
                sc += pr[2] * c;
            }
            A[d] = sa / N;
            Bq[d] = sb / N;
            Cq[d] = sc / N;
        }
        // spring weight k/2 per squared bead step, from mode 1's entry
        // k lambda_1 / 2 of the propagation table
        const double s1 = std::sin(kPi / N);
        const double wsp = B.prop[5 * (size_t)(rg.row + (long long)n + i) + 4] / (4.0 * s1 * s1);
        for (int dim = 0; dim < 3; ++dim)
            for (int o0 = 0; o0 < N; o0 += kCircOut) {
                RpItem it = rg;
                it.c0 = 3 * i + dim;
                it.ncols = 1;
                it.o0 = o0;
                it.circ_off = off;
                it.stage0 = stage0;
                it.wsp = wsp;
                items.push_back(it);
            }
    }
}

// Matrix-core transform items of the groups whose N `use` accepts: the
// columns of all groups of one bead count share the basis (a cos table of N
// entries), 16 columns and 16 output rows per item.
template <typename Use>
void add_mfma_transforms(Build &B, std::vector<RpItem> &items, Use use)
{
    std::map<int, std::vector<int>> by_n;      // N -> groups
    for (size_t g = 0; g < B.groups.size(); ++g)
        if (use(B.groups[g].N)) by_n[B.groups[g].N].push_back((int)g);
    for (auto &kv : by_n) {
        const int N = kv.first;
        const int tab = (int)B.mf_tab.size();
        for (int m = 0; m < N; ++m) B.mf_tab.push_back(std::cos(2.0 * kPi * m / N));
        std::vector<MfmaCol> cols;
        std::vector<int> col_sys;
        for (int g : kv.second) {
            const auto &G = B.groups[g];
            for (int i = 0; i < G.n; ++i)
                for (int d = 0; d < 3; ++d) {
                    cols.push_back(MfmaCol{G.row + i, -1, G.n, d});
                    col_sys.push_back(G.sys);
                }
        }
        for (size_t c0 = 0; c0 < cols.size(); c0 += kMfCols) {
            const int nc = (int)std::min<size_t>(kMfCols, cols.size() - c0);
            const int base = (int)B.mf_cols.size();
            B.mf_cols.insert(B.mf_cols.end(), cols.begin() + c0, cols.begin() + c0 + nc);
            for (int o0 = 0; o0 < N; o0 += kMfRows) {
                RpItem it{};
                it.kind = RP_MFMA;
                it.sys = col_sys[c0];
                it.N = N;
                it.logN = ilog2(N);
                it.c0 = base;
                it.ncols = nc;
                it.o0 = o0;
                it.circ_off = tab;
                items.push_back(it);
            }
        }
    }
}

// Matrix-core propagation items for the groups marked in `use`: rings are
// put into propagator classes (equal bead count and equal propagation
// coefficients of every mode, so equal circulant rows a_d, b_d, c_d); the
// columns of a class, across groups and systems, share one table.  Every
// row of such a group gets a stage row (the items update q and p in place)
// and the epilogue's spring weight k/2.
void add_mfma_propagation(Build &B, const std::vector<char> &use, std::vector<int> &row_stage,
                          std::vector<long long> &stage_rows, std::vector<double> &row_spw,
                          std::vector<RpItem> &items)
{
    std::map<std::vector<double>, int> cls;    // coefficients -> class
    std::vector<std::vector<MfmaCol>> cls_cols;
    std::vector<int> cls_tab, cls_n, cls_sys;
    std::vector<double> cls_dtm;
    for (size_t g = 0; g < B.groups.size(); ++g) {
        if (!use[g]) continue;
        const auto &G = B.groups[g];
        const int N = G.N;
        const int stage0 = (int)stage_rows.size();
        for (long long x = 0; x < (long long)N * G.n; ++x) {
            row_stage[G.row + x] = stage0 + (int)x;
            stage_rows.push_back(G.row + x);
            row_spw[G.row + x] = 0.5 * B.row_ksp[G.row + x];
        }
        for (int i = 0; i < G.n; ++i) {
            std::vector<double> key((size_t)3 * N + 1);
            key[0] = N;
            for (int k = 0; k < N; ++k)
                for (int c = 0; c < 3; ++c)
                    key[1 + 3 * k + c] = B.prop[5 * (size_t)(G.row + (long long)k * G.n + i) + c];
            auto f = cls.find(key);
            int id;
            if (f == cls.end()) {
                id = (int)cls_cols.size();
                cls[key] = id;
                cls_cols.emplace_back();
                cls_n.push_back(N);
                cls_sys.push_back(G.sys);
                cls_dtm.push_back(key[1 + 1]);               // mode 0: dt / m_f
                cls_tab.push_back((int)B.mf_tab.size());
                // rows_d = (1/N) sum_k f_k cos(2 pi k d / N) of a, b, c
                std::vector<double> cs(N);
                for (int m = 0; m < N; ++m) cs[m] = std::cos(2.0 * kPi * m / N);
                const size_t off = B.mf_tab.size();
                B.mf_tab.resize(off + 3 * (size_t)N, 0.0);
                for (int d = 0; d < N; ++d)
                    for (int c = 0; c < 3; ++c) {
                        double acc = 0.0;
                        for (int k = 0; k < N; ++k)
                            acc += key[1 + 3 * k + c] * cs[(int)(((long long)k * d) % N)];
                        B.mf_tab[off + (size_t)c * N + d] = acc / N;
                    }
            } else {
                id = f->second;
            }
            for (int d = 0; d < 3; ++d)
                cls_cols[id].push_back(MfmaCol{G.row + i, (long long)stage0 + i, G.n, d});
        }
    }
    for (size_t id = 0; id < cls_cols.size(); ++id) {
        const auto &cols = cls_cols[id];
        const int N = cls_n[id];
        for (size_t c0 = 0; c0 < cols.size(); c0 += kMfCols) {
            const int nc = (int)std::min<size_t>(kMfCols, cols.size() - c0);
            const int base = (int)B.mf_cols.size();
            B.mf_cols.insert(B.mf_cols.end(), cols.begin() + c0, cols.begin() + c0 + nc);
            for (int o0 = 0; o0 < N; o0 += kMfRows) {
                RpItem it{};
                it.kind = RP_MFMA;
                it.sys = cls_sys[id];
                it.N = N;
                it.logN = ilog2(N);
                it.c0 = base;
                it.ncols = nc;
                it.o0 = o0;
                it.circ_off = cls_tab[id];
                it.dtm = cls_dtm[id];
                items.push_back(it);
            }
        }
    }
}

// Cuts pair block bi into items: for each j-bead b, the i-tiles of 64 iw
// beads of its contiguous i-run times runs of up to jrun consecutive j-tiles
// of tj particles (for a group with itself only tiles that hold some
// j > i).  The items of one (b, i0) follow each other, j0 ascending.
void block_items(const PairBlock &pb, int bi, int tj, int iw, int jrun, std::vector<PairItem> &out)
{
    const long long li = (long long)pb.na << pb.shift;
    for (int b = 0; b < pb.nbeads_b; ++b)
        for (long long i0 = 0; i0 < li; i0 += 64 * iw) {
            int j0 = 0;
            while (pb.same && j0 + tj <= i0) j0 += tj;
            for (; j0 < pb.nb; j0 += jrun * tj) {
                PairItem it{};
                it.block = bi;
                it.b = b;
                it.i0 = (int)i0;
                it.j0 = j0;
                it.tj = tj;
                it.nj = std::min(jrun, (pb.nb - j0 + tj - 1) / tj);
                out.push_back(it);
            }
        }
}

// Cost of sweeping one lane over W j-slots of an atom block, in VALU
// instructions of the FP32 build.  p: the expected share of candidates
// inside the cutoff, the cutoff sphere's volume over the box volume (at
// most 1).  The masked sweep spends 64.5 per slot with LJ, 45.5 without;
// the compacted sweep spends 22.5 per slot on the distance pass plus, per
// marked slot of the fullest lane (taken as the mean W p plus 2.4 standard
// deviations, the largest of 64 binomial counts), 69 on the pair math with
// LJ, 50 without (counted in the gfx950 assembly of the loops).
double atom_sweep_cost(const SysDev &S, bool lj, int W, bool compact)
{
    if (!compact) return (lj ? 64.5 : 45.5) * W;
    const double rc = std::max(S.rc_lj, S.rc_c);
    const double vol = S.box[0] * S.box[1] * S.box[2];
    const double p = std::min(1.0, 4.0 / 3.0 * kPi * rc * rc * rc / vol);
    const double hits = std::min((double)W, W * p + 2.4 * std::sqrt(W * p * (1.0 - p)));
    return 22.5 * W + (lj ? 69.0 : 50.0) * hits;
}

// Whether an atom block with W = tj slots per lane is swept in compacted
// form: when that saves at least a tenth, and only for W >= 32.  With 16
// slots per lane the saving is small and the marked-slot loop (not
// unrolled, one slot per iteration at scattered LDS addresses) runs slower
// per instruction than the masked loop, so it loses (measured on both forms).
bool sparse_pays(const SysDev &S, bool lj, int W)
{
    if (W < 32) return false;
    return atom_sweep_cost(S, lj, W, true) < 0.9 * atom_sweep_cost(S, lj, W, false);
}

// 64 x 64 tiles of the handle's pair blocks: the work size that picks the
// default tile shape.
size_t tiles64(const std::vector<PairBlock> &blocks)
{
    std::vector<PairItem> items;
    for (size_t bi = 0; bi < blocks.size(); ++bi) block_items(blocks[bi], (int)bi, 64, 1, 1, items);
    return items.size();
}

// Natural partial-force slots of the items, in order: 64 iw i-slots, then
// jrun tj j-slots each (a shorter run leaves some unused; for a launch of
// one width, item k's start at k (64 iw + jrun tj), as the kernel assumes).
// Returns the number of slots (-1 past 2^31 - 1).
long long assign_item_slots(std::vector<PairItem> &items, int iw, int jrun)
{
    long long next = 0;
    for (PairItem &it : items) {
        it.islot = (int)next;
        it.jslot = (int)(next + 64 * iw);
        next += 64 * iw + (long long)jrun * it.tj;
        if (next > (1LL << 31) - 1) return -1;
    }
    return next;
}

// Workgroup ranges over a list sorted by system: chunks of at most `per`
// entries that never span two systems.
std::vector<BlockRange> system_blocks(const std::vector<int> &sys_of, int begin, int end, int per)
{
    std::vector<BlockRange> out;
    int i = begin;
    while (i < end) {
        int j = i;
        while (j < end && j - i < per && sys_of[j] == sys_of[i]) ++j;
        out.push_back(BlockRange{sys_of[i], i, j - i, 0});
        i = j;
    }
    return out;
}

// Reducer plan for the slot ranges [begin, end): each system's slots (in
// range and slot order) cut into chunks of at most kChunkSlots consecutive
// slots of that system.
// Packed as chunk_begin[n_chunks] | chunk_len[n_chunks] | sys_chunk[n_sys + 1];
// off[] receives the three offsets.  Returns n_chunks.
int reducer_plan(const std::vector<int> &eslot_sys, const std::vector<std::pair<int, int>> &ranges,
                 int n_sys, std::vector<int> &out, int off[3])
{
    std::vector<std::vector<std::pair<int, int>>> runs(n_sys);
    for (const auto &rg : ranges)
        for (int k = rg.first, n = rg.second; k < n;) {
            int e = k;
            while (e < n && eslot_sys[e] == eslot_sys[k] && e - k < kChunkSlots) ++e;
            runs[eslot_sys[k]].push_back({k, e - k});
            k = e;
        }
    std::vector<int> cb, cl, sys_chunk(n_sys + 1, 0);
    for (int y = 0; y < n_sys; ++y) {
        sys_chunk[y] = (int)cb.size();
        for (auto &r : runs[y]) {
            cb.push_back(r.first);
            cl.push_back(r.second);
        }
    }
    sys_chunk[n_sys] = (int)cb.size();
    out.clear();
    off[0] = 0;
    out.insert(out.end(), cb.begin(), cb.end());
    off[1] = (int)out.size();
    out.insert(out.end(), cl.begin(), cl.end());
    off[2] = (int)out.size();
    out.insert(out.end(), sys_chunk.begin(), sys_chunk.end());
    return (int)cb.size();
}

// Partial-force slots and the per-row gather lists.  Natural slots: the
// pair items' (64 i-slots, then tj j-slots each, as assign_item_slots
// numbers them), then bonded term t owns
// part_bonded + 3t + (0, 1, 2) for its beads r[0], r[1] (and r[2] of an
// angle).  Rows list their slots in this order, so every gather sums in a
// fixed order.
struct Gather {
    std::vector<long long> row_ptr;   // [rows + 1] CSR positions of each row's slots
    std::vector<int> dest;            // [n_slots] position of each natural slot, -1 unused
    long long n_slots = 0;            // natural slots (pair items, then bonded terms)
};

Gather build_gather(long long rows, const std::vector<PairBlock> &blocks,
                    const std::vector<PairItem> &items, int iw, const std::vector<BondedTerm> &terms,
                    long long part_bonded)
{
    Gather G;
    std::vector<long long> cnt(rows + 1, 0);
    auto visit = [&](auto &&emit) {
        for (size_t k = 0; k < items.size(); ++k) {
            const PairItem &it = items[k];
            const PairBlock &pb = blocks[it.block];
            const long long li = (long long)pb.na << pb.shift;
            for (int l = 0; l < 64 * iw; ++l) {
                const long long idx = (long long)it.i0 + l;
                if (idx < li)
                    emit(pb.rowa + ((long long)it.b << pb.shift) * pb.na + idx, (long long)it.islot + l);
            }
            for (int k = 0; k < it.nj; ++k) {
                const int j0 = it.j0 + k * it.tj, jn = std::min(it.tj, pb.nb - j0);
                for (int l = 0; l < jn; ++l)
                    emit(pb.rowb + (long long)it.b * pb.nb + j0 + l, (long long)it.jslot + k * it.tj + l);
            }
        }
        for (size_t t = 0; t < terms.size(); ++t) {
            const long long b = part_bonded + 3 * (long long)t;
            emit(terms[t].r[0], b);
            emit(terms[t].r[1], b + 1);
            if (terms[t].kind == 1) emit(terms[t].r[2], b + 2);
        }
        return part_bonded + 3 * (long long)terms.size();
    };
    G.n_slots = visit([&](long long row, long long) { ++cnt[row + 1]; });
    for (long long r = 0; r < rows; ++r) cnt[r + 1] += cnt[r];
    G.row_ptr = cnt;
    G.dest.assign((size_t)G.n_slots, -1);
    std::vector<long long> fill(cnt.begin(), cnt.end() - 1);
    visit([&](long long row, long long sl) { G.dest[sl] = (int)fill[row]++; });
    return G;
}

int create_impl(const mixpi_system_desc *const *descs, int n_sys, mixpi_system **out)
{
    if (!out) return fail(MIXPI_E_INVALID, "out is null");
    *out = nullptr;
    if (!descs || n_sys < 1) return fail(MIXPI_E_INVALID, "need at least one system");
    if (n_sys > kMaxSystems)
        return fail(MIXPI_E_UNSUPPORTED, "at most %d systems per handle", kMaxSystems);
    for (int s = 0; s < n_sys; ++s) {
        int rc = validate(descs[s], s);
        if (rc) return rc;
        // the j-tile width may differ per system; every other flag is shared
        const int tjf = MIXPI_FLAG_TILE_J16 | MIXPI_FLAG_TILE_J32 | MIXPI_FLAG_TILE_J64;
        if (descs[s]->precision != descs[0]->precision ||
            (descs[s]->flags & ~tjf) != (descs[0]->flags & ~tjf))
            return fail(MIXPI_E_INVALID,
                        "all systems of a batch must share precision and flags (tile widths aside)");
    }
    Build B;
    for (int s = 0; s < n_sys; ++s) add_system(B, descs[s], s);
    if (B.rows > (1LL << 31) / 3)
        return fail(MIXPI_E_UNSUPPORTED, "too many beads (%lld)", B.rows);

    mixpi_system *S = new mixpi_system();
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return fail(MIXPI_E_HIP, "hipGetDevice failed (no GPU?)");
    }
    {
        // the static scratch of mixpi_forces_static: its address on this device
        const hipError_t e = static_scratch_init(S->device);
        if (e != hipSuccess) {
            delete S;
            return fail(MIXPI_E_HIP, "locating the static scratch on device %d: %s", S->device,
                        hipGetErrorString(e));
        }
    }
    S->n_sys = n_sys;
    S->precision = descs[0]->precision;
    S->flags = descs[0]->flags;
    S->rows = B.rows;
    S->n_part = B.n_part;
    S->n_groups = B.n_groups;
    S->candidates = B.candidates;
    S->bead_index = B.bead_index;
    for (const auto &g : B.groups)
        S->layout.insert(S->layout.end(), {g.row, (long long)g.N, (long long)g.n, (long long)g.p,
                                           (long long)g.sys});
    for (const auto &r : B.sys_rows) S->sys_row0.push_back(r.first);
    S->sys_row0.push_back(B.rows);

    // Pair items: per system with its j-tile width (a MIXPI_FLAG_TILE_J*
    // flag of its description, else MIXPI_PAIR_TJ = 16, 32 or 64, else
    // default_tj), in system and block order.
    // Default shape by the work size n64 (64 x 64 tiles), against 1024 SIMDs
    // (measured on the workloads of 1e3 to 1e5 such tiles): below 1024
    // tiles 16-wide j-tiles (more, shorter waves), below 8192 32-wide, else
    // 64-wide; from 16384 tiles on, 128 x 64 tiles (two i-split waves) that
    // sweep runs of four j-tiles: fewer partial-force slots to write and
    // gather.
    const size_t n64 = tiles64(B.blocks);
    {
        int tj0 = n64 < 1024 ? 16 : (n64 < 8192 ? 32 : 64);
        if (const char *env = getenv("MIXPI_PAIR_TJ")) {
            const int v = atoi(env);
            if (v == 16 || v == 32 || v == 64) tj0 = v;
        }
        S->pair_tj.assign(n_sys, tj0);
        for (int y = 0; y < n_sys; ++y) {
            const int f = descs[y]->flags;
            if (f & MIXPI_FLAG_TILE_J16) S->pair_tj[y] = 16;
            if (f & MIXPI_FLAG_TILE_J32) S->pair_tj[y] = 32;
            if (f & MIXPI_FLAG_TILE_J64) S->pair_tj[y] = 64;
        }
    }
    S->pair_tj_all = S->pair_tj[0];
    for (int y = 1; y < n_sys; ++y)
        if (S->pair_tj[y] != S->pair_tj_all) S->pair_tj_all = 0;
    // Waves per tile: two j-split waves while the launch has fewer than one
    // 64-bead tile per SIMD: more, shorter waves even out the SIMDs and hide
    // latency; else one, or two i-split waves from 16384 64 x 64 tiles on.
    // MIXPI_PAIR_WAVES = 1 or 2 and MIXPI_PAIR_IW = 1, 2 or 4 (i-split
    // waves, with one j-wave), or the TILE_WAVES / TILE_I flags, choose
    // instead.
    {
        std::vector<PairItem> one;
        for (size_t bi = 0; bi < B.blocks.size(); ++bi)
            block_items(B.blocks[bi], (int)bi, S->pair_tj[B.blocks[bi].sys], 1, 1, one);
        S->pair_waves = one.size() < 1024 ? 2 : 1;
        S->pair_iw = n64 >= 16384 ? 2 : 1;
        if (const char *env = getenv("MIXPI_PAIR_WAVES")) {
            const int v = atoi(env);
            if (v == 1 || v == 2) S->pair_waves = v;
        }
        if (const char *env = getenv("MIXPI_PAIR_IW")) {
            const int v = atoi(env);
            if (v == 1 || v == 2 || v == 4) S->pair_iw = v;
        }
        if (S->flags & (MIXPI_FLAG_TILE_WAVES1 | MIXPI_FLAG_TILE_WAVES2 | MIXPI_FLAG_TILE_I128 |
                        MIXPI_FLAG_TILE_I256)) {
            S->pair_waves = (S->flags & MIXPI_FLAG_TILE_WAVES2) ? 2 : 1;
            S->pair_iw = (S->flags & MIXPI_FLAG_TILE_I128) ? 2 : (S->flags & MIXPI_FLAG_TILE_I256) ? 4 : 1;
        }
        if (S->pair_iw > 1) S->pair_waves = 1;
        // j-runs: from 16384 64 x 64 tiles on, each item sweeps 4 j-tiles and
        // stores its i-forces once (fewer partial-force slots to write and
        // gather); MIXPI_PAIR_JRUN = 1, 2, 4 or 8 chooses instead
        S->pair_jrun = n64 >= 16384 ? 4 : 1;
        if (const char *env = getenv("MIXPI_PAIR_JRUN")) {
            const int v = atoi(env);
            if (v == 1 || v == 2 || v == 4 || v == 8) S->pair_jrun = v;
        }
    }
    std::vector<PairItem> items;
    for (size_t bi = 0; bi < B.blocks.size(); ++bi)
        block_items(B.blocks[bi], (int)bi, S->pair_tj[B.blocks[bi].sys], S->pair_iw, S->pair_jrun,
                    items);
    S->n_items = (int)items.size();
    {
        // compacted sweep for atom blocks with few in-cutoff candidates;
        // MIXPI_PAIR_SPARSE=0 or 1 forces it off or on for every atom block
        int force = -1;
        if (const char *env = getenv("MIXPI_PAIR_SPARSE")) {
            const int v = atoi(env);
            if (v == 0 || v == 1) force = v;
        }
        for (PairBlock &pb : B.blocks) {
            if (pb.kind != PK_ATOM) continue;
            pb.sparse = force >= 0 ? force
                                   : sparse_pays(B.sys[pb.sys], pb.lj != 0,
                                                 S->pair_tj[pb.sys] / S->pair_waves);
        }
    }
    {
        // launch order: the most expensive tiles first, so that the cheap
        // ones fill in at the end (stable within equal cost)
        std::vector<double> cost(B.blocks.size());
        for (size_t bi = 0; bi < B.blocks.size(); ++bi) {
            const PairBlock &pb = B.blocks[bi];
            const int W = S->pair_tj[pb.sys] / S->pair_waves;
            cost[bi] = S->pair_iw * (pb.kind == PK_ATOM
                                         ? atom_sweep_cost(B.sys[pb.sys], pb.lj != 0, W, pb.sparse != 0)
                                         : 41.0 * W);
        }
        std::stable_sort(items.begin(), items.end(), [&](const PairItem &x, const PairItem &y) {
            return cost[x.block] * x.nj > cost[y.block] * y.nj;
        });
    }
    const long long item_slots = assign_item_slots(items, S->pair_iw, S->pair_jrun);
    if (item_slots < 0) {
        delete S;
        return fail(MIXPI_E_UNSUPPORTED, "too many partial-force slots");
    }

    // bonded terms and their system-pure blocks
    std::vector<BondedTerm> terms = B.bterms;
    const int n_terms_fast = (int)terms.size();
    terms.insert(terms.end(), B.bterms_slow.begin(), B.bterms_slow.end());
    std::vector<int> term_sys(terms.size());
    for (size_t t = 0; t < terms.size(); ++t) term_sys[t] = terms[t].sys;
    std::vector<BlockRange> bblocks = system_blocks(term_sys, 0, n_terms_fast, 64);
    S->n_bblocks_fast = (int)bblocks.size();
    {
        auto slow = system_blocks(term_sys, n_terms_fast, (int)terms.size(), 64);
        bblocks.insert(bblocks.end(), slow.begin(), slow.end());
    }
    S->n_bblocks = (int)bblocks.size();

    std::vector<int> row_stage((size_t)B.rows, -1);
    std::vector<long long> stage_rows;
    std::vector<double> row_spw((size_t)B.rows, 0.0);
    // Matrix-core (MFMA) items for rings of 16 to 64 beads, in the
    // transforms and in the step (replacing the dense items there); larger
    // rings keep the FFT and circulant items, which do the same exact work in
    // O(N log N) or spread over many workgroups, where a 16-row matrix item
    // re-reads its whole 2N x 16 input (measured: C5's ring launch 34 us
    // with FFT items, 83-108 us with matrix items; C2's 32-bead hydrogens
    // 8.6 -> 6.8 us with them).  MIXPI_NM_MFMA / MIXPI_RING_MFMA = 0 or 1
    // turn them off or on for every ring with N >= 16.
    auto mfma_rule = [](const char *name) {
        const char *env = getenv(name);
        return env ? atoi(env) : -1;
    };
    const int nm_rule = mfma_rule("MIXPI_NM_MFMA"), ring_rule = mfma_rule("MIXPI_RING_MFMA");
    auto mfma_for = [](int rule, int N) {
        if (N < kMfMinN || rule == 0) return false;
        return rule == 1 || N <= kDenseMaxN;
    };
    std::vector<char> grp_mfma(B.groups.size(), 0);
    for (size_t g = 0; g < B.groups.size(); ++g) grp_mfma[g] = mfma_for(ring_rule, B.groups[g].N);
    auto grp_of_row = [&](long long row) {
        size_t g = 0;
        while (g + 1 < B.groups.size() && B.groups[g + 1].row <= row) ++g;
        return g;
    };
    // Langevin and velocity-Verlet launches: dense, then FFT items (whole columns)
    std::vector<RpItem> rp_lang = B.rp_dense;
    rp_lang.insert(rp_lang.end(), B.rp_fft.begin(), B.rp_fft.end());
    S->n_rp_lang = (int)rp_lang.size();
    // transforms: matrix-core items for N >= 16, dense / FFT items below
    std::vector<RpItem> rp_nm;
    for (const RpItem &it : rp_lang)
        if (!mfma_for(nm_rule, it.N)) rp_nm.push_back(it);
    add_mfma_transforms(B, rp_nm, [&](int N) { return mfma_for(nm_rule, N); });
    S->n_rp_nm = (int)rp_nm.size();
    // step items, longest first so that they start at once: FFT columns,
    // then circulant items, then matrix-core items, then the dense items
    std::vector<RpItem> rp;
    {
        std::vector<RpItem> rings;
        for (const RpItem &rg : B.rings)
            if (!grp_mfma[grp_of_row(rg.row)]) rings.push_back(rg);
        std::vector<char> circ_ring = choose_circulant(rings);
        std::vector<RpItem> circ_items, mf_items;
        for (size_t r = 0; r < rings.size(); ++r) {
            const RpItem &rg = rings[r];
            if (!circ_ring[r]) {
                for (const RpItem &it : B.rp_fft)
                    if (it.row == rg.row) rp.push_back(it);
                continue;
            }
            const int stage0 = (int)stage_rows.size();
            for (long long x = 0; x < (long long)rg.N * rg.n; ++x) {
                row_stage[rg.row + x] = stage0 + (int)x;
                stage_rows.push_back(rg.row + x);
            }
            add_circulant(B, rg, stage0, circ_items);
        }
        add_mfma_propagation(B, grp_mfma, row_stage, stage_rows, row_spw, mf_items);
        rp.insert(rp.end(), circ_items.begin(), circ_items.end());
        rp.insert(rp.end(), mf_items.begin(), mf_items.end());
        for (const RpItem &it : B.rp_dense)
            if (!grp_mfma[grp_of_row(it.row)]) rp.push_back(it);
        S->n_stage = (int)stage_rows.size();
        S->n_mf_step = (int)mf_items.size();
    }
    S->n_rp = S->n_rp_fast = (int)rp.size();
    const unsigned lds0 = (unsigned)(kReduceThreads * sizeof(double));
    S->rp_lds_step = S->rp_lds_nm = S->rp_lds_lang = lds0;
    for (const RpItem &it : rp)
        S->rp_lds_step = std::max(S->rp_lds_step, rp_item_lds(it, OP_STEP, 0));
    for (const RpItem &it : rp_nm)
        S->rp_lds_nm = std::max(S->rp_lds_nm, rp_item_lds(it, OP_FWD, S->precision));
    for (const RpItem &it : rp_lang) S->rp_lds_lang = std::max(S->rp_lds_lang, rp_item_lds(it));
    S->rp_lds = std::max({S->rp_lds_step, S->rp_lds_nm, S->rp_lds_lang});

    // partial-force slots
    S->part_bonded = item_slots;
    Gather G = build_gather(B.rows, B.blocks, items, S->pair_iw, terms, S->part_bonded);

    // epilogue blocks: 4 waves of rpw rows of one system.  Many rows with
    // short partial runs share a wave (64 / rpw lanes per row); few rows or
    // long runs keep a whole wave each.
    {
        const double avg = B.rows > 0 ? (double)G.row_ptr.back() / B.rows : 0.0;
        // rows per wave by the mean partial run: 4 up to 48 slots (16 lanes a
        // row, at most three rounds), 2 up to 96
        S->fin_rpw = B.rows < 4096 ? 1 : (avg <= 48.0 ? 4 : (avg <= 96.0 ? 2 : 1));
        if (const char *env = getenv("MIXPI_FIN_RPW")) {
            const int v = atoi(env);
            if (v == 1 || v == 2 || v == 4) S->fin_rpw = v;
        }
    }
    const int fin_rows = 4 * S->fin_rpw;
    std::vector<BlockRange> fblocks;
    for (int s = 0; s < n_sys; ++s)
        for (long long r = B.sys_rows[s].first; r < B.sys_rows[s].second; r += fin_rows)
            fblocks.push_back(BlockRange{s, (int)r,
                                         (int)std::min<long long>(fin_rows, B.sys_rows[s].second - r), 0});
    S->n_fblocks = (int)fblocks.size();
    if (G.n_slots > (1LL << 31) - 1) {
        delete S;
        return fail(MIXPI_E_UNSUPPORTED, "too many partial-force slots (%lld)", G.n_slots);
    }
    S->n_slots = G.n_slots;
    S->n_positions = G.row_ptr.back();

    // energy slots and their systems
    S->e_bonded = S->n_items;
    S->e_rp = S->e_bonded + S->n_bblocks;
    S->e_fin = S->e_rp + S->n_rp;
    S->e_ew = S->e_fin + S->n_fblocks;           // one centroid-Ewald slot per system
    S->n_eslots = S->e_ew + n_sys;
    std::vector<int> eslot_sys(S->n_eslots);
    for (int s = 0; s < n_sys; ++s) eslot_sys[S->e_ew + s] = s;
    for (int k = 0; k < S->n_items; ++k) eslot_sys[k] = B.blocks[items[k].block].sys;
    for (int b = 0; b < S->n_bblocks; ++b) eslot_sys[S->e_bonded + b] = bblocks[b].sys;
    for (int r = 0; r < S->n_rp; ++r) eslot_sys[S->e_rp + r] = rp[r].sys;
    for (int f = 0; f < S->n_fblocks; ++f) eslot_sys[S->e_fin + f] = fblocks[f].sys;
    // radial distribution: the blocks' 64 x 64 tiles in runs of at most K
    // tiles of one system, K chosen for about 2048 workgroups and so that no
    // LDS count can pass 2^32
    std::vector<BlockRange> rdf_ranges;
    std::vector<PairItem> rdf_items;
    {
        for (const SysDev &sd : B.sys) S->max_nt1 = std::max(S->max_nt1, sd.nt1);
        for (const PairBlock &pb : B.blocks)
            S->top_beads = std::max(S->top_beads, pb.nbeads_b << pb.shift);
        std::vector<int> rdf_sys;
        for (size_t bi = 0; bi < B.blocks.size(); ++bi) {
            block_items(B.blocks[bi], (int)bi, kRdfTj, 1, 1, rdf_items);
            rdf_sys.resize(rdf_items.size(), B.blocks[bi].sys);
        }
        const int n_rdf = (int)rdf_items.size();
        const long long per_item = 64LL * kRdfTj * S->top_beads;
        const long long cap = std::max(1LL, std::min(64LL, 0xffffffffLL / per_item));
        const long long want = (n_rdf + 2047) / 2048;
        const int K = (int)std::max(1LL, std::min(cap, want));
        rdf_ranges = system_blocks(rdf_sys, 0, n_rdf, K);
        S->n_rdf_ranges = (int)rdf_ranges.size();
    }
    // per-system slot lists (stable order) for the reducer
    // (the "E" plans add the centroid-Ewald slots, used while it is switched on)
    std::vector<int> red_f, red_a, red_fE, red_aE;
    const std::pair<int, int> ew_range{S->e_ew, S->n_eslots};
    S->nch_f = reducer_plan(eslot_sys, {{0, S->e_rp}}, n_sys, red_f, S->red_f_off);
    S->nch_a = reducer_plan(eslot_sys, {{0, S->e_ew}}, n_sys, red_a, S->red_a_off);
    S->nch_fE = reducer_plan(eslot_sys, {{0, S->e_rp}, ew_range}, n_sys, red_fE, S->red_fE_off);
    S->nch_aE = reducer_plan(eslot_sys, {{0, S->e_ew}, ew_range}, n_sys, red_aE, S->red_aE_off);
    std::vector<int> red_v, red_vE;   // velocity Verlet: no ring-polymer slots
    S->nch_v = reducer_plan(eslot_sys, {{0, S->e_rp}, {S->e_fin, S->e_ew}}, n_sys, red_v,
                            S->red_v_off);
    S->nch_vE = reducer_plan(eslot_sys, {{0, S->e_rp}, {S->e_fin, S->e_ew}, ew_range}, n_sys,
                             red_vE, S->red_vE_off);

    int rc = MIXPI_OK;
    auto T = [&](int r) {
        if (r && !rc) rc = r;
    };
    T(upload(&S->d_sys, B.sys));
    {
        // LJ tables in the sweep's form: 4 eps, sigma^2, V(rc), V'(rc)/rc
        std::vector<LjPar> td(B.lj_eps.size());
        for (const SysDev &sd : B.sys) {
            const double rc2 = sd.rc_lj * sd.rc_lj;
            for (int tp = 0; tp < sd.nt1 * sd.nt1; ++tp) {
                const size_t k = (size_t)sd.lj_off + tp;
                const double eps = B.lj_eps[k], sig = B.lj_sig[k];
                const double s2 = sig * sig;
                double c6 = s2 / rc2;
                c6 = c6 * c6 * c6;
                const double c12 = c6 * c6;
                td[k] = LjPar{4.0 * eps, s2, 4.0 * eps * (c12 - c6),
                              4.0 * eps * (-12.0 * c12 + 6.0 * c6) / rc2};
            }
        }
        T(upload(&S->d_ljpar, td));
    }
    T(upload(&S->d_charge, B.charge));
    T(upload(&S->d_ljt, B.ljt));
    T(upload(&S->d_mol, B.mol));
    T(upload(&S->d_row_sys, B.row_sys));
    T(upload(&S->d_row_fm, B.row_fm));
    T(upload(&S->d_row_hk, B.row_hk));
    T(upload(&S->d_blocks, B.blocks));
    T(upload(&S->d_items, items));
    {
        std::vector<PairBlock> ib(items.size());
        for (size_t k = 0; k < items.size(); ++k) ib[k] = B.blocks[items[k].block];
        T(upload(&S->d_iblocks, ib));
    }
    T(upload(&S->d_rdf_items, rdf_items));
    T(upload(&S->d_rdf_ranges, rdf_ranges));
    {
        std::vector<int> sp = B.sys_part;
        sp.push_back(B.n_part);
        T(upload(&S->d_parts, B.parts));
        {
            std::vector<unsigned char> ps(B.parts.size());
            for (size_t k = 0; k < ps.size(); ++k) ps[k] = (unsigned char)B.parts[k].spec;
            T(upload(&S->d_pspec, ps));
        }
        T(upload(&S->d_sys_part, sp));
        S->h_parts = B.parts;
        S->h_sys_part = sp;
        S->h_ew_z = B.ew_z;
    }
    T(upload(&S->d_bterms, terms));
    T(upload(&S->d_bblocks, bblocks));
    T(upload(&S->d_bond_k, B.bond_k));
    T(upload(&S->d_bond_r0, B.bond_r0));
    T(upload(&S->d_angle_k, B.angle_k));
    T(upload(&S->d_angle_t0, B.angle_t0));
    T(upload(&S->d_rp, rp));
    T(upload(&S->d_rp_nm, rp_nm));
    T(upload(&S->d_rp_lang, rp_lang));
    T(upload(&S->d_mf_cols, B.mf_cols.empty() ? std::vector<MfmaCol>(1, MfmaCol{}) : B.mf_cols));
    T(upload(&S->d_mf_tab, B.mf_tab.empty() ? std::vector<double>(1, 0.0) : B.mf_tab));
    if (S->n_mf_step > 0) T(upload(&S->d_row_spw, row_spw));
    T(upload(&S->d_circ, B.circ.empty() ? std::vector<double>(1, 0.0) : B.circ));
    T(upload(&S->d_row_stage, row_stage));
    T(upload(&S->d_stage_rows, stage_rows.empty() ? std::vector<long long>(1, 0) : stage_rows));
    T(upload(&S->d_stage, std::vector<double>((size_t)6 * std::max<size_t>(stage_rows.size(), 1), 0.0)));
    T(upload(&S->d_basis, B.basis));
    T(upload(&S->d_tw, B.tw));
    T(upload(&S->d_prop, B.prop));
    S->h_prop = B.prop;
    S->h_row_fm = B.row_fm;
    S->h_row_sys = B.row_sys;
    S->h_sys = B.sys;
    T(upload(&S->d_row_ptr, G.row_ptr));
    T(upload(&S->d_dest, G.dest.empty() ? std::vector<int>(1, -1) : G.dest));
    T(upload(&S->d_part, std::vector<double>((size_t)3 * std::max<long long>(G.row_ptr.back(), 1), 0.0)));
    T(upload(&S->d_fblocks, fblocks));
    T(upload(&S->d_eslot, std::vector<double>((size_t)2 * A_N * std::max(S->n_eslots, 1), 0.0)));
    T(upload(&S->d_red_f, red_f));
    T(upload(&S->d_red_a, red_a));
    T(upload(&S->d_red_v, red_v));
    T(upload(&S->d_red_fE, red_fE));
    T(upload(&S->d_red_aE, red_aE));
    T(upload(&S->d_red_vE, red_vE));
    T(upload(&S->d_row_prev, B.row_prev));
    T(upload(&S->d_row_next, B.row_next));
    T(upload(&S->d_row_ksp, B.row_ksp));
    {
        const int nch = std::max({1, S->nch_v, S->nch_f, S->nch_a, S->nch_vE, S->nch_fE, S->nch_aE});
        T(upload(&S->d_partial, std::vector<double>((size_t)A_N * nch, 0.0)));
    }
    T(upload(&S->d_npairs, std::vector<unsigned long long>(2, 0ull)));
    T(upload(&S->d_nonfinite, std::vector<int>(1, 0)));
    T(upload(&S->d_cent, std::vector<double>((size_t)3 * B.rows, 0.0)));
    T(upload(&S->d_scratch, std::vector<double>((size_t)9 * B.rows + MIXPI_NE * n_sys, 0.0)));
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

enum Part { ALL = 0, FAST = 1, SLOW = 2 };

double *eslot_buf(mixpi_system *s, int buf) { return s->d_eslot + (long long)buf * s->n_eslots * A_N; }

PairLaunch pair_args(mixpi_system *s, const double *q, const double *theta, int buf = 0)
{
    PairLaunch a{};
    a.items = s->d_items;
    a.n_items = s->n_items;
    a.tj = s->pair_tj_all;
    a.waves = s->pair_waves;
    a.iw = s->pair_iw;
    a.jrun = s->pair_jrun;
    a.iblocks = s->d_iblocks;
    a.sys = s->d_sys;
    a.ljpar = s->d_ljpar;
    a.charge = s->d_charge;
    a.ljt = s->d_ljt;
    a.mol = s->d_mol;
    a.q = q;
    a.part = s->d_part;
    a.dest = s->d_dest;
    a.theta = theta;
    a.eslot = eslot_buf(s, buf);
    return a;
}

BondedLaunch bonded_args(mixpi_system *s, const double *q, const double *theta, int buf = 0,
                         Part part = ALL)
{
    BondedLaunch b{};
    const int lo = part == SLOW ? s->n_bblocks_fast : 0;
    const int hi = part == FAST ? s->n_bblocks_fast : s->n_bblocks;
    b.terms = s->d_bterms;
    b.blocks = s->d_bblocks + lo;
    b.n_blocks = hi - lo;
    b.sys = s->d_sys;
    b.bond_k = s->d_bond_k;
    b.bond_r0 = s->d_bond_r0;
    b.angle_k = s->d_angle_k;
    b.angle_t0 = s->d_angle_t0;
    b.q = q;
    b.part = s->d_part;
    b.dest = s->d_dest;
    b.part_base = s->part_bonded;
    b.theta = theta;
    b.eslot = eslot_buf(s, buf) + (long long)(s->e_bonded + lo) * A_N;
    return b;
}

GatherArgs gather_args(mixpi_system *s)
{
    return GatherArgs{s->d_row_ptr, s->d_part};
}

// Stage A over buffer buf and stage B of the force-only slots (pair +
// bonded) or of the slots of a whole step.
enum { LIST_FORCE = 0, LIST_STEP = 1, LIST_VV = 2 };
const int *plan_of(mixpi_system *s, int list, const int **off, int *n)
{
    if (s->ew_use) {
        if (list == LIST_STEP) { *off = s->red_aE_off; *n = s->nch_aE; return s->d_red_aE; }
        if (list == LIST_VV) { *off = s->red_vE_off; *n = s->nch_vE; return s->d_red_vE; }
        *off = s->red_fE_off;
        *n = s->nch_fE;
        return s->d_red_fE;
    }
    if (list == LIST_STEP) { *off = s->red_a_off; *n = s->nch_a; return s->d_red_a; }
    if (list == LIST_VV) { *off = s->red_v_off; *n = s->nch_v; return s->d_red_v; }
    *off = s->red_f_off;
    *n = s->nch_f;
    return s->d_red_f;
}

ReduceA reduce_a_args(mixpi_system *s, int buf, int list)
{
    ReduceA r{};
    r.eslot = eslot_buf(s, buf);
    const int *off;
    const int *plan = plan_of(s, list, &off, &r.n_chunks);
    r.chunk_begin = plan + off[0];
    r.chunk_len = plan + off[1];
    r.partial = s->d_partial;
    return r;
}

ReduceB reduce_b_args(mixpi_system *s, int list)
{
    ReduceB r{};
    r.partial = s->d_partial;
    const int *off;
    int nch;
    const int *plan = plan_of(s, list, &off, &nch);
    r.sys_chunk = plan + off[2];
    r.n_wg = s->n_sys;
    r.sys = s->d_sys;
    r.n_sys = s->n_sys;
    r.npairs = s->d_npairs;
    r.nonfinite = s->d_nonfinite;
    return r;
}

// Centroid-Ewald launch arguments for positions q (outputs left unset).
EwaldLaunch ewald_args(mixpi_system *sys, const double *q)
{
    const auto &e = sys->ew;
    EwaldLaunch a{};
    a.parts = sys->d_parts;
    a.sys = sys->d_sys;
    a.sys_part = sys->d_sys_part;
    a.z = e.z;
    a.mol = sys->d_mol;
    a.q = q;
    a.cpos = e.cpos;
    a.freal = e.freal;
    a.fcent = e.fcent;
    a.spl_base = e.spl_base;
    a.spl_w = e.spl_w;
    a.grid_c = e.grid_c;
    a.G = e.G;
    a.tw = e.tw;
    a.e_real_part = e.e_real_part;
    a.e_recip_part = e.e_recip_part;
    a.real_items = e.real_items;
    a.real_first = e.real_first;
    a.e_const = e.e_const;
    a.alpha = e.alpha;
    a.r_cut = e.r_cut;
    a.scale = e.scale;
    a.inv_scale = 1.0 / e.scale;
    a.K = e.K;
    a.logK = e.logK;
    a.order = e.order;
    a.n_part = sys->n_part;
    a.n_sys = sys->n_sys;
    a.recip_wg = e.recip_wg;
    a.n_real = e.n_real;
    return a;
}

// The centroid-Ewald terms inside a force, energy or step pass: energies
// into the system's Ewald slot of buffer buf; bead forces added to f, or
// (step epilogue) written per row for the epilogue to add.
void enqueue_ewald_in_pass(mixpi_system *s, const double *q, double *f, int buf, bool rows,
                           hipStream_t st)
{
    EwaldLaunch a = ewald_args(s, q);
    a.f = rows ? nullptr : f;
    a.rowf = rows ? s->ew.rowf : nullptr;
    a.eslot_out = eslot_buf(s, buf) + (long long)s->e_ew * A_N;
    launch_ewald(a, st);
}

// Enqueues F(q): pair and bonded partials, then the per-row gather into f.
// The energy slots of the pair and bonded ranges are left for a reducer.
void enqueue_forces(mixpi_system *s, const double *q, const double *theta, double *f,
                    bool with_theta, hipStream_t st)
{
    launch_pair(pair_args(s, q, theta), bonded_args(s, q, theta), s->precision, with_theta, st);
    launch_gather(gather_args(s), s->rows, f, st, s->fin_rpw);
    if (s->ew_use) enqueue_ewald_in_pass(s, q, f, 0, false, st);
}

int last_launch_error()
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MIXPI_E_HIP, "kernel launch failed: %s", hipGetErrorString(e));
    return MIXPI_OK;
}

RpLaunch rp_args(mixpi_system *s, int op, const double *in, double *out, double *p, double *f,
                 int buf = 0, Part part = ALL)
{
    RpLaunch r{};
    const int lo = part == SLOW ? s->n_rp_fast : 0;
    const int hi = part == FAST ? s->n_rp_fast : s->n_rp;
    if (op == OP_STEP) {
        r.items = s->d_rp + lo;
        r.n_items = hi - lo;
    } else if (op == OP_FWD || op == OP_BWD) {
        r.items = s->d_rp_nm;
        r.n_items = s->n_rp_nm;
    } else {
        r.items = s->d_rp_lang;
        r.n_items = s->n_rp_lang;
    }
    r.mf_cols = s->d_mf_cols;
    r.mf_tab = s->d_mf_tab;
    r.precision = s->precision;
    r.circ = s->d_circ;
    r.stage = s->d_stage;
    r.lang = s->d_lang;
    r.row_stage = s->d_row_stage;
    r.row_hk = s->d_row_hk;
    r.sys = s->d_sys;
    r.basis = s->d_basis;
    r.twiddle = s->d_tw;
    r.prop = s->d_prop;
    r.op = op;
    r.in_q = in;
    r.out_q = out;
    r.p = p;
    r.f = f;
    r.cent = s->d_cent;
    r.eslot = eslot_buf(s, buf) + (long long)(s->e_rp + lo) * A_N;
    r.lds_bytes = op == OP_STEP ? s->rp_lds_step
                                : (op == OP_FWD || op == OP_BWD ? s->rp_lds_nm : s->rp_lds_lang);
    return r;
}

FinishLaunch finish_args(mixpi_system *s, const double *q, double *p, double *f, int buf = 0)
{
    FinishLaunch fl{};
    fl.blocks = s->d_fblocks;
    fl.rpw = s->fin_rpw;
    fl.n_blocks = s->n_fblocks;
    fl.uniform = s->n_sys == 1 ? 1 : 0;
    fl.rows = s->rows;
    fl.gather = gather_args(s);
    fl.row_fm = s->d_row_fm;
    fl.row_hk = s->d_row_hk;
    fl.p = p;
    fl.f = f;
    fl.q = q;
    fl.cent = s->d_cent;
    fl.eslot = eslot_buf(s, buf) + (long long)s->e_fin * A_N;
    fl.row_stage = s->d_row_stage;
    fl.stage = s->d_stage;
    fl.row_prev = s->d_row_prev;
    fl.row_next = s->d_row_next;
    fl.row_ksp = s->d_row_ksp;
    fl.row_spw = s->d_row_spw;
    return fl;
}

// Fills the stage rows of the circulant rings from (q, p, f) before a
// sequence of steps (later steps get them from the epilogue).
StageLaunch stage_args(mixpi_system *s, const double *q, const double *p, const double *f)
{
    StageLaunch a{};
    a.rows = s->d_stage_rows;
    a.n = s->n_stage;
    a.q = q;
    a.p = p;
    a.f = f;
    a.row_hk = s->d_row_hk;
    a.stage = s->d_stage;
    return a;
}

// Step k of a sequence: free ring polymers (with the first half-kick; extra
// workgroups sum the energy slots of step k-1 into chunk partials), pair and
// bonded partial forces, epilogue (gather F, second half-kick, kinetic sums;
// extra workgroups turn the partials into the log row of step k-1).  Steps
// alternate between the two energy-slot buffers so that the reduction of
// step k-1 never meets the writers of step k.
void enqueue_step(mixpi_system *s, int k, double *q, double *p, double *f, double *elog_prev,
                  hipStream_t st, bool count = true, bool vv = false)
{
    const int buf = k & 1;
    const int list = vv ? LIST_VV : LIST_STEP;
    // velocity Verlet: kick + drift on whole columns (transform items), the
    // spring force of the new positions and the spring energy in the epilogue
    RpLaunch r = rp_args(s, vv ? OP_VV : OP_STEP, q, q, p, f, buf);
    FinishLaunch fl = finish_args(s, q, p, f, buf);
    fl.vv = vv ? 1 : 0;
    if (k > 0) {
        r.with_reduce = 1;
        r.reduce = reduce_a_args(s, buf ^ 1, list);
        fl.with_reduce = 1;
        fl.reduce = reduce_b_args(s, list);
        fl.reduce.elog = elog_prev;
        if (!count) {
            fl.reduce.npairs = nullptr;
            fl.reduce.nonfinite = nullptr;
        }
    }
    launch_rp(r, st);
    launch_pair(pair_args(s, q, nullptr, buf), bonded_args(s, q, nullptr, buf), s->precision,
                false, st);
    if (s->ew_use) {
        enqueue_ewald_in_pass(s, q, nullptr, buf, true, st);
        fl.ew_rowf = s->ew.rowf;
    }
    launch_finish(fl, st);
}

// Finds or captures the graph of nsteps steps for these pointers.
// Langevin half steps (noise1, then noise2; either may be null) of the
// momenta of every ring in normal modes.
void enqueue_lang(mixpi_system *s, double *q, double *p, double *f, const double *noise1,
                  const double *noise2, hipStream_t st)
{
    RpLaunch r = rp_args(s, OP_LANG, q, q, p, f);
    r.noise1 = noise1;
    r.noise2 = noise2;
    launch_rp(r, st);
}

// Finds or captures the graph of nsteps steps for these pointers.  With
// noise ([nsteps][2][rows][3]) every step is O B A B O: the closing
// Langevin half step of step k and the opening one of step k+1 share one
// launch.
enum { MODE_NVE = 0, MODE_NVT = 1, MODE_VV = 2 };
int step_graph(mixpi_system *sys, int nsteps, double *q, double *p, double *f, double *elog,
               GraphEntry **out, const double *noise = nullptr, int mode = MODE_NVE)
{
    *out = nullptr;
    if (int rc = check_sys(sys)) return rc;
    if (nsteps < 0) return fail(MIXPI_E_INVALID, "nsteps must be >= 0");
    if (!q || !p || !f) return fail(MIXPI_E_INVALID, "q, p and f must be non-null");
    if (q == p || q == f || p == f) return fail(MIXPI_E_INVALID, "q, p and f must be distinct");
    if (noise && !sys->lang_set)
        return fail(MIXPI_E_INVALID, "no thermostat set (mixpi_set_thermostat)");
    if (nsteps == 0) return MIXPI_OK;
    HIP_TRY(hipSetDevice(sys->device));
    for (auto &g : sys->graphs)
        if (g.q == q && g.p == p && g.f == f && g.elog == elog && g.nsteps == nsteps &&
            g.noise == noise && g.mode == mode) {
            *out = &g;
            return MIXPI_OK;
        }
    if (sys->graphs.size() >= 8) {
        (void)hipGraphExecDestroy(sys->graphs.front().exec);
        (void)hipGraphDestroy(sys->graphs.front().graph);
        sys->graphs.erase(sys->graphs.begin());
    }
    GraphEntry g{q, p, f, elog, nsteps, nullptr, nullptr, noise, mode};
    auto row = [&](int k) { return elog ? elog + (size_t)k * sys->n_sys * MIXPI_NE : nullptr; };
    const size_t slice = (size_t)3 * sys->rows;    // one [rows][3] noise slice
    auto nz = [&](int k, int half) { return noise + (2 * (size_t)k + half) * slice; };
    HIP_TRY(hipStreamBeginCapture(sys->cap_stream, hipStreamCaptureModeRelaxed));
    const bool vv = mode == MODE_VV;
    if (noise) enqueue_lang(sys, q, p, f, nz(0, 0), nullptr, sys->cap_stream);
    else if (!vv) launch_stage(stage_args(sys, q, p, f), sys->cap_stream);
    for (int k = 0; k < nsteps; ++k) {
        enqueue_step(sys, k, q, p, f, k > 0 ? row(k - 1) : nullptr, sys->cap_stream, true, vv);
        if (noise)
            enqueue_lang(sys, q, p, f, nz(k, 1), k + 1 < nsteps ? nz(k + 1, 0) : nullptr,
                         sys->cap_stream);
    }
    {
        const int list = vv ? LIST_VV : LIST_STEP;
        ReduceB rb = reduce_b_args(sys, list);
        rb.elog = row(nsteps - 1);
        launch_reduce(reduce_a_args(sys, (nsteps - 1) & 1, list), rb, sys->cap_stream);
    }
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

int mixpi_layout(const mixpi_system *sys, int64_t *group_offsets, int32_t *n_groups)
{
    if (int rc = check_sys(sys)) return rc;
    if (!n_groups) return fail(MIXPI_E_INVALID, "n_groups is null");
    *n_groups = sys->n_groups;
    if (group_offsets) std::copy(sys->layout.begin(), sys->layout.end(), group_offsets);
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
    ReduceB rb = reduce_b_args(sys, LIST_FORCE);
    rb.e_out = e_out;
    launch_reduce(reduce_a_args(sys, 0, LIST_FORCE), rb, st);
    return last_launch_error();
}

int mixpi_forces_static(mixpi_system *sys, const double *q, const double *theta, double *f,
                        double *e_out, void *stream)
{
    if (int rc = check_sys(sys)) return rc;
    if (!q || !f) return fail(MIXPI_E_INVALID, "q and f must be non-null");
    if ((const void *)q == (const void *)f) return fail(MIXPI_E_INVALID, "f must not alias q");
    if (sys->ew_use)
        return fail(MIXPI_E_UNSUPPORTED, "mixpi_forces_static does not cover centroid Ewald "
                                         "terms (mixpi_use_ewald(sys, 0) first)");
    // scratch layout: partial-force positions [3 per position], the energy
    // slots of the force range [0, e_rp), the reducer's chunk partials;
    // each region 256-byte aligned
    auto up = [](size_t n) { return (n + 31) & ~size_t(31); };   // doubles, 256-byte steps
    const size_t n_part = up((size_t)3 * std::max<long long>(sys->n_positions, 1));
    const size_t n_eslot = up((size_t)A_N * std::max(sys->e_rp, 1));
    const size_t n_partial = up((size_t)A_N * std::max(sys->nch_f, 1));
    const size_t need = (n_part + n_eslot + n_partial) * sizeof(double);
    if (need > kStaticScratchBytes)
        return fail(MIXPI_E_UNSUPPORTED,
                    "mixpi_forces_static needs %zu bytes of scratch for this handle; the static "
                    "scratch holds %zu (use mixpi_forces)",
                    need, (size_t)kStaticScratchBytes);
    double *base = static_scratch_ptr(sys->device);
    if (!base) return fail(MIXPI_E_HIP, "static scratch not located on device %d", sys->device);
    double *part = base, *eslot = base + n_part, *partial = eslot + n_eslot;
    HIP_TRY(hipSetDevice(sys->device));
    hipStream_t st = (hipStream_t)stream;
    PairLaunch pa = pair_args(sys, q, theta);
    pa.part = part;
    pa.eslot = eslot;
    BondedLaunch ba = bonded_args(sys, q, theta);
    ba.part = part;
    ba.eslot = eslot + (long long)sys->e_bonded * A_N;
    launch_pair(pa, ba, sys->precision, false, st);
    GatherArgs ga = gather_args(sys);
    ga.part = part;
    launch_gather(ga, sys->rows, f, st, sys->fin_rpw);
    ReduceA ra = reduce_a_args(sys, 0, LIST_FORCE);
    ra.eslot = eslot;
    ra.partial = partial;
    ReduceB rb = reduce_b_args(sys, LIST_FORCE);
    rb.partial = partial;
    rb.e_out = e_out;
    launch_reduce(ra, rb, st);
    return last_launch_error();
}

int mixpi_energy(mixpi_system *sys, const double *q, const double *theta, double *e_out,
                 void *stream)
{
    if (int rc = check_sys(sys)) return rc;
    if (!q || !e_out) return fail(MIXPI_E_INVALID, "q and e_out must be non-null");
    HIP_TRY(hipSetDevice(sys->device));
    hipStream_t st = (hipStream_t)stream;
    launch_pair(pair_args(sys, q, theta), bonded_args(sys, q, theta), sys->precision, false, st);
    if (sys->ew_use) enqueue_ewald_in_pass(sys, q, nullptr, 0, false, st);
    ReduceB rb = reduce_b_args(sys, LIST_FORCE);
    rb.e_out = e_out;
    launch_reduce(reduce_a_args(sys, 0, LIST_FORCE), rb, st);
    return last_launch_error();
}

int mixpi_energy_adjoint(mixpi_system *sys, const double *q, const double *theta,
                         const double *grad_e, double *dq, double *dtheta, void *stream)
{
    if (int rc = check_sys(sys)) return rc;
    if (!q) return fail(MIXPI_E_INVALID, "q must be non-null");
    if ((const void *)q == (const void *)dq) return fail(MIXPI_E_INVALID, "dq must not alias q");
    if (sys->ew_use)
        return fail(MIXPI_E_UNSUPPORTED, "the adjoint does not cover centroid Ewald terms "
                                         "(mixpi_use_ewald(sys, 0) first)");
    HIP_TRY(hipSetDevice(sys->device));
    hipStream_t st = (hipStream_t)stream;
    launch_pair(pair_args(sys, q, theta), bonded_args(sys, q, theta), sys->precision, true, st);
    if (dq) {
        launch_gather(gather_args(sys), sys->rows, dq, st, sys->fin_rpw);
        launch_scale_rows(sys->rows, sys->d_row_sys, grad_e, dq, st);
    }
    ReduceB rb = reduce_b_args(sys, LIST_FORCE);
    rb.dtheta = dtheta;
    rb.grad_e = grad_e;
    launch_reduce(reduce_a_args(sys, 0, LIST_FORCE), rb, st);
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
    launch_rp(rp_args(sys, dir > 0 ? OP_FWD : OP_BWD, in, out, nullptr, nullptr),
              (hipStream_t)stream);
    return last_launch_error();
}

int mixpi_step_prepare(mixpi_system *sys, int32_t nsteps, double *q, double *p, double *f,
                       double *elog)
{
    GraphEntry *ge = nullptr;
    return step_graph(sys, nsteps, q, p, f, elog, &ge);
}

namespace {
int run_graph(mixpi_system *sys, GraphEntry *ge, void *stream);
}

int mixpi_step(mixpi_system *sys, int32_t nsteps, double *q, double *p, double *f, double *elog,
               void *stream)
{
    GraphEntry *ge = nullptr;
    if (int rc = step_graph(sys, nsteps, q, p, f, elog, &ge)) return rc;
    return run_graph(sys, ge, stream);
}

int mixpi_batch_step(mixpi_system *sys, int32_t nsteps, double *const *q, double *const *p,
                     double *const *f, double *elog, void *stream)
{
    if (int rc = check_sys(sys)) return rc;
    if (!q || !p || !f) return fail(MIXPI_E_INVALID, "q, p and f must be non-null arrays");
    const int n = sys->n_sys;
    bool packed = true;     // every system's arrays where the batch layout puts them
    for (int k = 0; k < n; ++k) {
        if (!q[k] || !p[k] || !f[k])
            return fail(MIXPI_E_INVALID, "system %d: null state pointer", k);
        const long long off = 3 * sys->sys_row0[k];
        packed = packed && q[k] == q[0] + off && p[k] == p[0] + off && f[k] == f[0] + off;
    }
    if (nsteps < 0) return fail(MIXPI_E_INVALID, "nsteps must be >= 0");
    if (packed) return mixpi_step(sys, nsteps, q[0], p[0], f[0], elog, stream);
    if (nsteps == 0) return MIXPI_OK;
    HIP_TRY(hipSetDevice(sys->device));
    const size_t words = 3 * (size_t)sys->rows;
    if (!sys->d_bstage) HIP_TRY(hipMalloc(&sys->d_bstage, 3 * words * sizeof(double)));
    double *sq = sys->d_bstage, *sp = sq + words, *sf = sp + words;
    hipStream_t st = (hipStream_t)stream;
    auto move = [&](bool in) -> hipError_t {
        for (int k = 0; k < n; ++k) {
            const long long off = 3 * sys->sys_row0[k];
            const size_t bytes = 3 * (size_t)(sys->sys_row0[k + 1] - sys->sys_row0[k]) * sizeof(double);
            double *const mine[3] = {sq + off, sp + off, sf + off};
            double *const theirs[3] = {q[k], p[k], f[k]};
            for (int a = 0; a < 3; ++a) {
                const hipError_t e =
                    in ? hipMemcpyAsync(mine[a], theirs[a], bytes, hipMemcpyDeviceToDevice, st)
                       : hipMemcpyAsync(theirs[a], mine[a], bytes, hipMemcpyDeviceToDevice, st);
                if (e != hipSuccess) return e;
            }
        }
        return hipSuccess;
    };
    HIP_TRY(move(true));
    if (int rc = mixpi_step(sys, nsteps, sq, sp, sf, elog, stream)) return rc;
    HIP_TRY(move(false));
    return MIXPI_OK;
}

int mixpi_set_thermostat(mixpi_system *sys, double tau0)
{
    if (int rc = check_sys(sys)) return rc;
    if (std::isnan(tau0)) return fail(MIXPI_E_INVALID, "tau0 is NaN");
    HIP_TRY(hipSetDevice(sys->device));
    // c1 = exp(-gamma dt/2), c2 = sqrt(1 - c1^2) sqrt(m_f k_B T) per mode row;
    // gamma = 1/tau0 for the centroid (0 if tau0 <= 0 or infinite), 2 omega_k
    // for mode k, omega_k^2 = k_spring lambda_k / m_f = 2 w4 / m_f with w4 the
    // spring entry k lambda_k / 2 of the propagation table
    const long long rows = sys->rows;
    std::vector<double> lang((size_t)2 * rows);
    const double g0 = (tau0 > 0.0 && std::isfinite(tau0)) ? 1.0 / tau0 : 0.0;
    for (long long r = 0; r < rows; ++r) {
        const SysDev &S = sys->h_sys[sys->h_row_sys[r]];
        const double dt = 2.0 * S.hkick / kKcal;
        const double fm = sys->h_row_fm[r];
        const double w4 = sys->h_prop[5 * (size_t)r + 4] * kKcal;     // amu A^2/fs^2 per A^2
        const double w = std::sqrt(2.0 * w4 / fm);
        const double gam = w4 > 0.0 ? 2.0 * w : g0;
        const double c1 = std::exp(-gam * 0.5 * dt);
        lang[2 * r] = c1;
        lang[2 * r + 1] = std::sqrt(1.0 - c1 * c1) * std::sqrt(fm * S.kT * kKcal);
    }
    if (!sys->d_lang) {
        hipError_t e = hipMalloc(&sys->d_lang, sizeof(double) * lang.size());
        if (e != hipSuccess) return fail(MIXPI_E_HIP, "hipMalloc: %s", hipGetErrorString(e));
    }
    HIP_TRY(hipMemcpy(sys->d_lang, lang.data(), sizeof(double) * lang.size(), hipMemcpyHostToDevice));
    sys->lang_set = true;
    return MIXPI_OK;
}

int mixpi_step_nvt(mixpi_system *sys, int32_t nsteps, double *q, double *p, double *f,
                   const double *noise, double *elog, void *stream)
{
    if (!noise) return fail(MIXPI_E_INVALID, "noise must be non-null");
    GraphEntry *ge = nullptr;
    if (int rc = step_graph(sys, nsteps, q, p, f, elog, &ge, noise, MODE_NVT)) return rc;
    return run_graph(sys, ge, stream);
}

int mixpi_step_vv(mixpi_system *sys, int32_t nsteps, double *q, double *p, double *f,
                  double *elog, void *stream)
{
    GraphEntry *ge = nullptr;
    if (int rc = step_graph(sys, nsteps, q, p, f, elog, &ge, nullptr, MODE_VV)) return rc;
    return run_graph(sys, ge, stream);
}

namespace {
int run_graph(mixpi_system *sys, GraphEntry *ge, void *stream)
{
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
}  // namespace

int mixpi_kernel_time(mixpi_system *sys, int32_t reps, const double *q, const double *p,
                      const double *f, double *avg_us, void *stream)
{
    if (int rc = check_sys(sys)) return rc;
    if (reps < 1 || reps > 1000 || !q || !p || !f || !avg_us)
        return fail(MIXPI_E_INVALID, "bad arguments (reps must be in [1, 1000])");
    if (sys->ew_use)
        return fail(MIXPI_E_UNSUPPORTED, "the per-launch timer covers the three step launches only "
                                         "(mixpi_use_ewald(sys, 0) first)");
    HIP_TRY(hipSetDevice(sys->device));
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = sizeof(double) * 3 * sys->rows;
    double *sq = sys->d_scratch, *sp = sq + 3 * sys->rows, *sf = sp + 3 * sys->rows;
    double *selog = sf + 3 * sys->rows;
    HIP_TRY(hipMemcpyAsync(sq, q, bytes, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(sp, p, bytes, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(sf, f, bytes, hipMemcpyDeviceToDevice, st));
    launch_stage(stage_args(sys, sq, sp, sf), st);
    // four timing-only events per step (no system-scope fence, so recording
    // them does not write back or invalidate caches between the launches)
    std::vector<hipEvent_t> ev(4 * (size_t)reps, nullptr);
    int rc = MIXPI_OK;
    for (auto &e : ev) {
        hipError_t h = hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
        if (h != hipSuccess) {
            rc = fail(MIXPI_E_HIP, "hipEventCreate: %s", hipGetErrorString(h));
            break;
        }
    }
    // chunks of 16 steps, each behind a bounded delay kernel (2 ms) that
    // holds the stream while the host enqueues the chunk, so the chunk's
    // launches run back to back and fit the hardware queue
    const int chunk = 16;
    for (int r0 = 0; r0 < reps && !rc; r0 += chunk) {
        launch_delay(200000LL, st);
        for (int r = r0; r < std::min(reps, r0 + chunk) && !rc; ++r) {
            const int buf = (r + 1) & 1;
            RpLaunch ra = rp_args(sys, OP_STEP, sq, sq, sp, sf, buf);
            ra.with_reduce = 1;
            ra.reduce = reduce_a_args(sys, buf ^ 1, LIST_STEP);
            FinishLaunch fl = finish_args(sys, sq, sp, sf, buf);
            fl.with_reduce = 1;
            fl.reduce = reduce_b_args(sys, LIST_STEP);
            fl.reduce.elog = selog;
            fl.reduce.npairs = nullptr;
            fl.reduce.nonfinite = nullptr;
            (void)hipEventRecord(ev[4 * r], st);
            launch_rp(ra, st);
            (void)hipEventRecord(ev[4 * r + 1], st);
            launch_pair(pair_args(sys, sq, nullptr, buf), bonded_args(sys, sq, nullptr, buf),
                        sys->precision, false, st);
            (void)hipEventRecord(ev[4 * r + 2], st);
            launch_finish(fl, st);
            if (hipEventRecord(ev[4 * r + 3], st) != hipSuccess)
                rc = fail(MIXPI_E_HIP, "hipEventRecord failed");
        }
    }
    if (!rc) {
        hipError_t h = hipStreamSynchronize(st);
        if (h != hipSuccess) rc = fail(MIXPI_E_HIP, "hipStreamSynchronize: %s", hipGetErrorString(h));
    }
    if (!rc) {
        double sum[3] = {0, 0, 0};
        for (int r = 0; r < reps; ++r)
            for (int k = 0; k < 3; ++k) {
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, ev[4 * r + k], ev[4 * r + k + 1]);
                sum[k] += ms;
            }
        // [0] force launch, [1] free ring polymer, [2] epilogue
        avg_us[0] = 1000.0 * sum[1] / reps;
        avg_us[1] = 1000.0 * sum[0] / reps;
        avg_us[2] = 1000.0 * sum[2] / reps;
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    if (rc) return rc;
    return last_launch_error();
}

int mixpi_rdf(mixpi_system *sys, const double *q, double r_max, int32_t nbins, int32_t nspec,
              double *hist, void *stream)
{
    if (int rc = check_sys(sys)) return rc;
    if (!q || !hist) return fail(MIXPI_E_INVALID, "q or hist is null");
    if (!(r_max > 0.0) || !std::isfinite(r_max))
        return fail(MIXPI_E_INVALID, "r_max must be positive and finite (got %g)", r_max);
    if (nbins < 1) return fail(MIXPI_E_INVALID, "nbins must be >= 1 (got %d)", nbins);
    if (nspec < sys->max_nt1)
        return fail(MIXPI_E_INVALID, "nspec = %d < %d species (LJ types + the null type)", nspec,
                    sys->max_nt1);
    const long long lds = (long long)sys->max_nt1 * (sys->max_nt1 + 1) / 2 * nbins * 4;
    if (lds > kRdfLdsBytes)
        return fail(MIXPI_E_UNSUPPORTED, "%d bins x %d species pairs exceed the %d-byte histogram",
                    nbins, sys->max_nt1 * (sys->max_nt1 + 1) / 2, kRdfLdsBytes);
    HIP_TRY(hipSetDevice(sys->device));
    RdfLaunch a{};
    a.items = sys->d_rdf_items;
    a.ranges = sys->d_rdf_ranges;
    a.blocks = sys->d_blocks;
    a.sys = sys->d_sys;
    a.ljt = sys->d_ljt;
    a.mol = sys->d_mol;
    a.q = q;
    a.hist = hist;
    a.rmax = r_max;
    a.unit = 1.0 / sys->top_beads;
    a.nbins = nbins;
    a.nspec = nspec;
    a.tj = kRdfTj;
    a.top = sys->top_beads;
    launch_rdf(a, sys->n_rdf_ranges, (int)lds, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return MIXPI_OK;
}

int mixpi_vacf_sample(mixpi_system *sys, const double *p, int64_t t, int32_t L, int32_t nspec,
                      double *ring, double *acc, void *stream)
{
    if (int rc = check_sys(sys)) return rc;
    if (!p || !ring || !acc) return fail(MIXPI_E_INVALID, "p, ring or acc is null");
    if (t < 0) return fail(MIXPI_E_INVALID, "t must be >= 0 (got %lld)", (long long)t);
    if (L < 1 || (long long)L * sys->n_sys > (1LL << 30))
        return fail(MIXPI_E_INVALID, "L must be in [1, 2^30 / systems] (got %d)", L);
    if (nspec < sys->max_nt1)
        return fail(MIXPI_E_INVALID, "nspec = %d < %d species (LJ types + the null type)", nspec,
                    sys->max_nt1);
    HIP_TRY(hipSetDevice(sys->device));
    TcfLaunch a{};
    a.parts = sys->d_parts;
    a.spec = sys->d_pspec;
    a.sys_part = sys->d_sys_part;
    a.sys = sys->d_sys;
    a.ring = ring;
    a.acc = acc;
    a.t = t;
    a.L = L;
    a.slot = (int)(t % L);
    a.n_lag = (int)std::min<int64_t>(t + 1, L);
    a.n_part = sys->n_part;
    a.n_sys = sys->n_sys;
    a.nspec = nspec;
    launch_tcf(a, p, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return MIXPI_OK;
}

namespace {
// Cardinal B-spline M_n(u) by its recursion (host tables of the SPME moduli).
double card_bspline(int n, double u)
{
    if (n == 2) return (u >= 0.0 && u <= 2.0) ? 1.0 - std::fabs(u - 1.0) : 0.0;
    return (u * card_bspline(n - 1, u) + (n - u) * card_bspline(n - 1, u - 1.0)) / (n - 1);
}
}  // namespace

int mixpi_set_ewald(mixpi_system *sys, double alpha, double r_cut, int32_t grid, int32_t order)
{
    if (int rc = check_sys(sys)) return rc;
    if (!finite_pos(alpha)) return fail(MIXPI_E_INVALID, "alpha must be positive and finite");
    if (!finite_pos(r_cut)) return fail(MIXPI_E_INVALID, "r_cut must be positive and finite");
    if (grid != 16 && grid != 32 && grid != 64)
        return fail(MIXPI_E_INVALID, "grid must be 16, 32 or 64 (got %d)", grid);
    if (order != 4 && order != 6 && order != 8)
        return fail(MIXPI_E_INVALID, "order must be 4, 6 or 8 (got %d)", order);
    const int n_sys = sys->n_sys, K = grid;
    for (int s = 0; s < n_sys; ++s)
        for (int k = 0; k < 3; ++k)
            if (r_cut > 0.5 * sys->h_sys[s].box[k])
                return fail(MIXPI_E_INVALID, "system %d: r_cut %g exceeds half the box (%g)", s,
                            r_cut, sys->h_sys[s].box[k]);
    HIP_TRY(hipSetDevice(sys->device));
    HIP_TRY(hipDeviceSynchronize());
    clear_graphs(sys);
    const bool was_in_use = sys->ew_use;   // kept across a successful reconfiguration
    sys->ew_use = false;
    release_ewald(sys);
    auto &e = sys->ew;
    e.alpha = alpha;
    e.r_cut = r_cut;
    e.K = K;
    e.logK = ilog2(K);
    e.order = order;
    const long long K3 = (long long)K * K * K;
    e.recip_wg = K * K / 16;   // x-line workgroups per system

    // Euler exponential spline moduli |b(m)|^2, the same on every axis
    std::vector<double> bmod(K);
    for (int m = 0; m < K; ++m) {
        double re = 0.0, im = 0.0;
        for (int k = 0; k <= order - 2; ++k) {
            const double Mk = card_bspline(order, k + 1.0);
            re += Mk * std::cos(2.0 * kPi * m * k / K);
            im += Mk * std::sin(2.0 * kPi * m * k / K);
        }
        bmod[m] = 1.0 / (re * re + im * im);
    }
    // influence function G = B C per system, constants, fixed-point scale
    std::vector<double> G((size_t)n_sys * K3), e_const(n_sys);
    double max_abs = 0.0;
    for (int s = 0; s < n_sys; ++s) {
        const SysDev &S = sys->h_sys[s];
        const double V = S.box[0] * S.box[1] * S.box[2];
        double Q = 0.0, z2 = 0.0, za = 0.0;
        for (int i = sys->h_sys_part[s]; i < sys->h_sys_part[s + 1]; ++i) {
            Q += sys->h_ew_z[i];
            z2 += sys->h_ew_z[i] * sys->h_ew_z[i];
            za += std::fabs(sys->h_ew_z[i]);
        }
        max_abs = std::max(max_abs, za);
        e_const[s] = -kCoulombKcal * alpha / std::sqrt(kPi) * z2 -
                     kCoulombKcal * kPi * Q * Q / (2.0 * V * alpha * alpha);
        double *g = G.data() + (size_t)s * K3;
        for (int m1 = 0; m1 < K; ++m1)
            for (int m2 = 0; m2 < K; ++m2)
                for (int m3 = 0; m3 < K; ++m3) {
                    const int a1 = m1 <= K / 2 ? m1 : m1 - K;
                    const int a2 = m2 <= K / 2 ? m2 : m2 - K;
                    const int a3 = m3 <= K / 2 ? m3 : m3 - K;
                    const double x = a1 / S.box[0], y = a2 / S.box[1], z = a3 / S.box[2];
                    const double msq = x * x + y * y + z * z;
                    const size_t k = ((size_t)m1 * K + m2) * K + m3;
                    g[k] = msq == 0.0 ? 0.0
                                      : bmod[m1] * bmod[m2] * bmod[m3] *
                                            std::exp(-kPi * kPi * msq / (alpha * alpha)) /
                                            (kPi * V * msq);
                }
    }
    // grid cells hold at most sum |z| (the weights of one particle sum to 1)
    const int bits = std::min(50, 61 - (int)std::ceil(std::log2(max_abs + 1.0)));
    e.scale = std::ldexp(1.0, bits);
    std::vector<double2> tw(K / 2);
    for (int j = 0; j < K / 2; ++j)
        tw[j] = make_double2(std::cos(2.0 * kPi * j / K), -std::sin(2.0 * kPi * j / K));
    // real-space workgroups: 64-particle i-tiles x kEwChunk-particle j-chunks
    // of each system, in system order
    std::vector<RealItem> items;
    std::vector<int> first(n_sys + 1, 0);
    int max_chunks = 1;
    for (int s = 0; s < n_sys; ++s) {
        first[s] = (int)items.size();
        const int p0 = sys->h_sys_part[s], p1 = sys->h_sys_part[s + 1];
        int c = 0;
        for (int j0 = p0; j0 < p1; j0 += kEwChunk, ++c)
            for (int i0 = p0; i0 < p1; i0 += 64)
                items.push_back(RealItem{s, i0, std::min(64, p1 - i0), j0,
                                         std::min(kEwChunk, p1 - j0), c});
        max_chunks = std::max(max_chunks, c);
    }
    first[n_sys] = (int)items.size();
    e.n_real = (int)items.size();

    int rc = MIXPI_OK;
    auto T = [&](int r) {
        if (r && !rc) rc = r;
    };
    const size_t np3 = (size_t)std::max(1, sys->n_part) * 3;
    T(upload(&e.z, sys->h_ew_z));
    T(upload(&e.G, G));
    T(upload(&e.tw, tw));
    T(upload(&e.e_const, e_const));
    T(upload(&e.real_items, items));
    T(upload(&e.real_first, first));
    T(alloc(&e.cpos, np3));
    T(alloc(&e.freal, np3 * max_chunks));
    T(alloc(&e.fcent, np3));
    T(alloc(&e.rowf, (size_t)3 * std::max<long long>(1, sys->rows)));
    T(alloc(&e.spl_base, (size_t)4 * std::max(1, sys->n_part)));
    T(alloc(&e.spl_w, (size_t)3 * kMaxOrder * std::max(1, sys->n_part)));
    T(alloc(&e.grid_c, (size_t)n_sys * K3));
    T(alloc(&e.e_real_part, (size_t)std::max(1, e.n_real)));
    T(alloc(&e.e_recip_part, (size_t)n_sys * e.recip_wg));
    if (!rc && hipDeviceSynchronize() != hipSuccess)
        rc = fail(MIXPI_E_HIP, "device synchronisation failed");
    if (rc) {
        release_ewald(sys);
        return rc;
    }
    e.on = true;
    sys->ew_use = was_in_use;
    return MIXPI_OK;
}

int mixpi_ewald(mixpi_system *sys, const double *q, double *f, double *e_out, void *stream)
{
    if (int rc = check_sys(sys)) return rc;
    if (!sys->ew.on) return fail(MIXPI_E_INVALID, "call mixpi_set_ewald first");
    if (!q || !e_out) return fail(MIXPI_E_INVALID, "q or e_out is null");
    HIP_TRY(hipSetDevice(sys->device));
    EwaldLaunch a = ewald_args(sys, q);
    a.f = f;
    a.e_out = e_out;
    launch_ewald(a, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return MIXPI_OK;
}

int mixpi_use_ewald(mixpi_system *sys, int32_t on)
{
    if (int rc = check_sys(sys)) return rc;
    if (on && !sys->ew.on) return fail(MIXPI_E_INVALID, "call mixpi_set_ewald first");
    HIP_TRY(hipSetDevice(sys->device));
    if ((bool)on != sys->ew_use) {
        HIP_TRY(hipDeviceSynchronize());
        clear_graphs(sys);
    }
    sys->ew_use = on != 0;
    return MIXPI_OK;
}

int mixpi_pair_shape(const mixpi_system *sys, int32_t *tj, int32_t *waves, int32_t *i_waves,
                     int32_t *j_run)
{
    if (int rc = check_sys(sys)) return rc;
    if (tj)
        for (int y = 0; y < sys->n_sys; ++y) tj[y] = sys->pair_tj[y];
    if (waves) *waves = sys->pair_waves;
    if (i_waves) *i_waves = sys->pair_iw;
    if (j_run) *j_run = sys->pair_jrun;
    return MIXPI_OK;
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
    unsigned long long h[2];
    HIP_TRY(hipMemcpyAsync(h, sys->d_npairs, sizeof h, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (evals) {
        evals[0] = (int64_t)h[0];
        evals[1] = (int64_t)h[1];
    }
    if (reset) {
        HIP_TRY(hipMemsetAsync(sys->d_npairs, 0, sizeof h, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    return MIXPI_OK;
}

}  // extern "C"
