// Internal structures of libmixpi shared by host code and kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mixpi {

// ---- physical constants (SI / CODATA 2022; the library's own copy) ---------
constexpr double kPi = 3.14159265358979323846;
constexpr double kAmuKg = 1.66053906892e-27;
constexpr double kPlanckSI = 6.62607015e-34;
constexpr double kBoltzSI = 1.380649e-23;
constexpr double kAvogadro = 6.02214076e23;
constexpr double kCoulombKcal = 332.0637133;  // e^2/(4 pi eps0), kcal A/mol
// amu A^2 / fs^2 in J
constexpr double kInternalJ = kAmuKg * 1e-20 / 1e-30;
// 1 kcal/mol in amu A^2 / fs^2
constexpr double kKcal = 4184.0 / kAvogadro / kInternalJ;
constexpr double kHbar = kPlanckSI / (2.0 * kPi) / (kAmuKg * 1e-20 / 1e-15);  // amu A^2/fs
constexpr double kBoltz = kBoltzSI / kInternalJ;                            // amu A^2/fs^2/K
constexpr double kBoltzKcal = kBoltzSI * kAvogadro / 4184.0;                 // kcal/mol/K

constexpr int kMaxLjTypes = 8;           // user types; one extra null type
constexpr int kLjTab = (kMaxLjTypes + 1) * (kMaxLjTypes + 1);
constexpr int kMaxBeads = 4096;
constexpr int kDenseMaxN = 64;           // normal modes by dense basis up to N

// Energy partials.  Every writer (pair tile, bonded block, normal-mode
// item, epilogue block) owns one slot of A_N doubles and stores its sums
// there; a reducer adds the slots of each system and writes the energies.
// Only the reducer's few per-system sums are shared addresses.
enum {
    A_LJ = 0, A_COUL, A_PP, A_BOND, A_ANGLE, A_SPRING, A_KIN, A_VIR,
    A_TH0, A_TH1, A_TH2, A_TH3, A_TH4, A_TH5, A_CNT_AA, A_CNT_EA, A_N = 16
};
constexpr int kMaxSystems = 1024;   // systems per batched handle

struct SysDev {
    double box[3], ibox[3];
    double rc_lj, rc_c, rc_pp;
    double theta0[6];     // pp_q, pp_a, eps_00, sigma_00, k_bond0, k_angle0
    double irc, irc3;     // 1 / rc_c and 1 / rc_c^3 (0 when rc_c = 0)
    // 1 / sqrt(u), -1 / u^(3/2), 1 / u^(5/2) at u = rc_pp^2 + pp_a^2 (theta0)
    double pp_phic, pp_psic, pp_chic;
    double bg_energy;     // uniform-background constant (kcal/mol)
    double kT;            // kcal/mol
    double cv_const;      // sum_i 3/(2 beta)
    double prim_const;    // sum_i 3 N_i/(2 beta)
    double hkick;         // dt/2 * kcal -> momentum units
    int lj_off;           // offset into the LJ tables ((nt+1)^2 entries)
    int nt1;              // LJ types + 1 (null type = nt)
    int bond_off;         // global index of this system's bond type 0
    int angle_off;        // global index of this system's angle type 0
};

// A pair block: all slice-pairs between particle group a (larger or equal
// bead count, N_a) and group b (N_b = N_a >> shift).  For j-bead b the
// i-list is the contiguous rows of group a at beads [b << shift, (b+1) << shift).
enum { PK_ATOM = 0, PK_E_ATOM = 1, PK_ATOM_E = 2 };
struct PairBlock {
    int sys, kind, same, shift;
    int na, nb;           // particles in groups a, b
    int pa0, pb0;         // first global particle of a, b
    long long rowa, rowb; // first bead row of groups a, b
    double w;             // 1 / N_a
    int nbeads_b;         // N_b
    int lj;               // some type pair of the two groups may have LJ (atom blocks)
    int sparse;           // atom block swept in compacted form (few in-cutoff candidates)
    int lj_off, nt1;      // the system's LJ table offset and LJ types + 1
    int mol;              // some pair of the two groups may share a molecule id
    int cull;             // electron-atom block whose tiles cull unreachable j-atoms
};

// LJ parameters of one type pair in the form the pair sweep uses: 4 eps,
// sigma^2, c0 = V(rc) and c1 = V'(rc) / rc of the unshifted potential.
struct alignas(16) LjPar {
    double e4, s2, c0, c1;
};
// A pair-sweep item of a pair block (iw: the launch's i-split waves): j-bead
// b, i-beads [i0, i0 + 64 iw) of the block's i-run against nj consecutive
// j-tiles of tj particles from j0 (a j-run).  Its i-forces go to natural
// partial-force slots islot + [0, 64 iw), the reactions of j-tile k to
// jslot + k tj + [0, tj).
struct PairItem {
    int block, b, i0, j0;
    int tj, islot, jslot, nj;
};
constexpr int kMaxTj = 64;

// One slice of a bonded term: kind 0 = bond (r[0], r[1]), kind 1 = angle
// (end r[0], vertex r[1], end r[2]); w = 1 / N_max.  Owns partial-force
// slots 3t, 3t+1, 3t+2 of the bonded range.
struct BondedTerm {
    int r[3];
    int type, kind, sys;
    double w;
};

// A workgroup's share of a list, never spanning two systems.
struct BlockRange {
    int sys, begin, count, pad;
};

// free ring-polymer / normal-mode work item
enum { RP_DENSE = 0, RP_FFT = 1, RP_CIRC = 2, RP_MFMA = 3 };
// A column of an MFMA item: component d of one ring.  Bead j of the column is
// element (row0 + j * stride) * 3 + d of a state array, and stage row
// srow0 + j * stride (propagation items; -1 otherwise).
struct MfmaCol {
    long long row0, srow0;
    int stride, d;
};
constexpr int kMfCols = 16;        // columns of an MFMA item (the instructions' 16-wide N)
constexpr int kMfRows = 16;        // output rows of an MFMA item
constexpr int kMfMinN = 16;        // smallest ring an MFMA item takes
constexpr int kCircOut = 16;       // bead outputs per circulant item
constexpr int kCircJg = 256 / (kCircOut / 4);   // j-groups of a circulant item (4 outputs per thread)
constexpr int kCircMaxN = 2048;    // largest ring propagated in bead space
enum { OP_STEP = 0, OP_FWD = 1, OP_BWD = 2, OP_LANG = 3, OP_VV = 4 };
struct RpItem {
    int kind, sys, N, logN;
    int n;                // particles in the group
    int p0;               // first global particle of the group
    long long row;        // first bead row of the group
    int c0, ncols;        // dense: column range (particle*3 + dim); fft: column c0
    int basis_off;        // offset (doubles) of the dense basis of size N
    int tw_off;           // offset (complex) of the stage-major twiddle table of N
    int o0;               // circulant: first bead output of the item
    int circ_off;         // circulant: offset (doubles) of the particle's a, b, c rows
    int stage0;           // circulant: stage row of the group's first bead row
    double wsp;           // circulant: spring energy per squared bead step, kcal/mol/A^2
    double dtm;           // MFMA propagation: dt / m_f of its columns (sum of the b row)
};

// ---- launchers (defined in the .hip files) --------------------------------
struct PairLaunch {
    const PairItem *items;
    int n_items;
    int tj;                  // j-tile width of every item (16, 32, 64), or 0: per item
    int waves;               // j-split waves per tile (1 or 2)
    int iw;                  // i-split waves per tile (1, 2 or 4; with waves = 1)
    int jrun;                // most j-tiles of an item (natural slot stride 64 iw + jrun tj)
    const PairBlock *iblocks; // the block of every item, copied per item
    const SysDev *sys;
    const LjPar *ljpar;      // per system at lj_off: (nt+1)^2 type pairs
    const double *charge;
    const int *ljt, *mol;
    const double *q;
    double *part;            // partial forces [positions][3], row-contiguous
    const int *dest;         // position of every natural slot (-1: unused)
    const double *theta;
    double *eslot;           // energy slot of item k: eslot + k * A_N
};

struct BondedLaunch {
    const BondedTerm *terms;
    const BlockRange *blocks; // one per workgroup (256 terms, one system)
    int n_blocks;
    const SysDev *sys;
    const double *bond_k, *bond_r0, *angle_k, *angle_t0;
    const double *q;
    double *part;            // partial forces [positions][3], row-contiguous
    const int *dest;         // position of every natural slot
    long long part_base;     // term t owns natural slots part_base + 3t .. +2
    const double *theta;
    double *eslot;           // energy slot of this launch's block b: eslot + b * A_N
};
// One launch: the pair tiles, then the bonded workgroups (64 terms each).
void launch_pair(const PairLaunch &a, const BondedLaunch &b, int precision, bool with_theta,
                 hipStream_t st);
// The bonded workgroups alone.
void launch_bonded(const BondedLaunch &b, bool with_theta, hipStream_t st);

// Energy reduction in two stages, each a few workgroups that ride along in
// the launches of the next step (or run alone):
//   A: chunk c of a slot list (at most kChunkSlots slots of one system)
//      summed into partial[c][A_N];
//   B: the chunks of each system summed in order and turned into the
//      outputs: e_out [n_sys][NV] or an energy-log row [n_sys][NE], the
//      pair-evaluation counts (npairs[2]) and grad_e * dV/dtheta.
// Every sum has one writer and a fixed order.
constexpr int kChunkSlots = 64;
constexpr int kReduceThreads = 256;   // a multiple of A_N
struct ReduceA {
    const double *eslot;
    const int *chunk_begin;    // [n_chunks] first slot
    const int *chunk_len;      // [n_chunks] slots
    int n_chunks;
    double *partial;           // [n_chunks][A_N]
};
struct ReduceB {
    const double *partial;
    const int *sys_chunk;      // [n_sys + 1] first chunk of each system
    int n_wg;                  // workgroups: one per system
    const SysDev *sys;
    int n_sys;
    double *e_out;             // [n_sys][NV] or null
    double *elog;              // [n_sys][NE] or null
    double *dtheta;            // [n_sys][6] or null
    const double *grad_e;      // [n_sys] or null (= 1)
    unsigned long long *npairs;
    int *nonfinite;
};

struct RpLaunch {
    const RpItem *items;
    int n_items;
    const SysDev *sys;
    const double *basis;     // dense bases C[j*N+k] then C^T, per N
    const double2 *twiddle;  // per N, stage-major exp(-2 pi i pos / 2^s), N - 1 entries
    const double *prop;      // [rows][5] a, b, c, d, spring coefficient
    const double *circ;      // circulant propagator rows a_d, b_d, c_d per particle
    // MFMA items: their columns, and the generator tables (propagation: rows
    // a_d, b_d, c_d of a propagator class; transforms: cos(2 pi m / N))
    const MfmaCol *mf_cols;
    const double *mf_tab;
    int precision;           // transforms: 0 FP64 matrix instructions, 1 FP32 with FP64 sums
    double *stage;           // circulant rings' step inputs [stage rows][6]: q, p + dt/2 F
                             // (read by OP_STEP, written by OP_LANG)
    // OP_LANG: Langevin half steps of p in normal modes, pi <- c1 pi + c2 eta
    const double *lang;      // [rows][2] c1, c2 (momentum units) per mode row
    const double *noise1;    // [rows][3] mode-indexed standard normals, or null
    const double *noise2;    // a second half step after the first, or null
    const int *row_stage;    // [rows] stage row of a circulant ring's bead row, or -1
    const double *row_hk;    // [rows] dt/2 in momentum units
    int op;
    const double *in_q;      // OP_STEP: q (in/out via out_q); FWD/BWD: input
    double *out_q;
    double *p;               // OP_STEP only
    double *f;               // OP_STEP only: read (first half-kick)
    double *cent;            // OP_STEP only: [rows][3] centroid of each bead's ring
    double *eslot;           // OP_STEP only: energy slot of item b: eslot + b * A_N
    unsigned lds_bytes;      // dynamic LDS: max over the items
    int with_reduce;         // reduce.n_chunks extra workgroups run stage A
    ReduceA reduce;
};
void launch_rp(const RpLaunch &a, hipStream_t st);

// LDS of an MFMA item: the generator table as FP64 or FP32 (propagation: the
// a, b, c rows; transforms: the cos table), then the four waves' results
// ([wave][2][4][64] doubles) and column sums ([wave][2][64]).
__host__ __device__ inline unsigned mfma_tab_doubles(int N, int op, int precision)
{
    const unsigned n = (unsigned)((op == OP_STEP ? 3 : 1) * N);
    const unsigned bytes = n * (precision ? 4u : 8u);
    return ((bytes + 7) / 8 + 31) / 32 * 32;
}
__host__ __device__ inline unsigned mfma_lds_bytes(int N, int op, int precision)
{
    return (mfma_tab_doubles(N, op, precision) + 4 * 2 * 4 * 64 + 4 * 2 * 64) * 8;
}
const void *rp_kernel_symbol();

// Gathers F[row] = sum of its partial-force slots.  The slots of a row are
// contiguous (CSR order): writers store each partial at its position
// dest[natural slot], so a row reads one contiguous run.
struct GatherArgs {
    const long long *row_ptr;  // [rows + 1]
    const double *part;        // [positions][3]
};

struct FinishLaunch {
    const BlockRange *blocks;  // one per workgroup: 4 rpw bead rows of one system
    int n_blocks;
    // one system: block b is rows [b * 4 rpw, (b + 1) * 4 rpw) of `rows`,
    // formed from the workgroup index (blocks unread)
    int uniform;
    long long rows;
    int rpw;                   // bead rows per wave: 1, 2 or 4
    GatherArgs gather;
    const double *row_fm;      // [rows] fictitious mass of the bead row
    const double *row_hk;      // [rows] dt/2 in momentum units of its system
    double *p;
    double *f;                 // written: gathered forces
    const double *q, *cent;
    double *eslot;             // energy slot of block b: eslot + b * A_N
    const int *row_stage;      // [rows] stage row of a circulant ring's bead row, or -1
    double *stage;             // written for those rows: q, p + dt/2 F (next step's input)
    int with_reduce;           // reduce.n_wg extra workgroups run stage B
    ReduceB reduce;
    // velocity Verlet with spring forces: the kick adds F_sp of the new q
    // (neighbour bead rows), and the spring energy of (row, next) is summed
    int vv;
    const long long *row_prev, *row_next;  // [rows] neighbour bead rows of the ring
    const double *row_ksp;                 // [rows] spring constant, kcal/mol/A^2
    // split-propagator steps: the spring energy k/2 |q - q_next|^2 of the
    // rows whose ring the matrix-core items propagate (row_spw = k/2 there,
    // 0 elsewhere; null: none)
    const double *row_spw;
    const double *ew_rowf;                 // [rows][3] centroid-Ewald force, added (may be null)
};
void launch_finish(const FinishLaunch &a, hipStream_t st);

// Fills the circulant rings' stage rows from (q, p, f): q, p + dt/2 f.
struct StageLaunch {
    const long long *rows;     // [n] bead row of each stage row
    int n;
    const double *q, *p, *f, *row_hk;
    double *stage;
};
void launch_stage(const StageLaunch &a, hipStream_t st);

void launch_reduce(const ReduceA &a, const ReduceB &b, hipStream_t st);

// Radial-distribution histogram over the pair tiles (one workgroup per
// system-pure range of tiles; dynamic LDS = (nt1 (nt1 + 1) / 2) nbins words).
struct RdfLaunch {
    const PairItem *items;
    const BlockRange *ranges;
    const PairBlock *blocks;
    const SysDev *sys;
    const int *ljt, *mol;
    const double *q;
    double *hist;            // [systems][nspec][nspec][nbins], added to
    double rmax, unit;       // unit = 1 / top
    int nbins, nspec, tj, top;
};
constexpr int kRdfLdsBytes = 56 * 1024;
constexpr int kRdfTj = 64;         // j-tile width of the histogram's tiles
void launch_rdf(const RdfLaunch &a, int n_ranges, int lds_bytes, hipStream_t st);

// A particle for centroid quantities: bead j sits at row row0 + j * stride.
struct PartDev {
    long long row0;
    int stride, nb;
    double inv_nm;           // 1 / (N m_f)
    int spec, sys;           // species (LJ type, null type nt), system
};

// One sample of the centroid velocity correlator.
struct TcfLaunch {
    const PartDev *parts;
    const unsigned char *spec;   // [n_part] species, as parts[i].spec (one byte per particle)
    const int *sys_part;     // [n_sys + 1] first particle of each system
    const SysDev *sys;
    double *ring;            // [L][n_part][3]
    double *acc;             // [n_sys][nspec][L], added to
    long long t;
    int L, slot, n_lag, n_part, n_sys, nspec;
};
void launch_tcf(const TcfLaunch &a, const double *p, hipStream_t st);

// Real-space Ewald work item: particles [i0, i0 + ni) against the j-chunk
// [j0, j0 + nj) (chunk-th kEwChunk-particle chunk of the system).
constexpr int kEwChunk = 64;
constexpr int kMaxOrder = 8;     // largest B-spline order
struct RealItem {
    int sys, i0, ni, j0, nj, chunk;
};

// Centroid Ewald electrostatics (all systems of a handle, one grid each).
struct EwaldLaunch {
    const PartDev *parts;
    const SysDev *sys;
    const int *sys_part;         // [n_sys + 1]
    const double *z;             // Ewald charge per particle (0 for electrons)
    const int *mol;
    const double *q;             // bead rows
    double *f;                   // bead rows, added to (may be null)
    double *rowf;                // bead rows, written: F_i / N_i (may be null)
    double *eslot_out;           // energy slot row per system (may be null): A_COUL = total
    double *cpos, *fcent;        // [n_part][3]
    double *freal;               // [max chunks][n_part][3] real-space partials
    int *spl_base;               // [n_part][4] grid bases floor(u) of x, y, z
    double *spl_w;               // [n_part][3][kMaxOrder] B-spline weights
    double2 *grid_c;             // [n_sys][K^3]
    const double *G;             // [n_sys][K^3] influence function B C
    const double2 *tw;           // exp(-2 pi i j / K), j < K/2
    double *e_real_part;         // [n_real]
    double *e_recip_part;        // [n_sys][recip_wg]
    const RealItem *real_items;
    const int *real_first;       // [n_sys + 1] first real item of each system
    const double *e_const;       // [n_sys] self + background
    double *e_out;               // [n_sys][3] (may be null)
    double alpha, r_cut, scale, inv_scale;
    int K, logK, order, n_part, n_sys, recip_wg, n_real;
    int tw_in_lds;               // plane launches: twiddles staged after the plane
};
void launch_ewald(const EwaldLaunch &a, hipStream_t st);

// Static device scratch of mixpi_forces_static (defined in misc.hip): its
// size, the per-device lookup of its address (at handle creation, with the
// device current) and the address found for a device (null before).
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
constexpr int kMaxDevices = 64;
hipError_t static_scratch_init(int device);
double *static_scratch_ptr(int device);

void launch_fill(double *x, long long n, double v, hipStream_t st);
void launch_delay(long long ticks_100mhz, hipStream_t st);
void launch_gather(const GatherArgs &g, long long rows, double *f, hipStream_t st, int rpw);
void launch_scale_rows(long long rows, const int *row_sys, const double *grad_e, double *dq,
                       hipStream_t st);

}  // namespace mixpi
