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
constexpr int kPairTile = 64;            // i and j tile of the pair kernel

// per-system accumulator slots (device, FP64).  Each system owns
// kAccCopies copies of the slot row; a workgroup adds into copy
// blockIdx.x % kAccCopies so same-address atomics are spread out, and the
// reader sums the copies.
enum {
    A_LJ = 0, A_COUL, A_PP, A_BOND, A_ANGLE, A_SPRING, A_KIN, A_VIR,
    A_TH0, A_TH1, A_TH2, A_TH3, A_TH4, A_TH5, A_N = 16
};
constexpr int kAccCopies = 16;
__host__ __device__ inline double *acc_row(double *eacc, int sys, unsigned blk)
{
    return eacc + ((long long)sys * kAccCopies + (blk % kAccCopies)) * A_N;
}

struct SysDev {
    double box[3], ibox[3];
    double rc_lj, rc_c, rc_pp;
    double theta0[6];     // pp_q, pp_a, eps_00, sigma_00, k_bond0, k_angle0
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
};
struct PairItem {
    int block, b, i0, j0;
};

struct BondTerm {
    int ra, rb, type, sys;
    double w;
};
struct AngleTerm {
    int ra, rv, rb, type;
    int sys, pad;
    double w;
};

// free ring-polymer / normal-mode work item
enum { RP_DENSE = 0, RP_FFT = 1 };
enum { OP_STEP = 0, OP_FWD = 1, OP_BWD = 2 };
struct RpItem {
    int kind, sys, N, logN;
    int n;                // particles in the group
    int p0;               // first global particle of the group
    long long row;        // first bead row of the group
    int c0, ncols;        // dense: column range (particle*3 + dim); fft: column c0
    int basis_off;        // offset (doubles) of the dense basis of size N
    int tw_off;           // offset (complex) of the twiddle table of size N
};

// ---- launchers (defined in the .hip files) --------------------------------
struct PairLaunch {
    const PairItem *items;
    int n_items;
    const PairBlock *blocks;
    const SysDev *sys;
    const double *lj_eps, *lj_sig;
    const double *charge;
    const int *ljt, *mol;
    const double *q;
    double *f;
    const double *theta;
    double *eacc;
    unsigned long long *npairs;
};
void launch_pair(const PairLaunch &a, int precision, bool with_theta, hipStream_t st);

struct BondedLaunch {
    const BondTerm *bonds;
    int n_bonds;
    const AngleTerm *angles;
    int n_angles;
    const SysDev *sys;
    const double *bond_k, *bond_r0, *angle_k, *angle_t0;
    const double *q;
    double *f;
    const double *theta;
    double *eacc;
};
void launch_bonded(const BondedLaunch &a, bool with_theta, hipStream_t st);

struct RpLaunch {
    const RpItem *items;
    int n_items;
    const SysDev *sys;
    const double *basis;     // dense bases C[j*N+k] then C^T, per N
    const double2 *twiddle;  // exp(-2 pi i m / N), m < N/2, per N
    const double *prop;      // [rows][5] a, b, c, d, spring coefficient
    int op;
    const double *in_q;      // OP_STEP: q (in/out via out_q); FWD/BWD: input
    double *out_q;
    double *p;               // OP_STEP only
    double *f;               // OP_STEP only: read (kick) then zeroed
    double *cent;            // OP_STEP only: [particles][3]
    double *eacc;            // OP_STEP only
    unsigned lds_bytes;      // dynamic LDS: max over the items
};
void launch_rp(const RpLaunch &a, hipStream_t st);
const void *rp_kernel_symbol();

struct FinishLaunch {
    long long n3;            // 3 * rows
    const int *row_part;     // [rows] global particle
    const int *part_sys;     // [particles]
    const double *fm;        // [particles]
    const SysDev *sys;
    int n_sys;
    double *p;
    const double *f, *q, *cent;
    double *eacc;
    double *elog;            // row for this step, [n_sys][NE], or null
    unsigned *ticket;
    int *nonfinite;
};
void launch_finish(const FinishLaunch &a, hipStream_t st);

void launch_fill(double *x, long long n, double v, hipStream_t st);
void launch_write_energy(const SysDev *sys, int n_sys, double *eacc, double *e_out,
                         hipStream_t st);
void launch_adjoint_finish(const SysDev *sys, int n_sys, long long rows,
                           const int *row_part, const int *part_sys,
                           const double *grad_e, double *dq, double *eacc,
                           double *dtheta, hipStream_t st);

}  // namespace mixpi
