/*
 * mixpi.h -- C-ABI of the MI355X (gfx950) mixed-time-slicing PIMD hot path.
 *
 * The library computes, on one GPU, the per-step work of mixTS path-integral
 * molecular dynamics as defined in arXiv 2411.11988 ("MixPI"):
 *   - bead forces of V_mix, Eq. (mts-hamiltonian): every pair, bond and angle
 *     is evaluated on N_max slices of its participants, participant p at
 *     bead floor(s * N_p / N_max) in slice s, each slice weighted 1/N_max;
 *   - the free ring polymers of Eq. (mts-hamiltonian-b) in normal modes and
 *     their exact propagation (Sec. "Evaluation");
 *   - the split propagator half-kick / free ring polymer / half-kick
 *     (Sec. "Evaluation", symmetric Liouvillian splitting);
 *   - energies and kinetic estimators after each step (Sec. "Output and
 *     Analysis").
 *
 * Conventions
 *   Units: Angstrom, fs, amu, kcal/mol, elementary charge, K.  Forces are
 *   kcal/mol/A; momenta amu*A/fs.
 *
 *   Bead counts must be powers of two (Sec. "Setup") and particles must be
 *   listed in non-increasing bead count (ring-polymer molecules first,
 *   Sec. "Setup").  A *group* is a maximal run of consecutive particles with
 *   equal bead count and equal electron flag.
 *
 *   State layout ("library layout"): FP64, for each group g in order a block
 *   [N_g][n_g][3] (bead-major: all particles of bead 0, then bead 1, ...),
 *   groups concatenated; for a batch, systems concatenated in order.
 *   mixpi_bead_index() gives the row of every (particle, bead).
 *
 *   Force field (readings of the paper's q-SPC/Fw water, cation-water LJ and
 *   electron pseudopotential): LJ 4 eps ((s/r)^12 - (s/r)^6), Coulomb
 *   k_e q_i q_j / r, and for electron-atom pairs only the softened Coulomb
 *   k_e pp_q q_j / sqrt(r^2 + pp_a^2).  Every cut term is shifted as
 *   V(r) - V(rc) - (r^2 - rc^2) V'(rc) / (2 rc) inside r^2 < rc^2.  Nearest
 *   image in a rectangular box.  Pairs with equal mol_id are excluded; two
 *   electrons do not interact.  Harmonic bonds k/2 (r - r0)^2 and harmonic
 *   angles k/2 (theta - theta0)^2 (vertex in the middle).  With background
 *   set, a neutralising uniform background adds -pi k_e rc_coul^2 Q^2 / (5 V)
 *   to V_Coul (Q = net charge of the non-electron particles).
 *
 *   Pointers: "device" pointers are GPU global memory on the current HIP
 *   device, allocated and owned by the caller; "host" pointers are read
 *   during the call only.  The stream argument is a hipStream_t (NULL = the
 *   legacy default stream); all work is enqueued asynchronously on it.
 *
 *   Errors: every function returns MIXPI_OK (0) or a negative MIXPI_E_*
 *   code and never aborts; mixpi_last_error() returns a message for the last
 *   failure on the calling thread.  Argument errors are detected before any
 *   work is enqueued.
 */
#ifndef MIXPI_H
#define MIXPI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MIXPI_OK = 0,
    MIXPI_E_INVALID = -1,      /* null pointer, bad size or parameter */
    MIXPI_E_NOT_POW2 = -2,     /* a bead count is not a power of two */
    MIXPI_E_ORDER = -3,        /* bead counts increase along the particle list */
    MIXPI_E_HIP = -4,          /* a HIP runtime call failed */
    MIXPI_E_NONFINITE = -5,    /* a non-finite energy appeared (checked steps) */
    MIXPI_E_UNSUPPORTED = -6   /* valid request outside the supported range */
};

/* Energy slots (kcal/mol). mixpi_forces/mixpi_energy write the first
 * MIXPI_NV; each mixpi_step log row has MIXPI_NE. */
enum {
    MIXPI_E_VMIX = 0,   /* V_mix = LJ + COUL + PP + BOND + ANGLE */
    MIXPI_E_LJ,
    MIXPI_E_COUL,
    MIXPI_E_PP,
    MIXPI_E_BOND,
    MIXPI_E_ANGLE,
    MIXPI_E_SPRING,     /* sum_i N_i m_i/(2 beta^2 hbar^2) sum_a |q_ia - q_i,a+1|^2 */
    MIXPI_E_KIN,        /* sum p^2 / (2 m_f) */
    MIXPI_E_KCV,        /* centroid virial: sum_i 3/(2 beta) - 1/2 sum (q - qbar).F */
    MIXPI_E_KPRIM,      /* primitive: sum_i 3 N_i/(2 beta) - E_spring */
    MIXPI_E_HAM,        /* conserved H = KIN + SPRING + VMIX */
    MIXPI_NE
};
#define MIXPI_NV 6
#define MIXPI_NTHETA 6   /* theta = (pp_q, pp_a, eps_00, sigma_00, k_bond0, k_angle0) */

typedef enum {
    MIXPI_FP64 = 0,        /* all pair arithmetic in FP64 */
    MIXPI_FP32_ACC64 = 1   /* FP32 electron-atom pseudopotential and FP32 1/r
                              seeds; atom-atom terms in FP64 from the seed
                              refined by one FP64 Newton step; FP64
                              separations and sums */
} mixpi_precision;

/* flags */
#define MIXPI_FLAG_CHECK_FINITE 1   /* mixpi_step syncs and reports non-finite H */
/* Tile shape of the pair sweep (at most one flag of each kind; none = the
 * library's choice from the work size).  TILE_J*: the j-tile width TJ of the
 * system's tiles (the systems of a batch may differ).  Waves per tile (equal
 * across a batch): TILE_WAVES1 one wave on a 64 x TJ tile; TILE_WAVES2 two
 * waves splitting its j-beads; TILE_I128 / TILE_I256 a 128 x TJ or 256 x TJ
 * tile, two or four waves of 64 i-beads sharing the j-beads (fewer
 * partial-force slots).  Results agree to rounding for every shape; an
 * autotuner times them and picks one per workload. */
#define MIXPI_FLAG_TILE_J16 (1 << 8)
#define MIXPI_FLAG_TILE_J32 (1 << 4)
#define MIXPI_FLAG_TILE_J64 (1 << 5)
#define MIXPI_FLAG_TILE_WAVES1 (1 << 6)
#define MIXPI_FLAG_TILE_WAVES2 (1 << 7)
#define MIXPI_FLAG_TILE_I128 (1 << 9)
#define MIXPI_FLAG_TILE_I256 (1 << 10)

typedef struct mixpi_system mixpi_system;   /* opaque, owned by the library */

/* Host description of one system; every array is host memory, copied by
 * mixpi_create.  Bead counts: non-increasing powers of two. */
typedef struct {
    int32_t n_particles;
    const int32_t *n_beads;        /* [n] */
    const double *mass;            /* [n] physical mass, amu (> 0) */
    const double *fict_mass;       /* [n] fictitious bead mass m_f, amu (> 0) */
    const double *charge;          /* [n] e */
    const int32_t *lj_type;        /* [n] in [0, n_lj_types) or -1 (no LJ) */
    const int32_t *mol_id;         /* [n] in [0, 2^27); equal ids exclude nonbonded pairs */
    const int32_t *is_electron;    /* [n] 0/1 */
    int32_t n_lj_types;            /* <= 8 */
    const double *lj_eps;          /* [n_lj_types^2] kcal/mol, symmetric */
    const double *lj_sigma;        /* [n_lj_types^2] A */
    int32_t n_bonds;
    const int32_t *bonds;          /* [n_bonds][2] particle indices */
    const int32_t *bond_type;      /* [n_bonds] */
    int32_t n_bond_types;
    const double *bond_k;          /* [n_bond_types] kcal/mol/A^2 */
    const double *bond_r0;         /* [n_bond_types] A */
    int32_t n_angles;
    const int32_t *angles;         /* [n_angles][3] (end, vertex, end) */
    const int32_t *angle_type;     /* [n_angles] */
    int32_t n_angle_types;
    const double *angle_k;         /* [n_angle_types] kcal/mol/rad^2 */
    const double *angle_t0;        /* [n_angle_types] rad */
    double pp_q;                   /* pseudopotential charge of an electron, e */
    double pp_a;                   /* softening length, A (> 0) */
    double rc_pp, rc_coul, rc_lj;  /* cutoffs, A (> 0) */
    int32_t background;            /* 0/1 */
    double box[3];                 /* rectangular periodic box, A */
    double temperature;            /* K (> 0) */
    double dt;                     /* fs */
    int32_t precision;             /* mixpi_precision */
    int32_t flags;                 /* MIXPI_FLAG_* */
} mixpi_system_desc;

/* Message of the last failure on this thread ("" if none). */
const char *mixpi_last_error(void);

/* Validates desc and builds a one-system handle on the current HIP device
 * for the mixed time-slicing ring-polymer Hamiltonian (arXiv 2411.11988,
 * Sec. Theory, MixTS Ring Polymer Hamiltonian, Eq. mts-hamiltonian): one
 * state holding every bead of every particle, with the bead pairing of each
 * interaction taken from the bead-index bookkeeping (Sec. Implementation,
 * Overview) and bead counts restricted to powers of two (Sec.
 * Implementation, Setup).  Builds the constant tables (normal-mode bases,
 * propagator coefficients) and the pair and bonded work lists.  Errors:
 * MIXPI_E_INVALID, _NOT_POW2, _ORDER, _UNSUPPORTED (more than 8 LJ types,
 * N > 4096), _HIP.  *out is NULL on failure. */
int mixpi_create(const mixpi_system_desc *desc, mixpi_system **out);

/* A batch of n independent systems sharing one handle: every entry point
 * then processes all systems in the same launches.  Arrays in the library
 * layout hold the systems back to back; per-system outputs are indexed by
 * system.  All systems must share precision and flags, except the j-tile
 * width flags (MIXPI_FLAG_TILE_J*), which may differ per system. */
int mixpi_batch_create(const mixpi_system_desc *const *descs, int32_t n,
                       mixpi_system **out);

int mixpi_destroy(mixpi_system *sys);

/* Sizes: total beads (rows of every state array), particles, groups,
 * systems.  Any pointer may be NULL. */
int mixpi_sizes(const mixpi_system *sys, int64_t *n_bead_rows, int32_t *n_particles,
                int32_t *n_groups, int32_t *n_systems);

/* Host int64 [total beads]: for particle i (batch: systems in order) and
 * bead a in particle-major order, the row of that bead in the library
 * layout. */
int mixpi_bead_index(const mixpi_system *sys, int64_t *rows_out);

/* The library layout by groups (the bead-index bookkeeping of Sec.
 * Implementation, Overview, kept as index arithmetic): a group is a maximal
 * run of particles of one system with equal bead count N and electron flag
 * (particles in descending N order, so every slice map between two groups
 * is a power-of-two shift).  Bead a of the group's particle i (0 <= i < n)
 * sits at row first_row + a n + i: bead-major, so the 64-row tiles of the
 * pair sweep hold consecutive particles of one bead.
 *   n_groups      out, required: the number of groups
 *   group_offsets out, int64 [5 * n_groups] or NULL (to ask the count
 *                 first): per group, in row order, (first row, N, n, first
 *                 particle over the handle, system)
 * Host memory; no device work. */
int mixpi_layout(const mixpi_system *sys, int64_t *group_offsets, int32_t *n_groups);

/* Bead forces F = -dV_mix/dq (Eq. mts-hamiltonian).
 *   q     device double [rows][3], library layout (positions, unwrapped)
 *   theta device double [n_systems][6] overriding (pp_q, pp_a, eps and
 *         sigma of LJ type pair (0,0), k of bond type 0, k of angle type 0),
 *         or NULL for the values given at create
 *   f     device double [rows][3], overwritten (must not alias q)
 *   e_out device double [n_systems][MIXPI_NV] or NULL
 * FP64 precision: arithmetic in FP64.  FP32_ACC64: the electron-atom
 * pseudopotential in FP32, everything else in FP64 (see mixpi_precision);
 * every force and energy term is summed in FP64. */
int mixpi_forces(mixpi_system *sys, const double *q, const double *theta,
                 double *f, double *e_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * forces and energies of mixpi_forces, computed by the same kernels in the
 * same order (equal results bit for bit), with the partial-force slots,
 * energy slots and reducer partials of the evaluation in a static device
 * array of the library instead of the handle's buffers.  The call performs
 * no allocation.  Arguments as mixpi_forces.  The array holds 16 MiB
 * (MIXPI_STATIC_SCRATCH_BYTES) on every device the library runs on, until
 * the process ends; its address on a device is looked up by mixpi_create /
 * mixpi_batch_create with that device current.  Needed: 24 bytes per
 * partial-force position of the handle plus 128 bytes per energy slot of
 * its force evaluation (about 3.6 MB for one 1024-bead electron with 512
 * waters, 7 MB for 256 waters at 32/4 beads); a larger handle gets
 * MIXPI_E_UNSUPPORTED.  Every call on a device shares that device's array
 * and overwrites it entirely before reading it: calls that overlap in time
 * on one device (different streams, host threads or handles without
 * ordering) race and give wrong results.  With mixpi_use_ewald on it
 * returns MIXPI_E_UNSUPPORTED.  Asynchronous on stream. */
#define MIXPI_STATIC_SCRATCH_BYTES (16u << 20)
int mixpi_forces_static(mixpi_system *sys, const double *q, const double *theta, double *f,
                        double *e_out, void *stream);

/* V_mix only (the external potential of Eq. mts-hamiltonian, the part the
 * split propagator of Sec. Implementation, Evaluation kicks with): the
 * energies of mixpi_forces without the forces.  e_out device double
 * [n_systems][MIXPI_NV]; other arguments as mixpi_forces. */
int mixpi_energy(mixpi_system *sys, const double *q, const double *theta,
                 double *e_out, void *stream);

/* Adjoint of E = V_mix(q; theta) (recomputes every term; no per-pair
 * storage).  grad_e: device double [n_systems] (dL/dE) or NULL for 1.
 * dq: device double [rows][3] = grad_e * dE/dq (= -grad_e F).  dtheta:
 * device double [n_systems][6] = grad_e * dE/dtheta.  Either output may be
 * NULL. */
int mixpi_energy_adjoint(mixpi_system *sys, const double *q, const double *theta,
                         const double *grad_e, double *dq, double *dtheta,
                         void *stream);

/* Ring-polymer normal-mode transform (the modes in which the free
 * ring-polymer part, Eq. free-rp-hamiltonian, is integrated exactly; Sec.
 * Implementation, Evaluation) of each particle's beads, per Cartesian
 * component, in the orthonormal real basis C (bead j, mode k) of the cyclic
 * ring: k = 0: 1/sqrt(N); 0 < k < N/2: sqrt(2/N) cos(2 pi j k / N);
 * k = N/2: (-1)^j/sqrt(N); N/2 < k < N: sqrt(2/N) sin(2 pi j k / N).
 * dir = +1: out = C^T in (bead -> mode); dir = -1: out = C in (mode -> bead).
 * in/out: device double [rows][3], library layout (mode k of a group in the
 * place of bead k); must not alias. */
int mixpi_nm_transform(mixpi_system *sys, int32_t dir, const double *in, double *out,
                       void *stream);

/* nsteps of the split propagator (Sec. "Evaluation"):
 *   p += dt/2 F;  free ring polymers evolved exactly for dt in normal modes;
 *   F = F_mix(q);  p += dt/2 F;  energies -> elog.
 * q, p, f: device double [rows][3], updated in place; on entry f must hold
 * F_mix(q) (from mixpi_forces).  elog: device double
 * [nsteps][n_systems][MIXPI_NE] or NULL.  The first call with a set of
 * pointers and nsteps captures and instantiates a HIP graph (see
 * mixpi_step_prepare); later calls with the same pointers replay it. */
int mixpi_step(mixpi_system *sys, int32_t nsteps, double *q, double *p, double *f,
               double *elog, void *stream);

/* mixpi_step of a batch (mixpi_batch_create) whose state lives in separate
 * arrays per system: q[k], p[k], f[k] are device double [rows_k][3] of
 * system k in its own layout (the rows a handle of that system alone
 * would have; mixpi_layout gives each system's groups).  q, p, f are host
 * arrays of n_systems device pointers; nsteps and elog as mixpi_step
 * (nsteps = 0 does nothing; a negative count or a null pointer is
 * MIXPI_E_INVALID, with the state untouched).  Same results
 * bit for bit as mixpi_step on the systems' rows placed back to back.
 * Where the arrays already sit back to back in one allocation (q[k] =
 * q[0] + 3 x first row of system k, likewise p and f), it is mixpi_step on
 * q[0], p[0], f[0]; otherwise the states are copied (device to device, on
 * stream) into staging arrays of the handle, stepped, and copied back. The
 * staging arrays (72 bytes per bead row) are allocated by the first such
 * call and kept until mixpi_destroy: that call is not graph-capturable. */
int mixpi_batch_step(mixpi_system *sys, int32_t nsteps, double *const *q, double *const *p,
                     double *const *f, double *elog, void *stream);

/* Path-integral Langevin thermostat (the PILE thermostat of the paper's NVT
 * runs, Sec. "Examples and Discussion"), for mixpi_step_nvt.  Each ring's
 * momenta take Ornstein-Uhlenbeck steps in its normal modes (the basis of
 * mixpi_nm_transform): pi_k <- c1 pi_k + c2 eta_k with c1 = exp(-gamma_k
 * dt/2), c2 = sqrt(1 - c1^2) sqrt(m_f k_B T); gamma_0 = 1/tau0 for the
 * centroid (0 when tau0 <= 0 or infinite), gamma_k = 2 omega_k for mode k
 * (critical damping of the free-ring mode).  tau0 in fs; the system's own
 * temperature and dt.  Builds the coefficient table (host work and one
 * device copy); may be called again to change tau0. */
int mixpi_set_thermostat(mixpi_system *sys, double tau0);

/* nsteps of the thermostatted split propagator O B A B O: a Langevin half
 * step (noise slice [k][0]), p += dt/2 F, free ring polymers for dt,
 * F = F_mix(q), p += dt/2 F, energies -> elog (after the second half kick),
 * a Langevin half step (noise slice [k][1]).  noise: device double
 * [nsteps][2][rows][3] standard normals indexed by mode (mode k of a group
 * in the place of bead k, as in mixpi_nm_transform), read only; the caller
 * draws it.  Other arguments as mixpi_step; requires mixpi_set_thermostat.
 * The first call with a set of pointers captures a HIP graph. */
int mixpi_step_nvt(mixpi_system *sys, int32_t nsteps, double *q, double *p, double *f,
                   const double *noise, double *elog, void *stream);

/* nsteps of velocity Verlet with the ring-polymer springs as forces (the
 * paper's alternative to the exact normal-mode propagation, Sec.
 * "Evaluation"): with G = F_mix + F_sp, F_sp the force of the springs of
 * Eq. (mts-hamiltonian-b),
 *   p += dt/2 G(q);  q += dt p / m_f;  F = F_mix(q);  p += dt/2 G(q);
 *   energies -> elog.
 * Arguments as mixpi_step (f must hold F_mix(q) on entry).  The time step
 * must resolve the highest ring frequency, unlike the exact propagator. */
int mixpi_step_vv(mixpi_system *sys, int32_t nsteps, double *q, double *p, double *f,
                  double *elog, void *stream);

/* Path-integral radial distribution functions (the g(r) of Sec. "Examples
 * and Discussion"): the bead average of the pair count, taken like V_mix of
 * Eq. (mts-hamiltonian) -- every unordered, non-excluded particle pair
 * (different molecule ids, not two electrons) on its N_max slices, particle
 * p at bead floor(s N_p / N_max), weight 1/N_max -- binned by
 * nearest-image distance r < r_max into nbins bins of width r_max / nbins.
 * q: device [rows][3] in the handle's layout.  hist: device FP64
 * [n_systems][nspec][nspec][nbins] from hipMalloc (coarse-grained memory),
 * ADDED to, entry [s][a][b][k] with a <= b the species of the two particles
 * (their LJ type; the null type n_lj_types for particles without one);
 * entries with a > b are left alone.  nspec >= n_lj_types + 1 of every
 * system.  The sums are exact (dyadic addends), so the result is
 * independent of scheduling.  g_ab(r) follows by dividing by the number of
 * frames, the ideal-gas pair count of the bin and the number of pairs.
 * Asynchronous on stream.  Errors: MIXPI_E_INVALID (null pointer, r_max not
 * positive and finite, nbins < 1, nspec too small), MIXPI_E_UNSUPPORTED
 * (more than 14336 bins times species pairs (a <= b)). */
int mixpi_rdf(mixpi_system *sys, const double *q, double r_max, int32_t nbins, int32_t nspec,
              double *hist, void *stream);

/* One sample of the ring-polymer molecular dynamics (RPMD) centroid
 * velocity correlation function (real-time correlation functions from NVE
 * ring-polymer trajectories, Sec. "Output and Analysis"; for the velocity, a
 * linear operator, the Kubo-transformed correlation is estimated from the
 * centroids).  p: device [rows][3] bead momenta at sample t.  The centroid
 * velocity v_i = (1/N_i) sum_j p_ij / m_f,i of every particle (handle
 * order: systems, then particles) is written to slot t mod L of ring
 * (device FP64 [L][n_particles][3], caller-owned, kept between calls);
 * then for every lag tau < min(t + 1, L),
 *   acc[s][a][tau] += sum over particles i of system s with species a of
 *                     v_i(t - tau) . v_i(t),
 * species as in mixpi_rdf; acc is device FP64 [n_systems][nspec][L].
 * Calls must come with t = 0, 1, 2, ... on the same ring and L.  After T
 * samples, acc[s][a][tau] / ((T - tau) n_a 3) is the correlation function
 * of one velocity component at lag tau sample intervals.  Asynchronous on
 * stream.  Errors: MIXPI_E_INVALID (null pointer, t < 0, L < 1 or L times
 * the number of systems above 2^30, nspec too small). */
int mixpi_vacf_sample(mixpi_system *sys, const double *p, int64_t t, int32_t L, int32_t nspec,
                      double *ring, double *acc, void *stream);

/* Long-range electrostatics between ring-polymer centroids (Sec. "Theory":
 * the example systems' electrostatics by smooth-particle-mesh Ewald, with
 * the bead-bead energies and forces replaced by those between centroids).
 * Configures the Ewald sum of the atom charges (electrons carry none) at
 * the particles' centroids for every system of the handle: splitting
 * parameter alpha (1/A), real-space cutoff r_cut (A, at most half of every
 * box edge), a grid^3 reciprocal mesh (grid 16, 32 or 64)
 * and cardinal B-splines of order 4, 6 or 8 (Essmann et al., J. Chem. Phys.
 * 103, 8577 (1995)).  Builds the influence function on the host and
 * allocates the handle's Ewald buffers (24 grid^3 bytes per system plus
 * O(particles)); a second call replaces the first and keeps the
 * mixpi_use_ewald setting.  A rejected parameter changes nothing; a failed
 * allocation leaves the Ewald terms off and unconfigured.
 * Synchronous.  Errors:
 * MIXPI_E_INVALID (bad parameter), MIXPI_E_HIP. */
int mixpi_set_ewald(mixpi_system *sys, double alpha, double r_cut, int32_t grid, int32_t order);

/* The centroid Ewald electrostatics configured by mixpi_set_ewald, for the
 * bead positions q (device [rows][3]).  Energies, kcal/mol, to e_out
 * (device FP64 [n_systems][3]): [0] real space -- k_e z_i z_j
 * erfc(alpha r)/r over pairs of different molecules within r_cut, minus
 * k_e z_i z_j erf(alpha r)/r over pairs of one molecule (excluded pairs,
 * any distance); [1] reciprocal space (SPME); [2] the self term
 * -k_e alpha/sqrt(pi) sum z_i^2 and the neutralising background
 * -k_e pi Q^2/(2 V alpha^2); all with nearest-image centroid separations.
 * Forces: each bead of particle i gets F_i / N_i (the gradient with respect
 * to one of its beads), ADDED to f (device [rows][3]; null: energies
 * only).  Use with rc_coul = 0 in the system description, which turns the
 * bead-resolved cut atom-atom Coulomb term off.  The charge grid is summed
 * in fixed point (2^-50 e resolution or finer), so results are
 * independent of scheduling.  Asynchronous on stream; calls on one handle
 * must not overlap (they share its buffers).  Errors: MIXPI_E_INVALID (not
 * configured, null q or e_out). */
int mixpi_ewald(mixpi_system *sys, const double *q, double *f, double *e_out, void *stream);

/* Switches the centroid Ewald electrostatics configured by mixpi_set_ewald
 * into (on != 0) or out of (on = 0) the handle's force passes: with it on,
 * mixpi_forces, mixpi_energy, mixpi_step, mixpi_step_nvt and mixpi_step_vv
 * add the Ewald bead forces to F and the Ewald energy (real + reciprocal +
 * constant) to V_Coul and V_mix of their energies and logs, so the
 * dynamics run on V_mix + V_Ewald(centroids) (Sec. "Theory").  Use it with
 * rc_coul = 0, or the atom-atom electrostatics count twice.  While on,
 * mixpi_energy_adjoint and mixpi_kernel_time return MIXPI_E_UNSUPPORTED.
 * Forces of mixpi_forces equal the pair forces plus those of mixpi_ewald,
 * bit for bit, and the steps use the same sum.  Drops the handle's captured
 * step graphs when the setting changes (so does mixpi_set_ewald).
 * Synchronous.  Errors: MIXPI_E_INVALID (on without mixpi_set_ewald). */
int mixpi_use_ewald(mixpi_system *sys, int32_t on);

/* Candidate slice-pairs of one force evaluation: every unordered,
 * non-excluded particle pair times N_max of the pair, summed over systems
 * (from the work lists; no device work). */
int mixpi_pair_candidates(const mixpi_system *sys, int64_t *candidates);

/* Tile shape the handle's pair sweep runs with (the MIXPI_FLAG_TILE_* flags
 * or the library's choice): tj (host int32 [n_systems], or NULL) the j-tile
 * width of each system; waves the j-split waves per tile (1 or 2); i_waves
 * the i-split waves (1, 2 or 4: tiles of 64 i_waves i-beads); j_run the
 * most j-tiles one tile sweeps in turn (its i-forces stored once).  Any
 * pointer may be NULL.  No device work. */
int mixpi_pair_shape(const mixpi_system *sys, int32_t *tj, int32_t *waves, int32_t *i_waves,
                     int32_t *j_run);

/* Slice-pair evaluations with at least one term inside its cutoff, counted
 * on the device by every force evaluation since the last reset (forces,
 * energy, adjoint and each step).  evals: host int64 [2] = (atom-atom
 * pairs, electron-atom pairs).  Waits for the stream.  reset != 0 zeroes
 * the counters after reading. */
int mixpi_pair_evals(mixpi_system *sys, int64_t *evals, int32_t reset, void *stream);

/* Builds and caches the HIP graph that mixpi_step would use for these
 * arguments, without launching it (moves graph construction out of a
 * latency-critical or timed region).  Same argument rules as mixpi_step. */
int mixpi_step_prepare(mixpi_system *sys, int32_t nsteps, double *q, double *p, double *f,
                       double *elog);

/* Measurement aid: runs `reps` steps (1..1000) eagerly on library copies of
 * q, p, f (the caller's buffers are not changed) with a HIP event before and
 * after each of a step's three launches, and returns their mean durations in
 * microseconds: avg_us[0] = force launch (pair sweep + bonded workgroups),
 * avg_us[1] = free ring-polymer launch (normal modes + the energy reducer of
 * the previous step), avg_us[2] = half-kick/energy epilogue.  The events
 * are timing-only (no system-scope fence), and the steps are enqueued in
 * chunks of 16 behind a bounded delay kernel (2 ms) that holds the stream
 * meanwhile, so each chunk's launches run back to back with the same inputs
 * and cache state as in mixpi_step.
 * q, p, f: device double [rows][3]; avg_us: host double[3].  Waits for the
 * stream. */
int mixpi_kernel_time(mixpi_system *sys, int32_t reps, const double *q, const double *p,
                      const double *f, double *avg_us, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MIXPI_H */
