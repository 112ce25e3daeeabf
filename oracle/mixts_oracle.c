/*
 * mixts_oracle.c -- plain FP64 CPU oracle for mixed-time-slicing PIMD.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never does.  It shares no code, header, table or constant
 * with the GPU library.
 *
 * What it computes (arXiv 2411.11988, Sec. "Theory" and "Evaluation"):
 *   - V_mix of Eq. (mts-hamiltonian): every 1-, 2-, 3-body term is evaluated
 *     on N_max(term) slices; at slice s participant p sits at bead
 *     floor(s * N_p / N_max) (the paper's nested indices written as one
 *     floor map, the worked example being N_1 = 4, N_2 = 2: beads 1,2 of
 *     particle 1 meet bead 1 of particle 2, beads 3,4 meet bead 2), each
 *     slice weighted 1/N_max.  [orc_forces_o2]
 *   - The same V_mix as an average over N_G = max_p N_p global slices of a
 *     classical evaluation (each term then repeats N_G/N_max times with
 *     weight 1/N_G); used only as an independent brute-force check.
 *     [orc_forces_o1]
 *   - The free ring-polymer springs of Eq. (mts-hamiltonian-b), spring
 *     constant N_i m_i / (beta hbar)^2, cyclic q_{N+1} = q_1.  [orc_springs]
 *   - Normal modes of each free ring polymer and their exact propagation,
 *     and the split propagator half-kick / free ring polymer / half-kick
 *     (Sec. "Evaluation", the symmetric Liouvillian splitting).  [orc_step]
 *   - Energies and kinetic estimators written after each step (Sec. "Output
 *     and Analysis").  [orc_observables]
 *   - The path-integral Langevin thermostat the paper's NVT runs use (Sec.
 *     "Examples and Discussion", PILE): an Ornstein-Uhlenbeck step of the
 *     momenta in each ring's normal modes, friction 1/tau0 on the centroid
 *     and 2 omega_k on mode k; noise is an input.  [orc_pile, orc_step_nvt]
 *   - The alternative velocity-Verlet integration with the springs as
 *     forces (Sec. "Evaluation").  [orc_step_vv]
 *   - The radial distribution functions the paper reports (Sec. "Examples
 *     and Discussion"), as bead-averaged slice-pair histograms.  [orc_rdf]
 *   - Long-range electrostatics on the ring-polymer centroids (Sec.
 *     "Theory"): the Ewald sum by its definition.  [orc_ewald]
 *
 * Force field (the paper names q-SPC/Fw water, a cation-water LJ and an
 * electron pseudopotential; the functional forms below are the readings this
 * project uses): Lennard-Jones, Coulomb and a softened Coulomb
 * k_e q_e q_j / sqrt(r^2 + a^2), each shifted at its cutoff as
 * V_c(r) = V(r) - V(rc) - (r^2 - rc^2) V'(rc) / (2 rc) for r^2 < rc^2
 * (continuous energy and force at rc, smooth at r = 0); harmonic bonds
 * and harmonic angles; nearest-image distances; intramolecular nonbonded
 * pairs (equal mol id) excluded; electrons interact only with atoms, only
 * through the pseudopotential.  A uniform neutralising background adds the
 * constant -pi k_e rc^2 Q^2 / (5 V) for the net atomic charge Q (the
 * integral of the shifted Coulomb kernel over the cutoff sphere is
 * 2 pi rc^2 / 5; charge-background plus background-background terms).
 *
 * Units: Angstrom, fs, amu, kcal/mol, e.  Forces in kcal/mol/A.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------- constants (SI / CODATA 2022; oracle's own copy) -------- */
#define O_AMU_KG   1.66053906892e-27
#define O_H_SI     6.62607015e-34
#define O_KB_SI    1.380649e-23
#define O_NA       6.02214076e23
#define O_KE_KCAL  332.0637133          /* e^2/(4 pi eps0) in kcal A / mol */
#define O_PI       3.14159265358979323846
#define O_HBAR_SI  (O_H_SI / (2.0 * O_PI))

static double o_amu_a2_fs2_J(void) { return O_AMU_KG * 1e-20 / 1e-30; }
/* kcal/mol expressed in amu A^2 / fs^2 */
static double o_kcal(void) { return 4184.0 / O_NA / o_amu_a2_fs2_J(); }
static double o_hbar(void) { return O_HBAR_SI / (O_AMU_KG * 1e-20 / 1e-15); }
static double o_kb(void) { return O_KB_SI / o_amu_a2_fs2_J(); }
/* k_B in kcal/mol/K */
static double o_kb_kcal(void) { return O_KB_SI * O_NA / 4184.0; }

/* Energy slots of the oracle's output arrays. */
enum { E_VMIX = 0, E_LJ, E_COUL, E_PP, E_BOND, E_ANGLE,
       E_SPRING, E_KIN, E_KCV, E_KPRIM, E_HAM, E_N };

typedef struct {
    int n;                    /* particles */
    const int *nb;            /* beads per particle */
    const long *off;          /* bead offsets [n+1] into the bead table */
    const double *mass;       /* physical mass (amu) */
    const double *fm;         /* fictitious bead mass (amu) */
    const double *charge;     /* e */
    const int *ljt, *mol, *ele;
    int nt;                   /* LJ types */
    const double *eps, *sig;  /* [nt*nt] */
    int nbond; const int *bond; const int *btype; const double *bk, *br0;
    int nangle; const int *angle; const int *atype; const double *ak, *at0;
    double pp_q, pp_a, rc_pp, rc_coul, rc_lj;
    int background;
    double box[3];
    double temperature, dt;
} orc_sys;

/* ---------------- slice map ---------------------------------------------- */

/* Bead of a participant with Np beads at slice s of a term with Nmax slices. */
int orc_slice_bead(int s, int np, int nmax)
{
    return (int)(((long)s * (long)np) / (long)nmax);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ---------------- classical pieces --------------------------------------- */

static void min_image(const orc_sys *S, const double *a, const double *b, double d[3])
{
    for (int k = 0; k < 3; ++k) {
        double x = a[k] - b[k];
        d[k] = x - S->box[k] * nearbyint(x / S->box[k]);
    }
}

/* One nonbonded pair at separation d = x_i - x_j.  Adds the energies
 * (times w) to e[] and returns g with F_i = g d, F_j = -g d (already times w).
 * Every cut term uses V_c(r) = V(r) - V(rc) - (r^2 - rc^2) V'(rc) / (2 rc)
 * for r^2 < rc^2 (else 0), so V_c(rc) = 0 and dV_c/dr(rc) = 0, and V_c is as
 * smooth at r = 0 as V itself.  With c1 = V'(rc)/rc the force scalar is
 * g = -V'(r)/r + c1.  Returns 0 when the pair does not interact. */
static int pair_term(const orc_sys *S, int i, int j, const double d[3], double w,
                     double e[E_N], double *gout)
{
    if (S->mol[i] == S->mol[j]) return 0;
    int ei = S->ele[i], ej = S->ele[j];
    if (ei && ej) return 0;
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double g = 0.0;
    int hit = 0;
    if (ei || ej) {
        /* electron - atom pseudopotential V = K / sqrt(r^2 + a^2) */
        double rc = S->rc_pp;
        if (r2 < rc * rc) {
            int atom = ei ? j : i;
            double K = O_KE_KCAL * S->pp_q * S->charge[atom];
            double a2 = S->pp_a * S->pp_a;
            double v_r = K / sqrt(r2 + a2);
            double v_c = K / sqrt(rc * rc + a2);
            double dvr_over_r = -K / pow(r2 + a2, 1.5);       /* V'(r)/r */
            double c1 = -K / pow(rc * rc + a2, 1.5);          /* V'(rc)/rc */
            e[E_PP] += w * (v_r - v_c - 0.5 * (r2 - rc * rc) * c1);
            g += w * (-dvr_over_r + c1);
            hit = 1;
        }
    } else {
        int ti = S->ljt[i], tj = S->ljt[j];
        double eps = (ti >= 0 && tj >= 0 && ti < S->nt && tj < S->nt)
                         ? S->eps[ti * S->nt + tj] : 0.0;
        double rc = S->rc_lj;
        if (eps != 0.0 && r2 < rc * rc) {
            double sg = S->sig[ti * S->nt + tj];
            double sr6 = pow(sg * sg / r2, 3), sr12 = sr6 * sr6;
            double sc6 = pow(sg / rc, 6), sc12 = sc6 * sc6;
            double v_r = 4.0 * eps * (sr12 - sr6);
            double v_c = 4.0 * eps * (sc12 - sc6);
            double dvr_over_r = 4.0 * eps * (-12.0 * sr12 + 6.0 * sr6) / r2;
            double c1 = 4.0 * eps * (-12.0 * sc12 + 6.0 * sc6) / (rc * rc);
            e[E_LJ] += w * (v_r - v_c - 0.5 * (r2 - rc * rc) * c1);
            g += w * (-dvr_over_r + c1);
            hit = 1;
        }
        double qq = S->charge[i] * S->charge[j];
        rc = S->rc_coul;
        if (qq != 0.0 && r2 < rc * rc) {
            double K = O_KE_KCAL * qq;
            double r = sqrt(r2);
            double v_r = K / r, v_c = K / rc;
            double dvr_over_r = -K / (r2 * r);
            double c1 = -K / (rc * rc * rc);
            e[E_COUL] += w * (v_r - v_c - 0.5 * (r2 - rc * rc) * c1);
            g += w * (-dvr_over_r + c1);
            hit = 1;
        }
    }
    *gout = g;
    return hit;
}

/* Harmonic bond between positions xa, xb. Adds w*V, returns forces on a, b. */
static void bond_term(const orc_sys *S, int b, const double *xa, const double *xb,
                      double w, double e[E_N], double fa[3], double fb[3])
{
    int t = S->btype[b];
    double d[3];
    min_image(S, xa, xb, d);
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double dr = r - S->br0[t];
    e[E_BOND] += w * 0.5 * S->bk[t] * dr * dr;
    double g = -w * S->bk[t] * dr / r;
    for (int k = 0; k < 3; ++k) { fa[k] = g * d[k]; fb[k] = -g * d[k]; }
}

/* Harmonic angle a-v-b (vertex v).  Adds w*V, returns forces on a, v, b. */
static void angle_term(const orc_sys *S, int an, const double *xa, const double *xv,
                       const double *xb, double w, double e[E_N],
                       double fa[3], double fv[3], double fb[3])
{
    int t = S->atype[an];
    double r1[3], r2[3];
    min_image(S, xa, xv, r1);
    min_image(S, xb, xv, r2);
    double l1 = sqrt(r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
    double l2 = sqrt(r2[0] * r2[0] + r2[1] * r2[1] + r2[2] * r2[2]);
    double c = (r1[0] * r2[0] + r1[1] * r2[1] + r1[2] * r2[2]) / (l1 * l2);
    if (c > 1.0) c = 1.0;
    if (c < -1.0) c = -1.0;
    double th = acos(c);
    double dth = th - S->at0[t];
    e[E_ANGLE] += w * 0.5 * S->ak[t] * dth * dth;
    double s = sqrt(1.0 - c * c);
    double pref = w * S->ak[t] * dth / s;   /* (dV/dtheta) / sin(theta) */
    for (int k = 0; k < 3; ++k) {
        double dc1 = r2[k] / (l1 * l2) - c * r1[k] / (l1 * l1);
        double dc2 = r1[k] / (l1 * l2) - c * r2[k] / (l2 * l2);
        fa[k] = pref * dc1;
        fb[k] = pref * dc2;
        fv[k] = -(fa[k] + fb[k]);
    }
}

static double background_energy(const orc_sys *S)
{
    if (!S->background) return 0.0;
    double Q = 0.0;
    for (int i = 0; i < S->n; ++i)
        if (!S->ele[i]) Q += S->charge[i];
    double V = S->box[0] * S->box[1] * S->box[2];
    return -O_PI * O_KE_KCAL * S->rc_coul * S->rc_coul * Q * Q / (5.0 * V);
}

static void finish_potential(const orc_sys *S, double e[E_N])
{
    e[E_COUL] += background_energy(S);
    e[E_VMIX] = e[E_LJ] + e[E_COUL] + e[E_PP] + e[E_BOND] + e[E_ANGLE];
}

/* ---------------- V_mix, term by term on N_max slices (O2) --------------- */

/* F: bead table [B][3] (overwritten).  e: first 6 slots written. */
void orc_forces_o2(const orc_sys *S, const double *q, double *F, double *eout)
{
    long B = S->off[S->n];
    memset(F, 0, sizeof(double) * 3 * B);
    double e[E_N] = {0};
    int nth = orc_num_threads();
    double *Fth = (double *)calloc((size_t)nth * 3 * B, sizeof(double));
    double *eth = (double *)calloc((size_t)nth * E_N, sizeof(double));

    /* nonbonded pairs; particles are dealt to the threads round-robin, so for
       a given thread count every sum has a fixed order (a dynamic schedule
       would make the rounding, and chaotic trajectories, vary run to run) */
#pragma omp parallel for schedule(static, 1)
    for (int i = 0; i < S->n; ++i) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *Ft = Fth + (size_t)tid * 3 * B;
        double *et = eth + (size_t)tid * E_N;
        for (int j = i + 1; j < S->n; ++j) {
            int ni = S->nb[i], nj = S->nb[j];
            int nmax = ni > nj ? ni : nj;
            double w = 1.0 / nmax;
            for (int s = 0; s < nmax; ++s) {
                long bi = S->off[i] + orc_slice_bead(s, ni, nmax);
                long bj = S->off[j] + orc_slice_bead(s, nj, nmax);
                double d[3], g;
                min_image(S, q + 3 * bi, q + 3 * bj, d);
                if (pair_term(S, i, j, d, w, et, &g)) {
                    for (int k = 0; k < 3; ++k) {
                        Ft[3 * bi + k] += g * d[k];
                        Ft[3 * bj + k] -= g * d[k];
                    }
                }
            }
        }
    }
    for (int t = 0; t < nth; ++t) {
        for (long x = 0; x < 3 * B; ++x) F[x] += Fth[(size_t)t * 3 * B + x];
        for (int k = 0; k < E_N; ++k) e[k] += eth[(size_t)t * E_N + k];
    }
    free(Fth);
    free(eth);

    /* bonds */
    for (int b = 0; b < S->nbond; ++b) {
        int i = S->bond[2 * b], j = S->bond[2 * b + 1];
        int ni = S->nb[i], nj = S->nb[j];
        int nmax = ni > nj ? ni : nj;
        for (int s = 0; s < nmax; ++s) {
            long bi = S->off[i] + orc_slice_bead(s, ni, nmax);
            long bj = S->off[j] + orc_slice_bead(s, nj, nmax);
            double fa[3], fb[3];
            bond_term(S, b, q + 3 * bi, q + 3 * bj, 1.0 / nmax, e, fa, fb);
            for (int k = 0; k < 3; ++k) { F[3 * bi + k] += fa[k]; F[3 * bj + k] += fb[k]; }
        }
    }
    /* angles */
    for (int a = 0; a < S->nangle; ++a) {
        int i = S->angle[3 * a], v = S->angle[3 * a + 1], j = S->angle[3 * a + 2];
        int ni = S->nb[i], nv = S->nb[v], nj = S->nb[j];
        int nmax = ni > nv ? ni : nv;
        if (nj > nmax) nmax = nj;
        for (int s = 0; s < nmax; ++s) {
            long bi = S->off[i] + orc_slice_bead(s, ni, nmax);
            long bv = S->off[v] + orc_slice_bead(s, nv, nmax);
            long bj = S->off[j] + orc_slice_bead(s, nj, nmax);
            double fa[3], fv[3], fb[3];
            angle_term(S, a, q + 3 * bi, q + 3 * bv, q + 3 * bj, 1.0 / nmax, e, fa, fv, fb);
            for (int k = 0; k < 3; ++k) {
                F[3 * bi + k] += fa[k]; F[3 * bv + k] += fv[k]; F[3 * bj + k] += fb[k];
            }
        }
    }
    finish_potential(S, e);
    for (int k = 0; k <= E_ANGLE; ++k) eout[k] = e[k];
}

/* Centroid of particle i: the mean of its bead positions. */
static void centroid(const orc_sys *S, const double *q, int i, double c[3])
{
    c[0] = c[1] = c[2] = 0.0;
    for (int j = 0; j < S->nb[i]; ++j)
        for (int k = 0; k < 3; ++k) c[k] += q[3 * (S->off[i] + j) + k];
    for (int k = 0; k < 3; ++k) c[k] /= S->nb[i];
}

/* Long-range electrostatics of the atoms in the centroid approximation
 * (Sec. "Theory", the smooth-particle-mesh Ewald treatment of the example
 * systems: the bead-bead electrostatic energies and forces are replaced by
 * those between the ring-polymer centroids).  The Ewald sum of the atom
 * charges z_i at the centroids c_i (electrons carry no Ewald charge; pairs
 * of one molecule are excluded; conducting boundary), with k_e the
 * Coulomb constant, V the cell volume and Q = sum_i z_i:
 *   real   sum over non-excluded pairs with r < rc of k_e z_i z_j erfc(alpha r)/r,
 *          minus the excluded pairs' k_e z_i z_j erf(alpha r)/r (any r),
 *   recip  (2 pi k_e / V) sum over k = 2 pi (n1/L1, n2/L2, n3/L3), 0 < |n_a| <= kmax
 *          per component, of exp(-k^2 / (4 alpha^2)) / k^2 |sum_j z_j exp(i k.c_j)|^2,
 *   const  -k_e alpha / sqrt(pi) sum_i z_i^2 - k_e pi Q^2 / (2 V alpha^2),
 * all with nearest-image separations.  e[0..2] = real, recip, const; the
 * reciprocal sum is skipped (e[1] = 0) for kmax < 0.  Each bead j of
 * particle i receives F_i / N_i (the gradient of a function of the centroid
 * with respect to one of its N_i beads); forces are added to F. */
void orc_ewald(const orc_sys *S, const double *q, double alpha, double rc, int kmax, double *F,
               double e[3])
{
    const int n = S->n;
    double *c = (double *)malloc(sizeof(double) * 3 * (n > 0 ? n : 1));
    double *fc = (double *)calloc(3 * (n > 0 ? n : 1), sizeof(double));
    double *z = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int i = 0; i < n; ++i) {
        centroid(S, q, i, c + 3 * i);
        z[i] = S->ele[i] ? 0.0 : S->charge[i];
    }
    const double V = S->box[0] * S->box[1] * S->box[2];
    double er = 0.0, ek = 0.0, e0 = 0.0, Q = 0.0, z2 = 0.0;
    for (int i = 0; i < n; ++i) {
        Q += z[i];
        z2 += z[i] * z[i];
    }
    /* real space and exclusions */
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double zz = z[i] * z[j];
            if (zz == 0.0) continue;
            double d[3];
            min_image(S, c + 3 * i, c + 3 * j, d);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double r = sqrt(r2);
            double gauss = 2.0 * alpha / sqrt(O_PI) * exp(-alpha * alpha * r2);
            double g;   /* F_i = g d */
            if (S->mol[i] == S->mol[j]) {
                /* -erf(alpha r)/r; d/dr = -(gauss r - erf) / r^2 */
                double v = erf(alpha * r) / r;
                er -= O_KE_KCAL * zz * v;
                double dv = (gauss * r - erf(alpha * r)) / r2;   /* d/dr of erf(ar)/r */
                g = O_KE_KCAL * zz * dv / r;                  /* -d(-v)/dr / r */
            } else if (r < rc) {
                double v = erfc(alpha * r) / r;
                er += O_KE_KCAL * zz * v;
                double dv = -(gauss * r + erfc(alpha * r)) / r2;  /* d/dr of erfc(ar)/r */
                g = -O_KE_KCAL * zz * dv / r;
            } else {
                continue;
            }
            for (int k = 0; k < 3; ++k) {
                fc[3 * i + k] += g * d[k];
                fc[3 * j + k] -= g * d[k];
            }
        }
    /* reciprocal space by the direct sum over wave vectors */
    if (kmax >= 0) {
        for (int n1 = -kmax; n1 <= kmax; ++n1)
            for (int n2 = -kmax; n2 <= kmax; ++n2)
                for (int n3 = -kmax; n3 <= kmax; ++n3) {
                    if (n1 == 0 && n2 == 0 && n3 == 0) continue;
                    double kv[3] = {2.0 * O_PI * n1 / S->box[0], 2.0 * O_PI * n2 / S->box[1],
                                    2.0 * O_PI * n3 / S->box[2]};
                    double k2 = kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2];
                    double A = 2.0 * O_PI * O_KE_KCAL / V * exp(-k2 / (4.0 * alpha * alpha)) / k2;
                    double sr = 0.0, si = 0.0;
                    for (int j = 0; j < n; ++j) {
                        double ph = kv[0] * c[3 * j] + kv[1] * c[3 * j + 1] + kv[2] * c[3 * j + 2];
                        sr += z[j] * cos(ph);
                        si += z[j] * sin(ph);
                    }
                    ek += A * (sr * sr + si * si);
                    /* F_j = 2 A z_j k Im(exp(i k.c_j) conj(S)) */
                    for (int j = 0; j < n; ++j) {
                        if (z[j] == 0.0) continue;
                        double ph = kv[0] * c[3 * j] + kv[1] * c[3 * j + 1] + kv[2] * c[3 * j + 2];
                        double im = sin(ph) * sr - cos(ph) * si;
                        for (int k = 0; k < 3; ++k) fc[3 * j + k] += 2.0 * A * z[j] * kv[k] * im;
                    }
                }
    }
    e0 = -O_KE_KCAL * alpha / sqrt(O_PI) * z2 - O_KE_KCAL * O_PI * Q * Q / (2.0 * V * alpha * alpha);
    e[0] = er;
    e[1] = ek;
    e[2] = e0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < S->nb[i]; ++j)
            for (int k = 0; k < 3; ++k) F[3 * (S->off[i] + j) + k] += fc[3 * i + k] / S->nb[i];
    free(c);
    free(fc);
    free(z);
}

/* Path-integral radial distribution: every non-excluded particle pair of
 * V_mix (different molecules, not two electrons) on its N_max slices with
 * weight 1/N_max (the bead average of Eq. (mts-hamiltonian) applied to a
 * pair count), binned by nearest-image distance, r < rmax, nbins bins of
 * rmax/nbins.  hist[a][b][bin] with a <= b the species (LJ type; the null
 * type nt for particles without one), nspec species per axis; added to. */
void orc_rdf(const orc_sys *S, const double *q, double rmax, int nbins, int nspec, double *hist)
{
    double dr = rmax / nbins;
    for (int i = 0; i < S->n; ++i)
        for (int j = i + 1; j < S->n; ++j) {
            if (S->mol[i] == S->mol[j]) continue;
            if (S->ele[i] && S->ele[j]) continue;
            int ti = S->ljt[i] < 0 ? S->nt : S->ljt[i];
            int tj = S->ljt[j] < 0 ? S->nt : S->ljt[j];
            int a = ti < tj ? ti : tj, b = ti < tj ? tj : ti;
            int ni = S->nb[i], nj = S->nb[j];
            int nmax = ni > nj ? ni : nj;
            for (int s = 0; s < nmax; ++s) {
                long bi = S->off[i] + orc_slice_bead(s, ni, nmax);
                long bj = S->off[j] + orc_slice_bead(s, nj, nmax);
                double d[3];
                min_image(S, q + 3 * bi, q + 3 * bj, d);
                double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                if (r >= rmax) continue;
                int bin = (int)(r / dr);
                if (bin >= nbins) bin = nbins - 1;
                hist[((long)a * nspec + b) * nbins + bin] += 1.0 / nmax;
            }
        }
}

/* Counts the slice-pairs of orc_forces_o2 with at least one term inside its
 * cutoff: out[0] atom-atom, out[1] electron-atom. */
void orc_pair_evals(const orc_sys *S, const double *q, long *out)
{
    long na = 0, ne = 0;
    double e[E_N];
    for (int i = 0; i < S->n; ++i)
        for (int j = i + 1; j < S->n; ++j) {
            int ni = S->nb[i], nj = S->nb[j];
            int nmax = ni > nj ? ni : nj;
            for (int s = 0; s < nmax; ++s) {
                long bi = S->off[i] + orc_slice_bead(s, ni, nmax);
                long bj = S->off[j] + orc_slice_bead(s, nj, nmax);
                double d[3], g;
                min_image(S, q + 3 * bi, q + 3 * bj, d);
                if (pair_term(S, i, j, d, 1.0, e, &g)) {
                    if (S->ele[i] || S->ele[j]) ++ne;
                    else ++na;
                }
            }
        }
    out[0] = na;
    out[1] = ne;
}

/* ---------------- V_mix as an average over global slices (O1) ------------ */

/* Classical potential and forces of one configuration X[n][3]. */
static void classical(const orc_sys *S, const double *X, double *Fc, double e[E_N])
{
    memset(Fc, 0, sizeof(double) * 3 * S->n);
    for (int i = 0; i < S->n; ++i)
        for (int j = i + 1; j < S->n; ++j) {
            double d[3], g;
            min_image(S, X + 3 * i, X + 3 * j, d);
            if (pair_term(S, i, j, d, 1.0, e, &g))
                for (int k = 0; k < 3; ++k) { Fc[3 * i + k] += g * d[k]; Fc[3 * j + k] -= g * d[k]; }
        }
    for (int b = 0; b < S->nbond; ++b) {
        int i = S->bond[2 * b], j = S->bond[2 * b + 1];
        double fa[3], fb[3];
        bond_term(S, b, X + 3 * i, X + 3 * j, 1.0, e, fa, fb);
        for (int k = 0; k < 3; ++k) { Fc[3 * i + k] += fa[k]; Fc[3 * j + k] += fb[k]; }
    }
    for (int a = 0; a < S->nangle; ++a) {
        int i = S->angle[3 * a], v = S->angle[3 * a + 1], j = S->angle[3 * a + 2];
        double fa[3], fv[3], fb[3];
        angle_term(S, a, X + 3 * i, X + 3 * v, X + 3 * j, 1.0, e, fa, fv, fb);
        for (int k = 0; k < 3; ++k) { Fc[3 * i + k] += fa[k]; Fc[3 * v + k] += fv[k]; Fc[3 * j + k] += fb[k]; }
    }
}

void orc_forces_o1(const orc_sys *S, const double *q, double *F, double *eout)
{
    long B = S->off[S->n];
    memset(F, 0, sizeof(double) * 3 * B);
    int ng = 1;
    for (int i = 0; i < S->n; ++i) if (S->nb[i] > ng) ng = S->nb[i];
    double *X = (double *)malloc(sizeof(double) * 3 * S->n);
    double *Fc = (double *)malloc(sizeof(double) * 3 * S->n);
    double e[E_N] = {0};
    for (int s = 0; s < ng; ++s) {
        double es[E_N] = {0};
        for (int i = 0; i < S->n; ++i) {
            long b = S->off[i] + orc_slice_bead(s, S->nb[i], ng);
            for (int k = 0; k < 3; ++k) X[3 * i + k] = q[3 * b + k];
        }
        classical(S, X, Fc, es);
        for (int k = 0; k < E_N; ++k) e[k] += es[k] / ng;
        for (int i = 0; i < S->n; ++i) {
            long b = S->off[i] + orc_slice_bead(s, S->nb[i], ng);
            for (int k = 0; k < 3; ++k) F[3 * b + k] += Fc[3 * i + k] / ng;
        }
    }
    free(X);
    free(Fc);
    finish_potential(S, e);
    for (int k = 0; k <= E_ANGLE; ++k) eout[k] = e[k];
}

/* Classical energy/forces of one configuration X[n][3] (exported for tests). */
void orc_classical(const orc_sys *S, const double *X, double *Fc, double *eout)
{
    double e[E_N] = {0};
    classical(S, X, Fc, e);
    finish_potential(S, e);
    for (int k = 0; k <= E_ANGLE; ++k) eout[k] = e[k];
}

/* ---------------- derivative of V_mix with respect to parameters --------- */
/* theta = (pseudopotential charge q_e, softening a, eps of LJ type pair (0,0),
 * sigma of LJ type pair (0,0), k of bond type 0, k of angle type 0).
 * Term-by-term analytic derivatives of the shifted-force forms. */
void orc_dvdtheta(const orc_sys *S, const double *q, double *g6)
{
    double g[6] = {0};
    for (int i = 0; i < S->n; ++i)
        for (int j = i + 1; j < S->n; ++j) {
            if (S->mol[i] == S->mol[j]) continue;
            int ei = S->ele[i], ej = S->ele[j];
            if (ei && ej) continue;
            int ni = S->nb[i], nj = S->nb[j];
            int nmax = ni > nj ? ni : nj;
            double w = 1.0 / nmax;
            for (int s = 0; s < nmax; ++s) {
                long bi = S->off[i] + orc_slice_bead(s, ni, nmax);
                long bj = S->off[j] + orc_slice_bead(s, nj, nmax);
                double d[3];
                min_image(S, q + 3 * bi, q + 3 * bj, d);
                double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (ei || ej) {
                    double rc = S->rc_pp;
                    if (!(r2 < rc * rc)) continue;
                    int atom = ei ? j : i;
                    double a = S->pp_a, a2 = a * a;
                    double Kq = O_KE_KCAL * S->charge[atom];      /* K / q_e */
                    double phi_r = 1.0 / sqrt(r2 + a2), phi_c = 1.0 / sqrt(rc * rc + a2);
                    double psi_c = -1.0 / pow(rc * rc + a2, 1.5);  /* c1 / K */
                    g[0] += w * Kq * (phi_r - phi_c - 0.5 * (r2 - rc * rc) * psi_c);
                    double K = Kq * S->pp_q;
                    double da_phi_r = -a / pow(r2 + a2, 1.5);
                    double da_phi_c = -a / pow(rc * rc + a2, 1.5);
                    double da_psi_c = 3.0 * a / pow(rc * rc + a2, 2.5);
                    g[1] += w * K * (da_phi_r - da_phi_c - 0.5 * (r2 - rc * rc) * da_psi_c);
                } else {
                    if (!(S->ljt[i] == 0 && S->ljt[j] == 0)) continue;
                    double eps = S->eps[0], sg = S->sig[0], rc = S->rc_lj;
                    if (eps == 0.0 || !(r2 < rc * rc)) continue;
                    double sr6 = pow(sg * sg / r2, 3), sr12 = sr6 * sr6;
                    double sc6 = pow(sg / rc, 6), sc12 = sc6 * sc6;
                    double u_r = 4.0 * (sr12 - sr6), u_c = 4.0 * (sc12 - sc6);
                    double c1u = 4.0 * (-12.0 * sc12 + 6.0 * sc6) / (rc * rc);
                    g[2] += w * (u_r - u_c - 0.5 * (r2 - rc * rc) * c1u);
                    double ds_r = 4.0 * eps * (12.0 * sr12 - 6.0 * sr6) / sg;
                    double ds_c = 4.0 * eps * (12.0 * sc12 - 6.0 * sc6) / sg;
                    double ds_c1 = 4.0 * eps * (-144.0 * sc12 + 36.0 * sc6) / (sg * rc * rc);
                    g[3] += w * (ds_r - ds_c - 0.5 * (r2 - rc * rc) * ds_c1);
                }
            }
        }
    for (int b = 0; b < S->nbond; ++b) {
        if (S->btype[b] != 0) continue;
        int i = S->bond[2 * b], j = S->bond[2 * b + 1];
        int ni = S->nb[i], nj = S->nb[j];
        int nmax = ni > nj ? ni : nj;
        for (int s = 0; s < nmax; ++s) {
            long bi = S->off[i] + orc_slice_bead(s, ni, nmax);
            long bj = S->off[j] + orc_slice_bead(s, nj, nmax);
            double d[3];
            min_image(S, q + 3 * bi, q + 3 * bj, d);
            double dr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) - S->br0[0];
            g[4] += 0.5 * dr * dr / nmax;
        }
    }
    for (int a = 0; a < S->nangle; ++a) {
        if (S->atype[a] != 0) continue;
        int i = S->angle[3 * a], v = S->angle[3 * a + 1], j = S->angle[3 * a + 2];
        int ni = S->nb[i], nv = S->nb[v], nj = S->nb[j];
        int nmax = ni > nv ? ni : nv;
        if (nj > nmax) nmax = nj;
        for (int s = 0; s < nmax; ++s) {
            long bi = S->off[i] + orc_slice_bead(s, ni, nmax);
            long bv = S->off[v] + orc_slice_bead(s, nv, nmax);
            long bj = S->off[j] + orc_slice_bead(s, nj, nmax);
            double r1[3], r2[3];
            min_image(S, q + 3 * bi, q + 3 * bv, r1);
            min_image(S, q + 3 * bj, q + 3 * bv, r2);
            double l1 = sqrt(r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
            double l2 = sqrt(r2[0] * r2[0] + r2[1] * r2[1] + r2[2] * r2[2]);
            double c = (r1[0] * r2[0] + r1[1] * r2[1] + r1[2] * r2[2]) / (l1 * l2);
            if (c > 1.0) c = 1.0;
            if (c < -1.0) c = -1.0;
            double dth = acos(c) - S->at0[0];
            g[5] += 0.5 * dth * dth / nmax;
        }
    }
    for (int k = 0; k < 6; ++k) g6[k] = g[k];
}

/* ---------------- ring-polymer springs ----------------------------------- */

double orc_beta(const orc_sys *S) { return 1.0 / (o_kb() * S->temperature); }

/* Spring constant N m / (beta hbar)^2 in amu/fs^2. */
static double spring_k(const orc_sys *S, int i)
{
    double bh = orc_beta(S) * o_hbar();
    return S->nb[i] * S->mass[i] / (bh * bh);
}

/* Returns E_sp in kcal/mol; Fsp (may be NULL) gets -dE_sp/dq in kcal/mol/A. */
double orc_springs(const orc_sys *S, const double *q, double *Fsp)
{
    double esum = 0.0;
    long B = S->off[S->n];
    if (Fsp) memset(Fsp, 0, sizeof(double) * 3 * B);
    for (int i = 0; i < S->n; ++i) {
        int n = S->nb[i];
        double k = spring_k(S, i) / o_kcal();      /* kcal/mol/A^2 */
        for (int a = 0; a < n; ++a) {
            long b0 = S->off[i] + a, b1 = S->off[i] + (a + 1) % n;
            for (int c = 0; c < 3; ++c) {
                double d = q[3 * b0 + c] - q[3 * b1 + c];
                esum += 0.5 * k * d * d;
                if (Fsp) { Fsp[3 * b0 + c] -= k * d; Fsp[3 * b1 + c] += k * d; }
            }
        }
    }
    return esum;
}

/* ---------------- normal modes ------------------------------------------ */

/* Orthonormal real basis C[j*N + k] (bead j, mode k) of the cyclic ring:
 * k = 0: 1/sqrt(N); 1 <= k < N/2: sqrt(2/N) cos(2 pi j k / N);
 * k = N/2: (-1)^j / sqrt(N); N/2 < k < N: sqrt(2/N) sin(2 pi j k / N).
 * The phase uses j k mod N (the functions have period N in j k), which keeps
 * the argument below 2 pi and the basis accurate to rounding for large N. */
void orc_nm_basis(int N, double *C)
{
    for (int j = 0; j < N; ++j)
        for (int k = 0; k < N; ++k) {
            double v;
            double ph = 2.0 * O_PI * (double)(((long)j * k) % N) / N;
            if (k == 0) v = 1.0 / sqrt((double)N);
            else if (2 * k < N) v = sqrt(2.0 / N) * cos(ph);
            else if (2 * k == N) v = ((j % 2) ? -1.0 : 1.0) / sqrt((double)N);
            else v = sqrt(2.0 / N) * sin(ph);
            C[(long)j * N + k] = v;
        }
}

/* Eigenvalue of the cyclic second-difference matrix for mode k. */
double orc_nm_lambda(int N, int k)
{
    double s = sin(O_PI * k / N);
    return 4.0 * s * s;
}

/* Mode angular frequency (1/fs) of particle i: sqrt(k_spring lambda_k / m_f). */
double orc_nm_omega(const orc_sys *S, int i, int k)
{
    return sqrt(spring_k(S, i) * orc_nm_lambda(S->nb[i], k) / S->fm[i]);
}

/* dir = +1: out = C^T in (bead -> mode); dir = -1: out = C in (mode -> bead).
 * Arrays are bead tables [B][3]; each particle/component column separately. */
void orc_nm_transform(const orc_sys *S, int dir, const double *in, double *out)
{
    for (int i = 0; i < S->n; ++i) {
        int N = S->nb[i];
        double *C = (double *)malloc(sizeof(double) * N * N);
        orc_nm_basis(N, C);
        for (int c = 0; c < 3; ++c)
            for (int o = 0; o < N; ++o) {
                double acc = 0.0;
                for (int x = 0; x < N; ++x) {
                    double m = dir > 0 ? C[x * N + o] : C[o * N + x];
                    acc += m * in[3 * (S->off[i] + x) + c];
                }
                out[3 * (S->off[i] + o) + c] = acc;
            }
        free(C);
    }
}

/* Exact evolution of the free ring polymers for time t (Sec. "Evaluation"):
 * in normal modes each mode is a harmonic oscillator of mass m_f and
 * frequency omega_k (the k = 0 centroid mode moves freely). */
void orc_free_propagate(const orc_sys *S, double *q, double *p, double t)
{
    for (int i = 0; i < S->n; ++i) {
        int N = S->nb[i];
        double *C = (double *)malloc(sizeof(double) * N * N);
        double *xi = (double *)malloc(sizeof(double) * N);
        double *pi = (double *)malloc(sizeof(double) * N);
        orc_nm_basis(N, C);
        double m = S->fm[i];
        for (int c = 0; c < 3; ++c) {
            for (int k = 0; k < N; ++k) {
                double a = 0.0, b = 0.0;
                for (int j = 0; j < N; ++j) {
                    a += C[j * N + k] * q[3 * (S->off[i] + j) + c];
                    b += C[j * N + k] * p[3 * (S->off[i] + j) + c];
                }
                xi[k] = a;
                pi[k] = b;
            }
            for (int k = 0; k < N; ++k) {
                double w = orc_nm_omega(S, i, k);
                if (k == 0 || w == 0.0) {
                    xi[k] += pi[k] * t / m;
                } else {
                    double cw = cos(w * t), sw = sin(w * t);
                    double x0 = xi[k], p0 = pi[k];
                    xi[k] = x0 * cw + p0 * sw / (m * w);
                    pi[k] = p0 * cw - m * w * x0 * sw;
                }
            }
            for (int j = 0; j < N; ++j) {
                double a = 0.0, b = 0.0;
                for (int k = 0; k < N; ++k) {
                    a += C[j * N + k] * xi[k];
                    b += C[j * N + k] * pi[k];
                }
                q[3 * (S->off[i] + j) + c] = a;
                p[3 * (S->off[i] + j) + c] = b;
            }
        }
        free(C);
        free(xi);
        free(pi);
    }
}

/* ---------------- observables -------------------------------------------- */

/* e[0..5]: potential terms as given in vpot (V_mix..V_angle); fills the rest:
 * spring energy, kinetic energy sum p^2/2m_f, centroid-virial kinetic
 * estimator sum_i 3/(2 beta) - 1/2 sum_{i,a} (q_ia - qbar_i) . F_ia, primitive
 * estimator sum_i 3 N_i/(2 beta) - E_sp, and H = KE + E_sp + V_mix.
 * Energies in kcal/mol; F are the V_mix bead forces. */
void orc_observables(const orc_sys *S, const double *q, const double *p,
                     const double *F, const double *vpot, double *e)
{
    for (int k = 0; k <= E_ANGLE; ++k) e[k] = vpot[k];
    double esp = orc_springs(S, q, NULL);
    double kin = 0.0, vir = 0.0;
    double kT = o_kb_kcal() * S->temperature;
    double kcv = 0.0, kprim = 0.0;
    for (int i = 0; i < S->n; ++i) {
        int N = S->nb[i];
        double qbar[3] = {0, 0, 0};
        for (int a = 0; a < N; ++a)
            for (int c = 0; c < 3; ++c) qbar[c] += q[3 * (S->off[i] + a) + c] / N;
        for (int a = 0; a < N; ++a)
            for (int c = 0; c < 3; ++c) {
                long x = 3 * (S->off[i] + a) + c;
                kin += p[x] * p[x] / (2.0 * S->fm[i]);
                vir += (q[x] - qbar[c]) * F[x];
            }
        kcv += 1.5 * kT;
        kprim += 1.5 * N * kT;
    }
    e[E_SPRING] = esp;
    e[E_KIN] = kin / o_kcal();
    e[E_KCV] = kcv - 0.5 * vir;
    e[E_KPRIM] = kprim - esp;
    e[E_HAM] = e[E_KIN] + esp + e[E_VMIX];
}

/* ---------------- integrator --------------------------------------------- */

/* nsteps of the split propagator: p += dt/2 F; exact free ring polymers for
 * dt; F = F_mix(q); p += dt/2 F.  On entry F must hold F_mix(q).  elog (may
 * be NULL) receives E_N energies per step, evaluated after the step. */
void orc_step(const orc_sys *S, int nsteps, double *q, double *p, double *F,
              double *elog)
{
    long B = S->off[S->n];
    double kick = 0.5 * S->dt * o_kcal();     /* kcal/mol/A * fs -> amu A/fs */
    double vpot[E_N];
    for (int st = 0; st < nsteps; ++st) {
        for (long x = 0; x < 3 * B; ++x) p[x] += kick * F[x];
        orc_free_propagate(S, q, p, S->dt);
        orc_forces_o2(S, q, F, vpot);
        for (long x = 0; x < 3 * B; ++x) p[x] += kick * F[x];
        if (elog) orc_observables(S, q, p, F, vpot, elog + (size_t)st * E_N);
    }
}

/* ---------------- path-integral Langevin thermostat ---------------------- */

/* Friction of mode k of particle i: the centroid (k = 0) gets 1/tau0 (0 for
 * tau0 <= 0 or infinite), every internal mode 2 omega_k (the local PILE
 * choice: critical damping of each free-ring mode). */
double orc_pile_gamma(const orc_sys *S, int i, int k, double tau0)
{
    if (k == 0) return (tau0 > 0.0 && isfinite(tau0)) ? 1.0 / tau0 : 0.0;
    return 2.0 * orc_nm_omega(S, i, k);
}

/* One Ornstein-Uhlenbeck half step of the momenta in the normal modes of
 * each ring: pi_k <- c1 pi_k + c2 sqrt(m_f k_B T) eta_k with
 * c1 = exp(-gamma_k t), c2 = sqrt(1 - c1^2).  eta is a bead table [B][3]
 * of standard normals indexed by mode: particle i, mode k, component c at
 * eta[3 (off_i + k) + c]. */
void orc_pile(const orc_sys *S, double *p, const double *eta, double t, double tau0)
{
    double kT = o_kb() * S->temperature;      /* amu A^2 / fs^2 */
    for (int i = 0; i < S->n; ++i) {
        int N = S->nb[i];
        double *C = (double *)malloc(sizeof(double) * N * N);
        double *pi = (double *)malloc(sizeof(double) * N);
        orc_nm_basis(N, C);
        double sd = sqrt(S->fm[i] * kT);
        for (int c = 0; c < 3; ++c) {
            for (int k = 0; k < N; ++k) {
                double b = 0.0;
                for (int j = 0; j < N; ++j) b += C[j * N + k] * p[3 * (S->off[i] + j) + c];
                double c1 = exp(-orc_pile_gamma(S, i, k, tau0) * t);
                double c2 = sqrt(1.0 - c1 * c1);
                pi[k] = c1 * b + c2 * sd * eta[3 * (S->off[i] + k) + c];
            }
            for (int j = 0; j < N; ++j) {
                double b = 0.0;
                for (int k = 0; k < N; ++k) b += C[j * N + k] * pi[k];
                p[3 * (S->off[i] + j) + c] = b;
            }
        }
        free(C);
        free(pi);
    }
}

/* nsteps of the thermostatted split propagator O B A B O: a Langevin half
 * step of length dt/2 (noise[st][0]), p += dt/2 F, exact free ring polymers
 * for dt, F = F_mix(q), p += dt/2 F, a Langevin half step (noise[st][1]).
 * noise: [nsteps][2][B][3] standard normals, mode-indexed as in orc_pile.
 * elog (may be NULL) gets the energies after the second half kick (before
 * the closing Langevin half step). */
void orc_step_nvt(const orc_sys *S, int nsteps, double *q, double *p, double *F,
                  const double *noise, double tau0, double *elog)
{
    long B = S->off[S->n];
    double kick = 0.5 * S->dt * o_kcal();
    double vpot[E_N];
    for (int st = 0; st < nsteps; ++st) {
        orc_pile(S, p, noise + (size_t)(2 * st) * 3 * B, 0.5 * S->dt, tau0);
        for (long x = 0; x < 3 * B; ++x) p[x] += kick * F[x];
        orc_free_propagate(S, q, p, S->dt);
        orc_forces_o2(S, q, F, vpot);
        for (long x = 0; x < 3 * B; ++x) p[x] += kick * F[x];
        if (elog) orc_observables(S, q, p, F, vpot, elog + (size_t)st * E_N);
        orc_pile(S, p, noise + (size_t)(2 * st + 1) * 3 * B, 0.5 * S->dt, tau0);
    }
}

/* nsteps of velocity Verlet with the ring-polymer springs as forces (the
 * paper's "manual" integrator, Sec. "Evaluation"): with G = F_mix + F_sp,
 * p += dt/2 G(q); q += dt p / m_f; p += dt/2 G(q).  On entry F must hold
 * F_mix(q).  elog (may be NULL) gets the energies after each step. */
void orc_step_vv(const orc_sys *S, int nsteps, double *q, double *p, double *F,
                 double *elog)
{
    long B = S->off[S->n];
    double kick = 0.5 * S->dt * o_kcal();
    double vpot[E_N];
    double *Fsp = (double *)malloc(sizeof(double) * 3 * B);
    orc_springs(S, q, Fsp);
    for (int st = 0; st < nsteps; ++st) {
        for (long x = 0; x < 3 * B; ++x) p[x] += kick * (F[x] + Fsp[x]);
        for (int i = 0; i < S->n; ++i)
            for (long a = S->off[i]; a < S->off[i + 1]; ++a)
                for (int c = 0; c < 3; ++c) q[3 * a + c] += S->dt * p[3 * a + c] / S->fm[i];
        orc_forces_o2(S, q, F, vpot);
        orc_springs(S, q, Fsp);
        for (long x = 0; x < 3 * B; ++x) p[x] += kick * (F[x] + Fsp[x]);
        if (elog) orc_observables(S, q, p, F, vpot, elog + (size_t)st * E_N);
    }
    free(Fsp);
}

/* Constants as the oracle uses them, for tests: kcal, hbar, kB, k_e, kB(kcal). */
void orc_constants(double *out5)
{
    out5[0] = o_kcal();
    out5[1] = o_hbar();
    out5[2] = o_kb();
    out5[3] = O_KE_KCAL;
    out5[4] = o_kb_kcal();
}
