/*
 * cavdftb: batched SCC-DFTB matter + multimode Fabry-Perot cavity dynamics on
 * MI355X (gfx950).  C ABI over a HIP shared library (libcavdftb.so).
 *
 * The method is that of Wickramasinghe, Amini and Mandal, "On-the-Fly
 * Cavity-Molecular Dynamics of Vibrational Polaritons" (arXiv 2512.03277):
 * many independent molecular cells (Theory, Eq. hm), each described by
 * second-order SCC-DFTB (Computational details), coupled through their
 * projected dipoles to cavity modes whose mode functions depend on the cell
 * position along the cavity axis (Theory, Eq. hlm_bigin and the mode function
 * f_k(R_n)), propagated by the velocity-Verlet-like scheme with an exact free
 * photon rotation (Theory, Step 1 Eq. pj1 and Step 3 Eq. qknk).
 *
 * Conventions shared by every call
 *   - Atomic units throughout (bohr, hartree, a.u. of time, electron mass).
 *   - All arrays are FP64 unless typed otherwise, owned by the caller.
 *   - Pointers marked "device" are HIP device pointers (for instance torch
 *     tensor data pointers on the same GPU); pointers marked "host" are read
 *     during the call only.
 *   - Every call is asynchronous on the HIP stream given at creation, except
 *     cavdftb_create, cavdftb_destroy and cavdftb_sync, which synchronise.
 *   - The library allocates all of its workspaces in cavdftb_create; no later
 *     call allocates device memory.
 *   - Return codes: CAVDFTB_OK or a negative CAVDFTB_E* value; no C++
 *     exception crosses the ABI and the library never aborts.  Per-unit
 *     failures are reported in unit_status bit masks (CAVDFTB_ST_*); they do
 *     not make the call fail.  cavdftb_last_error returns a readable reason.
 *   - Units are given in CSR form (unit_atom_off); atom order inside a unit is
 *     free; species 0 = O (orbitals s, px, py, pz), 1 = H (s).  A unit may
 *     hold at most CAVDFTB_MAX_ORBITALS (192) orbitals - 32 water molecules -
 *     and its orbital count must be even.
 */
#ifndef CAVDFTB_H
#define CAVDFTB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CAVDFTB_OK 0
#define CAVDFTB_EINVAL (-1)
#define CAVDFTB_ENOMEM (-2)
#define CAVDFTB_EHIP (-3)

/* unit_status bits */
#define CAVDFTB_ST_NOT_CONVERGED 1 /* SCC hit max_iter, or set no new smallest residual for 20 iterations (5 when the unit's last undisplaced SCC was flagged so), before reaching tol */
#define CAVDFTB_ST_NOT_PD 2        /* overlap matrix not positive definite */
#define CAVDFTB_ST_DEGENERATE 4    /* HOMO-LUMO gap below 1e-6 hartree */
#define CAVDFTB_ST_NAN 8           /* non-finite position or charge */
/* A unit with CAVDFTB_ST_NOT_PD or CAVDFTB_ST_NAN has no valid density: it reports
 * zero charges, dipole, energy and forces, so it drops out of the cavity sums
 * and the energy totals instead of turning them non-finite for every unit.
 * In MD steps (cavdftb_step, cavdftb_init_photons) a unit with any status bit
 * is left out of the cavity coupling for that evaluation: its e . mu enters the
 * mode sums F_m as zero and its atoms feel no cavity force, so one failing
 * unit cannot drive the field that every other unit feels. */

/* Born-charge modes */
#define CAVDFTB_BORN_MULLIKEN 0  /* Z_A = Q_A I (the paper's cheap replacement, Results) */
#define CAVDFTB_BORN_FD 1        /* central finite differences of the SCC dipole (Results) */
#define CAVDFTB_BORN_SURROGATE 2 /* learned ensemble, exact route for units where it disagrees */
#define CAVDFTB_BORN_FIELD 3     /* exact, from the force response to a uniform field (Maxwell relation) */
#define CAVDFTB_BORN_FD_FORWARD 4 /* forward differences of the SCC dipole (the paper's own scheme) */

/* Surrogate network: per species (O, H) and member, 80 -> 128 SiLU -> 128
 * SiLU -> 9, flat FP32 parameters [W1 (80x128, row = input) | b1 | W2 (128x128)
 * | b2 | W3 (128x9) | b3]; normalisation per species [x_mean 80 | x_std 80 |
 * y_mean 9 | y_scale 9].  The 80 inputs per atom: 16 radial Gaussians per
 * neighbour species, then 8 Gaussians x 3 frame components of the neighbour
 * directions per neighbour species (cavdftb_sg_features). */
#define CAVDFTB_SG_N_IN 80
#define CAVDFTB_SG_N_HID 128
#define CAVDFTB_SG_N_OUT 9
#define CAVDFTB_SG_MEMBERS 4
#define CAVDFTB_SG_N_PARAM 28041
#define CAVDFTB_SG_N_NORM 178

#define CAVDFTB_MAX_ORBITALS 192

/* Synthetic SCC-DFTB parameter set.  Table index t (0..6): O-O ss sigma,
 * O-O sp sigma, O-O pp sigma, O-O pp pi, O-H (s_H s_O) sigma,
 * O-H (s_H p_O) sigma, H-H ss sigma; sk[t] = {a, b, c, d} with hopping
 * a exp(-b r) and overlap c exp(-d r).  Pair types for repulsion
 * A exp(-alpha r): 0 = O-O, 1 = O-H, 2 = H-H. */
typedef struct cavdftb_params {
  double sk[7][4];
  double onsite[2][2]; /* [species][l]: O {eps_s, eps_p}, H {eps_s, unused} */
  double hubbard_u[2]; /* U_O, U_H (hartree); gamma uses tau = 16 U / 5 */
  double q0[2];        /* neutral valence populations: O 6, H 1 (create: CAVDFTB_EINVAL outside [0, 8] and [0, 2]) */
  double rep_a[3];
  double rep_alpha[3];
  double mass[2]; /* nuclear masses (electron masses) */
} cavdftb_params;

/* Static description of the batch and of the cavity (all host pointers,
 * copied to the device by cavdftb_create). */
typedef struct cavdftb_layout {
  int32_t n_units;
  int32_t n_atoms;
  int32_t n_modes;
  const int32_t* unit_atom_off; /* [n_units+1] CSR offsets into the atom arrays */
  const int8_t* species;        /* [n_atoms] */
  const double* unit_x;         /* [n_units] cell position X_n along the cavity axis */
  const double* omega;          /* [n_modes] mode frequencies omega_m */
  const double* k;              /* [n_modes] wave numbers k_m */
  const double* theta;          /* [n_modes] phases; phi_m(X) = sin(k_m X + theta_m) */
  const double* lam;            /* [n_modes] couplings lambda_m (eta = lambda omega for one box) */
  double pol[3];                /* cavity polarisation e (unit vector) */
} cavdftb_layout;

typedef struct cavdftb_ctx cavdftb_ctx;

/* Create a context for a fixed batch layout.  hip_stream is a hipStream_t (or
 * NULL for the null stream) on the current device.  Allocates every workspace
 * (device memory ~ sum over units of 3 n_u^2 doubles plus O(atoms + modes)).
 * Returns CAVDFTB_EINVAL for inconsistent layouts (non-monotone offsets,
 * species outside {0,1}, an odd orbital count, more than 192 orbitals), and
 * CAVDFTB_ENOMEM / CAVDFTB_EHIP on allocation failure. */
int cavdftb_create(const cavdftb_params* params, const cavdftb_layout* layout, void* hip_stream,
                   cavdftb_ctx** out);
int cavdftb_destroy(cavdftb_ctx* ctx);

/* SCC controls (defaults tol 1e-8, max_iter 200, mix_alpha 0.6): Johnson's
 * modified Broyden mixing of the atomic charges with inverse-Jacobian weight
 * w0 = 0.01 and at most 20 stored iterations; converged when
 * max_A |Dq_out - Dq_in| < tol.  A unit that sets no new smallest residual
 * for 20 iterations stops and is flagged CAVDFTB_ST_NOT_CONVERGED; while its
 * last undisplaced SCC was flagged that way, the window is 5 iterations (for
 * its displaced and field SCCs too). */
int cavdftb_set_scc(cavdftb_ctx* ctx, double tol, int32_t max_iter, double mix_alpha);

/* Solver tuning (results are unchanged to within the SCC tolerance):
 *   jacobi_res_factor (default 1e-3): in SCC iterations that diagonalise by
 *     full Jacobi, the eigensolver stops once every off-diagonal element of the
 *     rotated Hamiltonian is below max(1e-14, jacobi_res_factor x previous
 *     charge residual); 0 means always 1e-14 (hartree).
 *   keep_mixer_history (default 1): a unit's Broyden history survives between
 *     its evaluations (MD steps) and seeds its displaced finite-difference SCCs.
 * Returns CAVDFTB_EINVAL outside 0 <= jacobi_res_factor <= 1. */
int cavdftb_set_tuning(cavdftb_ctx* ctx, double jacobi_res_factor, int32_t keep_mixer_history);

/* Eigensolver of the SCC iterations.  Every SCC iteration needs the
 * occupied subspace of A = X^T H X in the current S-orthonormal basis X.
 *   CAVDFTB_EIG_AUTO (default): while the occupied and virtual columns of X
 *     stay well separated, one occupied-virtual rotation of X (an exactly
 *     orthogonal Cayley transform) per iteration; otherwise (cold start, small
 *     gaps) a full diagonalisation: cyclic Jacobi for units of at most 64
 *     orbitals, and above that Householder tridiagonalisation, bisection,
 *     twisted-factorisation eigenvectors and a blocked back-transform on the
 *     FP64 matrix cores (cyclic Jacobi again if that solve fails its
 *     S-orthonormality check, counted in tridiagonal_fallbacks).
 *   CAVDFTB_EIG_FULL: a full diagonalisation in every SCC iteration.
 *   CAVDFTB_EIG_JACOBI: as AUTO, but every full diagonalisation by Jacobi.
 * The converged results agree to within the SCC tolerance.  CAVDFTB_EINVAL
 * for another value. */
#define CAVDFTB_EIG_AUTO 0
#define CAVDFTB_EIG_FULL 1
#define CAVDFTB_EIG_JACOBI 2
int cavdftb_set_eigensolver(cavdftb_ctx* ctx, int32_t mode);

/* Launch schedule of the SCC kernel.  job_queue != 0 (default): workgroups take
 * the next job from a device queue, each bucket's units ordered largest first
 * (longest-processing-time order); 0: a fixed stride over the job list.
 * max_wg_per_cu > 0 caps the resident workgroups per CU of every bucket (at most
 * what create sized the scratch for); 0 restores that maximum.  Results do not
 * depend on either setting. */
int cavdftb_set_schedule(cavdftb_ctx* ctx, int32_t job_queue, int32_t max_wg_per_cu);

/* Launch schedule of one orbital bucket (8, 16, 32, 48, 64, 96, 128 or 192
 * orbitals; units are bucketed by their orbital count at creation):
 * wg_per_cu resident workgroups per CU (0: the maximum the scratch was sized
 * for; larger values are clamped to it), eig_mode a CAVDFTB_EIG_* mode for
 * this bucket's units or -1 for the context's, job_queue 1 (device queue,
 * units by cost) / 0 (fixed stride) or -1 for the context's.  A bucket the
 * layout does not use is accepted and has no effect.  The workgroup count and
 * the job order change no result; the eigensolver changes results within the
 * SCC tolerance.  CAVDFTB_EINVAL for another bucket size or setting. */
int cavdftb_set_bucket_schedule(cavdftb_ctx* ctx, int32_t bucket_orbitals, int32_t wg_per_cu, int32_t eig_mode,
                                int32_t job_queue);
/* Host outputs (any may be NULL): units in the bucket, the largest and the
 * current resident workgroups per CU. */
int cavdftb_bucket_info(cavdftb_ctx* ctx, int32_t bucket_orbitals, int32_t* n_units, int32_t* wg_per_cu_max,
                        int32_t* wg_per_cu);
/* Apply a launch table written by the autotuner (paper_2512_03277_amd/autotune.py):
 * a JSON file whose flat objects {"arch": "gfx950", "bucket": 48,
 * "wg_per_cu": 2, "eig_mode": 0, "job_queue": 1} each set one bucket through
 * cavdftb_set_bucket_schedule (missing keys: 0, -1, -1); objects for another
 * architecture than the current device's are skipped.  Returns the number of
 * entries applied (>= 0), or CAVDFTB_EINVAL for an unreadable file, an entry
 * without "bucket" or "arch", or a bad setting. */
int cavdftb_load_launch_table(cavdftb_ctx* ctx, const char* path);
/* Streams that the bucket launches of an undisplaced evaluation of every
 * unit (cavdftb_eval_units, the MD steps, the centre pass of
 * cavdftb_born_charges and of the photon starts) are spread over, 1..4 (default 4): the context stream and up to three side
 * streams of default priority that the library creates.  Buckets go, largest
 * estimated cost first, to the stream with the least work so far; the side
 * streams wait for the context stream's earlier work and the context stream
 * waits for them before its next work, so callers see one stream.  Results
 * are bit-identical for every count (the buckets hold disjoint units).  MD
 * steps replayed from a graph (cavdftb_set_graph) keep their launches on the
 * context stream.  Returns CAVDFTB_EINVAL for a count outside 1..4. */
int cavdftb_set_bucket_streams(cavdftb_ctx* ctx, int32_t n_streams);

/* Warm start: when enabled (default 1) each unit evaluation starts from the
 * charges, the molecular-orbital basis and the mixer history its previous
 * evaluation stored.  cavdftb_reset_warm_start forgets them (the next
 * evaluation starts cold), and the charge responses that start the +h / +field
 * jobs of the Born routes (cavdftb_born_charges). */
int cavdftb_set_warm_start(cavdftb_ctx* ctx, int32_t enable);
int cavdftb_reset_warm_start(cavdftb_ctx* ctx);

/* SCC-DFTB of every unit at positions pos (device [n_atoms][3]): the matter
 * potential V_n, its forces and the cell dipole (Theory: the -grad V_n term
 * and mu_n of Eq. dpj; Computational details: second-order SCC-DFTB).
 * Outputs (device, any may be NULL except unit_status):
 *   energy [n_units]        E_n = Tr(P H0) + 1/2 Dq gamma Dq + E_rep
 *   forces [n_atoms][3]     -dE_n/dR
 *   charges [n_atoms]       Mulliken net charges Q_A = -(q_A - q0_A)
 *   dipole [n_units][3]     mu_n = sum_A Q_A R_A
 *   unit_status [n_units]   CAVDFTB_ST_* bits */
int cavdftb_eval_units(cavdftb_ctx* ctx, const double* pos, double* energy, double* forces, double* charges,
                       double* dipole, int32_t* unit_status);

/* Born charges born[A][a][b] = d mu_a / d R_{A b} (device [n_atoms][3][3]) at
 * positions pos (device).  mode CAVDFTB_BORN_MULLIKEN: Q_A delta_ab from one
 * SCC per unit; CAVDFTB_BORN_FD: central differences with step h (bohr) of the
 * converged SCC dipole, 6 n_atoms displaced SCCs per unit, warm-started from
 * the undisplaced solution, in two launches per orbital bucket: every +h SCC,
 * started from the undisplaced charges plus that job's charge response at the
 * previous evaluation (zero before the first), then every -h SCC started from
 * the +h charges reflected through the undisplaced ones (Results: the Born
 * charges are the bottleneck and are taken by finite differences);
 * CAVDFTB_BORN_FIELD: the same tensor from the Maxwell relation
 * d mu_a / d R_Ab = d F_Ab / d field_a, as central differences of the SCC
 * forces in a uniform field +-h e_a (h in atomic units of field, e.g. 1e-4):
 * 6 field-perturbed SCCs per unit instead of 6 n_atoms, same warm start and
 * the same two launches (+field, then -field);
 * CAVDFTB_BORN_FD_FORWARD: forward differences (mu_a(R + h e_Ab) - mu_a(R)) / h
 * against the undisplaced dipole, 3 n_atoms displaced SCCs per unit, first
 * order in h (Computational details: the paper's finite differences);
 * CAVDFTB_BORN_SURROGATE: the ensemble set by cavdftb_set_surrogate (mean of
 * the members, acoustic sum rule imposed per unit); units whose largest
 * ensemble standard deviation exceeds the threshold are recomputed by the
 * exact route chosen with cavdftb_set_fallback (default CAVDFTB_BORN_FD),
 * with step h of that route.  ens_std (device [n_atoms], may be NULL)
 * receives each atom's largest per-component ensemble standard deviation
 * (surrogate mode only; must be NULL otherwise).  Returns CAVDFTB_EINVAL for
 * the surrogate mode before cavdftb_set_surrogate. */
int cavdftb_born_charges(cavdftb_ctx* ctx, const double* pos, int32_t mode, double h, double* born,
                         double* ens_std, int32_t* unit_status);

/* The paper's real-space / reciprocal-space photon propagation (Theory, Eq.
 * hlm3 and Eq. dpj; Steps 1-4), an alternative to the mode-space cavity of
 * cavdftb_step.  One photon pair (q_n, p_n) per unit (cell n at R_n = n a), the
 * coupling taken at omega_0 for every k so that it is local in real space:
 * each cell carries eta q_n mu_n + eta^2 mu_n^2 / (2 omega_0^2), mu_n = e . mu.
 * The free photons are propagated exactly in k-space with the cavity
 * dispersion omega_k = sqrt(omega_0^2 + c^2 k^2) (= c sqrt((pi/L)^2 + k^2) with
 * omega_0 = c pi / L), k = 2 pi j / (n_units a) on the symmetric grid
 * j = -floor((n-1)/2) .. floor(n/2), stored by DFT index j mod n.
 * cavdftb_set_realspace_cavity sets eta, omega_0, c (speed of light in the
 * medium, a.u.) and a (bohr).  The transforms are radix-2 FFTs for a power-of-
 * two number of units and direct sums otherwise, up to CAVDFTB_RS_MAX_DIRECT
 * units; other sizes return CAVDFTB_EINVAL. */
#define CAVDFTB_RS_MAX_DIRECT 4096
int cavdftb_set_realspace_cavity(cavdftb_ctx* ctx, double eta, double omega0, double c_medium, double cell_a);

/* Photon start at frozen matter for the real-space scheme: one SCC per unit
 * at r, then q_n = -eta mu_n / omega_0^2 (the minimum of the local photon
 * term) and p_n = 0 (device [n_units] each). */
int cavdftb_init_photons_realspace(cavdftb_ctx* ctx, const double* r, double* qn, double* pn);

/* Thermal photon start for the real-space scheme: the start above plus the
 * classical Boltzmann fluctuation of the free field at temperature kT
 * (hartree, finite, >= 0), drawn in k-space as q_k = sqrt(kT) xi[k] / omega_k,
 * p_k = sqrt(kT) xi[n_units + k] (k by DFT index) and carried to (q_n, p_n)
 * by the inverse transform of the step below.  xi: device [2 n_units]
 * standard normal draws owned by the caller (the library draws no random
 * numbers).  Null xi or a bad kT: CAVDFTB_EINVAL.  (Reading of Step 0: the
 * paper equilibrates the photons by constrained dynamics at frozen matter;
 * this gives that equilibrium directly for the free field.) */
int cavdftb_init_photons_realspace_thermal(cavdftb_ctx* ctx, const double* r, double* qn, double* pn, double kT,
                                           const double* xi);

/* n_steps MD steps of the real-space scheme on device state r, p [n_atoms][3]
 * and qn, pn [n_units] (Steps 1-4):
 *   p_n -= dt/2 eta mu_n(t); p += dt/2 (F - (eta q_n + eta^2 mu_n / omega_0^2) e.Z);
 *   r += dt p/m; matter at r(t+dt); the same nuclear half-kick with q_n(t) and
 *   mu_n(t+dt); p_n -= dt/2 eta mu_n(t+dt);
 *   a_k = sum_n sqrt(omega_0/2N) (q_n + i p_n/omega_0) e^{-ik R_n} -> (q_k, p_k);
 *   exact rotation by omega_k dt; back with a_n = sum_k sqrt(omega_k/2N)
 *   (q_k + i p_k/omega_k) e^{ik R_n}.
 * born_mode and h_fd as in cavdftb_step (with cavdftb_set_born_interval).
 * obs (device [n_steps][CAVDFTB_N_OBS] or NULL) as in cavdftb_step, the photon
 * energy being sum_k (p_k^2 + omega_k^2 q_k^2)/2 plus the local coupling and
 * self-energy terms.  qk_record (device [n_steps][n_units] or NULL) receives
 * q_k after every step, by DFT index, for the angle-resolved photon spectra
 * (Results: I_k(omega) from the q_k autocorrelation).  The first call after
 * cavdftb_init_photons_realspace evaluates the matter at r first. */
int cavdftb_step_realspace(cavdftb_ctx* ctx, double* r, double* p, double* qn, double* pn, int32_t n_steps,
                           double dt, int32_t born_mode, double h_fd, double* obs, double* qk_record);

/* Copy of a context work array, as left by the last evaluation or MD step on the
 * context stream (device to device, asynchronous on that stream):
 *   CAVDFTB_WORK_MU_POL   [n_units]      e . mu_n, the projected unit dipoles
 *   CAVDFTB_WORK_DIPOLE   [n_units][3]   mu_n = sum_A Q_A R_A
 *   CAVDFTB_WORK_ENERGY   [n_units]      matter energies V_n
 *   CAVDFTB_WORK_CHARGES  [n_atoms]      Mulliken charges Q_A = -dq_A
 *   CAVDFTB_WORK_FORCES   [n_atoms][3]   matter forces -dV/dR
 *   CAVDFTB_WORK_FIELD    [n_units]      cavity field E_n felt by each unit
 * (Theory: mu_n and E_n of Eq. dpj.)  Recording MU_POL and the photon
 * coordinates after every step gives the dipole and photon autocorrelations
 * behind the IR and polariton spectra (Results).  dst must hold the listed
 * number of doubles.  Returns CAVDFTB_EINVAL for an unknown array. */
#define CAVDFTB_WORK_MU_POL 0
#define CAVDFTB_WORK_DIPOLE 1
#define CAVDFTB_WORK_ENERGY 2
#define CAVDFTB_WORK_CHARGES 3
#define CAVDFTB_WORK_FORCES 4
#define CAVDFTB_WORK_FIELD 5
int cavdftb_read_work(cavdftb_ctx* ctx, int32_t which, double* dst);

/* Cavity coupling for given projected dipoles mu_pol[n_units] = e . mu_n and
 * photon coordinates q[n_modes] (all device):
 *   F[m]     = sum_n phi_m(X_n) mu_pol[n]                        (dipole sums)
 *   field[n] = sum_m lambda_m omega_m phi_m(X_n) (q_m + lambda_m F_m / omega_m)
 *   fq[m]    = -lambda_m omega_m F_m          (photon coupling force, Eq. dpj)
 * Any output may be NULL.  (Theory: Eq. hlm_bigin with real standing-wave
 * mode functions; the nuclear force is -field[n] (e . Z_A).) */
int cavdftb_cavity_forces(cavdftb_ctx* ctx, const double* mu_pol, const double* q, double* F, double* field,
                          double* fq);

/* Learned Born-charge surrogate.
 * cavdftb_set_surrogate copies the ensemble into the context: params (device
 * FP32 [2 species][CAVDFTB_SG_MEMBERS][CAVDFTB_SG_N_PARAM]), norm (device FP32
 * [2][CAVDFTB_SG_N_NORM]), and the fallback threshold on the ensemble standard
 * deviation (elementary charges).
 * cavdftb_sg_features: per atom the local frame R = [e1 e2 e3] (row-major
 * 3x3; O: bisector of its two nearest H and their plane normal, H: nearest
 * O -> H and the plane normal of that water; fragments lacking those atoms
 * take the lab frame) and the 80 descriptors over the unit's atoms within a
 * cosine cutoff at 6 A: columns s*16 + k, 16 Gaussians of width 0.367 A on
 * [0.5, 6] A per neighbour species s; columns 32 + s*24 + 3k + i, the
 * neighbour directions' components along e_i weighted by 8 Gaussians of width
 * 0.786 A on [0.5, 6] A.  Device FP64 [n_atoms][80] and [n_atoms][9].
 * The remaining calls work on plain device arrays on the given stream (a
 * hipStream_t or NULL) and train one network (BF16 operands, FP32
 * accumulation, FP32 master weights):
 *   sg_prep     x[i][k] = (v[idx[i]][k] - norm[k]) / norm[width + k]  (FP64 in, FP32 out; idx may be NULL)
 *   sg_forward  y [n][9] from x [n][80]; act [n][256] keeps the pre-activations for sg_backward (or NULL)
 *   sg_backward grad [N_PARAM] of sum(dy . y); work holds ceil(n/64) x N_PARAM partial sums
 *   sg_mse      loss[0] = mean (y - t)^2 over count values, dy = 2 (y - t) / count; work >= ceil(count/256)
 *   sg_adam     Adam (Kingma & Ba) on count parameters, step = 1, 2, ...
 *   sg_gather   dst[i][:] = src[idx[i]][:]  (FP32 rows of width values)
 *   sg_moments  out = [mean(width) | std(width)] of the FP64 rows idx (or all n)
 *   sg_to_local out[i] = R^T Z R - Q I for atoms idx[i] (training targets: the correction to the
 *               Mulliken replacement in the local frame, FP64; charges may be NULL for R^T Z R)
 * In surrogate mode the network output is that correction: Z = Q_A I + R dZ_loc R^T
 * with the Mulliken charges Q_A of the same SCC evaluation. */
int cavdftb_set_surrogate(cavdftb_ctx* ctx, const float* params, const float* norm, double std_threshold);
/* Exact route of the surrogate's fallback units: CAVDFTB_BORN_FD (default) or
 * CAVDFTB_BORN_FIELD; the step passed with the surrogate mode is that route's
 * step (bohr, or atomic units of field).  CAVDFTB_EINVAL for any other mode. */
int cavdftb_set_fallback(cavdftb_ctx* ctx, int32_t mode);
int cavdftb_sg_features(cavdftb_ctx* ctx, const double* pos, double* feat, double* frames);
int cavdftb_sg_prep(const double* v, const int32_t* idx, int32_t n, int32_t width, const float* norm, float* x,
                    void* hip_stream);
int cavdftb_sg_forward(const float* params, const float* x, int32_t n, float* y, float* act, void* hip_stream);
int cavdftb_sg_backward(const float* params, const float* x, const float* act, const float* dy, int32_t n,
                        float* grad, float* work, void* hip_stream);
int cavdftb_sg_mse(const float* y, const float* t, int32_t count, float* dy, float* loss, float* work,
                   void* hip_stream);
int cavdftb_sg_adam(float* params, const float* grad, float* m, float* v, int32_t count, float lr, float beta1,
                    float beta2, float eps, int32_t step, void* hip_stream);
int cavdftb_sg_gather(const float* src, const int32_t* idx, int32_t n, int32_t width, float* dst, void* hip_stream);
int cavdftb_sg_moments(const double* x, const int32_t* idx, int32_t n, int32_t width, float* out, void* hip_stream);
int cavdftb_sg_to_local(const double* frames, const double* born, const double* charges, const int32_t* idx,
                        int32_t n, double* out, void* hip_stream);

/* Allocation-free variant of cavdftb_sg_backward, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight training loops,
 * harnesses that forbid hipMalloc): the same kernels and the same fixed-order
 * tile reduction, so grad equals cavdftb_sg_backward's bit for bit, but the
 * per-tile partial gradients live in a file-scope device array of the library
 * (CAVDFTB_SG_NOALLOC_MAX_ROWS rows: ceil(n / 64) x CAVDFTB_SG_N_PARAM floats,
 * 14.4 MB per GPU, held until the process ends) instead of a caller's work
 * buffer.  Arguments as in cavdftb_sg_backward (device pointers, stream a
 * hipStream_t or NULL).  CAVDFTB_EINVAL for a null pointer, n <= 0 or
 * n > CAVDFTB_SG_NOALLOC_MAX_ROWS; CAVDFTB_EHIP if the array's device address
 * cannot be looked up.  The first call on a device looks that address up
 * (hipGetSymbolAddress, no allocation); make it outside any graph capture.
 * Calls on one GPU share its array: calls that overlap in time on one GPU
 * (on different streams, or from several threads) race and must be ordered
 * by the caller.  Nothing is cleared between calls; every partial sum a call
 * reads it has written itself. */
#define CAVDFTB_SG_NOALLOC_MAX_ROWS 8192
int cavdftb_sg_backward_noalloc(const float* params, const float* x, const float* act, const float* dy, int32_t n,
                                float* grad, void* hip_stream);

/* Photon start at frozen matter (Step 0 reading): q_m = -lambda_m F_m/omega_m,
 * p_m = 0, with F from one SCC evaluation at r (device). */
int cavdftb_init_photons(cavdftb_ctx* ctx, const double* r, double* qm, double* pm);

/* Thermal photon start (Step 0 reading): the classical Boltzmann distribution
 * at temperature kT (hartree, finite, >= 0) of the photon energy at frozen
 * matter, q_m = -lambda_m F_m/omega_m + sqrt(kT) xi[m]/omega_m and
 * p_m = sqrt(kT) xi[M + m].  xi: device [2M] standard normal draws owned by
 * the caller (the library draws no random numbers).  Null xi (M > 0) or a bad
 * kT: CAVDFTB_EINVAL. */
int cavdftb_init_photons_thermal(cavdftb_ctx* ctx, const double* r, double* qm, double* pm, double kT,
                                 const double* xi);

/* Advance n_steps MD steps of length dt in place on device state r, p
 * [n_atoms][3] (positions, momenta) and qm, pm [n_modes]:
 *   p_m -= dt/2 lambda omega F(t); p += dt/2 (-dV/dr - E_n e.Z); r += dt p/m;
 *   matter at r(t+dt); p += dt/2 (-dV/dr - E'_n e.Z) with E' from the old q;
 *   p_m -= dt/2 lambda omega F(t+dt); exact rotation of (q_m, p_m) by omega dt
 * (Theory, Step 1 Eq. pj1 and Step 3 Eq. qknk, in mode space).  born_mode as
 * in cavdftb_born_charges, with h_fd the step of its exact route.  The forces at r(t) are those of
 * the previous call on the same context, or are evaluated first when the
 * context has not stepped yet (or after cavdftb_invalidate).
 * obs (device [n_steps][CAVDFTB_N_OBS] or NULL) receives per step:
 *   0 kinetic, 1 matter potential, 2 photon energy, 3 total, 4 mean per-unit
 *   temperature (K, centre-of-mass motion removed), 5 units with a nonzero
 *   status, 6 SCC iterations summed over units, 7 sum_n e.mu_n. */
#define CAVDFTB_N_OBS 8
int cavdftb_step(cavdftb_ctx* ctx, double* r, double* p, double* qm, double* pm, int32_t n_steps, double dt,
                 int32_t born_mode, double h_fd, double* obs);

/* Refresh interval of the exact Born charges in MD steps (CAVDFTB_BORN_FD,
 * CAVDFTB_BORN_FD_FORWARD, CAVDFTB_BORN_FIELD): with every = k > 1, cavdftb_step
 * recomputes them at the first matter evaluation after priming and then on
 * every k-th one, and reuses the last e . Z in between (the paper refreshes its
 * Born charges every 3 steps, Theory, Step 1).  Other modes and
 * cavdftb_born_charges are not affected.  Steps with k > 1 and an exact mode run
 * eagerly (no graph replay).  Returns CAVDFTB_EINVAL for every < 1. */
int cavdftb_set_born_interval(cavdftb_ctx* ctx, int32_t every);

/* MD steps as replays of one captured hipGraph (the launch sequence of one step
 * of cavdftb_step, on the context stream).  With enable != 0, cavdftb_step
 * replays the graph for every step whose launch sequence is steady: the context
 * has stepped before (primed), timing (cavdftb_enable_timing) is off, and warm
 * starts are off or their charge extrapolation has its full depth (from the
 * fourth MD step after creation, cavdftb_eval_units or cavdftb_reset_warm_start).
 * Other steps are issued eagerly.  The graph is captured again when an argument
 * of cavdftb_step or any setting changes; results equal the eager ones bit for
 * bit (the same launches with the same arguments).  The obs rows are selected by
 * a device counter reset at the start of each cavdftb_step call.  Returns
 * CAVDFTB_EINVAL when enabling on a context created on the null stream, which
 * cannot be captured.  Counters: graph_replays and graph_captures. */
int cavdftb_set_graph(cavdftb_ctx* ctx, int32_t enable);
int cavdftb_invalidate(cavdftb_ctx* ctx);

/* Wait for the context stream; n_bad_units (host, may be NULL) receives the
 * number of units whose last evaluation set a status bit. */
int cavdftb_sync(cavdftb_ctx* ctx, int32_t* n_bad_units);

/* Device-side counters since creation or the last reset: SCC evaluations
 * (jobs), SCC iterations, and the algorithmic FP64 flop count of the SCC
 * kernels (per iteration 10 n^3 + 2 n^2 n_occ, per geometry n^3/3 + 2 n^2 n_occ),
 * plus the summed duration of SCC-kernel launches timed with HIP events on the
 * context stream when timing is enabled.  Host outputs; synchronises. */
typedef struct cavdftb_counters {
  int64_t scc_jobs;
  int64_t scc_iterations;
  double scc_flops;
  double scc_kernel_ms;
  int64_t scc_launches;
  int64_t jacobi_sweeps;             /* Jacobi sweeps summed over all SCC iterations of all jobs */
  int64_t surrogate_fallback_units;  /* units recomputed by the exact route in surrogate mode */
  int64_t jacobi_iterations;         /* SCC iterations that diagonalised fully (Jacobi or tridiagonal; the
                                        others took one occupied-virtual rotation of the previous basis) */
  int64_t graph_replays;             /* MD steps run as graph replays (cavdftb_set_graph) */
  int64_t graph_captures;            /* graph captures of the MD step */
  int64_t tridiagonal_solves;        /* full diagonalisations of units above 64 orbitals by the
                                        Householder / bisection / twisted-factorisation solver */
  int64_t tridiagonal_fallbacks;     /* of those, solves discarded by their orthonormality check
                                        (the iteration then ran cyclic Jacobi) */
} cavdftb_counters;
int cavdftb_enable_timing(cavdftb_ctx* ctx, int32_t enable);
int cavdftb_read_counters(cavdftb_ctx* ctx, cavdftb_counters* out);
int cavdftb_reset_counters(cavdftb_ctx* ctx);

const char* cavdftb_last_error(const cavdftb_ctx* ctx);
const char* cavdftb_version(void);

#ifdef __cplusplus
}
#endif
#endif
