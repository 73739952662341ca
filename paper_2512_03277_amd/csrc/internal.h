// Internal declarations shared by the HIP translation units of libcavdftb.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cavdftb.h"

namespace cavdftb {

struct DevParams {
  double sk[7][4];
  double onsite[2][2];
  double U[2];
  double q0[2];
  double rep_a[3];
  double rep_alpha[3];
};

// job flags
enum : int32_t {
  JF_FORCES = 1,   // energy and forces
  JF_WARM_C = 2,   // start from the stored MO basis of the unit
  JF_WARM_DQ = 4,  // start from the stored charges of the unit
  JF_STORE = 8,    // store basis and charges after convergence
  JF_WARM_HIST = 16,   // start the mixer from the unit's stored Broyden history
  JF_STORE_HIST = 32,  // keep the Broyden history in the unit's store afterwards
};

constexpr int kMaxHist = 20;  // Broyden window

struct SccArgs {
  DevParams prm;
  const double* pos;        // [n_atoms][3]
  const int32_t* unit_off;  // [n_units+1]
  const int8_t* species;    // [n_atoms]
  const int32_t* job_unit;  // [n_jobs]
  const int32_t* job_disp;  // [n_jobs] or nullptr; -1 = undisplaced, >= 0: displaced job
                            // (atom*3+dir)*2 + (step<0); <= -2: field job -2 - (dir*2 + (field<0))
  const int32_t* unit_mask; // [n_units] or nullptr: jobs of units with mask 0 are skipped
  int32_t n_jobs;
  const int32_t* n_jobs_dev; // if set, the job count is read from device memory (compacted job lists)
  unsigned int* job_counter; // if set, jobs are taken from a queue (reset to 0 before the launch)
  double fd_h;              // displacement (bohr) of displaced jobs, field (a.u.) of field jobs
  const int64_t* ws_off;    // [n_units] offset of the unit's stored basis in ws_C (doubles)
  double* ws_C;             // stored MO bases, NMAX x NMAX per unit of the bucket
  double* ws_dq;            // [n_atoms] stored charges (electron excess)
  double* ws_dq_hist;       // [2][n_atoms] charges of the two MD steps before, or nullptr
  int32_t n_extrap;         // stored MD steps usable for extrapolating the start charges (0..3)
  int32_t fd_pass;          // displaced or field jobs of central differences: 0 all; 1 only +h / +field,
                            // 2 only -h / -field
  double* fd_dq;            // per + job the charge response ddq = dq(+) - dq_centre of its last converged
                            // run (NaN after a failed one): fd_dq_off[u] + slot n_a + t, slot 3 atom + dir
                            // (displaced) or 3 n_a + dir (field).  A -h job starts from dq_centre - ddq of
                            // this pass 1; a +h job from dq_centre + ddq of the previous evaluation.
  const int64_t* fd_dq_off; // [n_units] offsets into fd_dq (3 n_a^2 + 3 n_a per unit)
  int32_t n_atoms;
  double* hist;             // per-unit Broyden history store (or nullptr)
  const int64_t* hist_off;  // [n_units] offset of each unit's history block
  double* scratch;          // [gridDim.x][scratch_per_wg]
  int64_t scratch_per_wg;
  double* energy;           // [n_units] or nullptr
  double* forces;           // [n_atoms][3] or nullptr
  double* charges;          // [n_atoms] or nullptr
  double* dipole;           // [n_units][3] or nullptr (written for undisplaced jobs)
  double* mu_job;           // [n_jobs][3] or nullptr (written for displaced and field jobs)
  double* f_job;            // [6][n_atoms][3] or nullptr: forces of the field jobs, by field code
  int32_t* f_status;        // [n_units][6] or nullptr: status of the field jobs, by field code
  int32_t* status;          // [n_units] (undisplaced jobs) or nullptr
  int32_t* unit_fail;       // [n_units] or nullptr: 1 when the unit's last undisplaced SCC did not
                            // converge (read by every job of the unit, written by undisplaced jobs)
  int32_t* job_status;      // [n_jobs] or nullptr
  int32_t* job_iters;       // [n_jobs] or nullptr
  unsigned long long* counters;  // [8]: jobs, iterations, algorithmic flops, Jacobi sweeps, surrogate fallback units,
                                 // full diagonalisations, tridiagonal solves, tridiagonal solves discarded
  double tol;
  int32_t max_iter;
  double alpha;
  double w0;
  double jac_factor;        // Jacobi off-diagonal target = max(1e-14, jac_factor * previous SCC residual)
  int32_t eig_mode;         // CAVDFTB_EIG_*: eigensolver choice of the SCC iterations
  int32_t flags;
};

// doubles of Broyden history kept per unit of a bucket
inline int64_t hist_doubles(int nmax) { return 2 + (int64_t)kMaxHist * kMaxHist + 2LL * kMaxHist * nmax; }

// scratch doubles needed per workgroup for a bucket
int64_t scc_scratch_per_wg(int nmax);
// launch the SCC kernel of the bucket nmax over args.n_jobs jobs with n_wg workgroups
hipError_t launch_scc(int nmax, int n_wg, const SccArgs& args, hipStream_t stream);
// workgroups per CU the SCC kernel of a bucket can keep resident
int scc_blocks_per_cu(int nmax);

// ---- cavity / integrator kernels (md_kernels.hip) ----
struct CavArgs {
  int32_t n_units, n_atoms, n_modes;
  const double* unit_x;
  const double* k;
  const double* theta;
  const double* omega;
  const double* lam;
  double pol[3];
};

// e . mu_n, zero for units with a status bit (status may be null: no masking)
hipError_t launch_mu_pol(const double* dipole, const double pol[3], int n_units, const int32_t* status,
                         double* mu_pol, hipStream_t s);
hipError_t launch_cav_scatter(const CavArgs& c, const double* mu_pol, double* F, double* fq, hipStream_t s);
hipError_t launch_cav_gather(const CavArgs& c, const double* q, const double* F, double* field, hipStream_t s);
hipError_t launch_init_photons(const CavArgs& c, const double* F, double* qm, double* pm, hipStream_t s);
// q_m += sqrt(kT) xi_m / omega_m, p_m = sqrt(kT) xi_{M+m} (xi: 2M standard normals)
hipError_t launch_photon_thermal(const CavArgs& c, double kT, const double* xi, double* qm, double* pm,
                                 hipStream_t s);
hipError_t launch_born_mulliken(const double* charges, int n_atoms, double* born, hipStream_t s);
hipError_t launch_zpol_mulliken(const double* charges, const double pol[3], int n_atoms, double* zpol,
                                hipStream_t s);
hipError_t launch_born_field_assemble(int n_atoms, const int32_t* atom_unit, const int32_t* unit_off,
                                      const double* f_job, double e, const double pol[3], const int32_t* f_status,
                                      const int32_t* unit_mask, double* born, double* zpol, int32_t* status,
                                      hipStream_t s);
hipError_t launch_born_fd_assemble(const int32_t* unit_off, const int32_t* fd_unit, const int32_t* fd_job0,
                                   int n_fd_units, const double* mu_job, double h, const double pol[3],
                                   const int32_t* job_status, const int32_t* unit_mask, double* born, double* zpol,
                                   int32_t* status, hipStream_t s);
// forward differences against the undisplaced dipoles (3 jobs per atom)
hipError_t launch_born_fd_forward_assemble(const int32_t* unit_off, const int32_t* fd_unit, const int32_t* fd_job0,
                                           int n_fd_units, const double* mu_job, const double* dipole, double h,
                                           const double pol[3], const int32_t* job_status, double* born,
                                           double* zpol, int32_t* status, hipStream_t s);
hipError_t launch_kick_drift(int n_atoms, const int32_t* atom_unit, const double* inv_mass, const double* forces,
                             const double* zpol, const double* field, double dt, double* r, double* p,
                             int do_drift, const int32_t* status, hipStream_t s);  // no cavity force on flagged units
hipError_t launch_photon_kick(int n_modes, const double* omega, const double* lam, const double* F, double dt,
                              double* pm, int rotate, double* qm, hipStream_t s);
// rows of 8 doubles of partial sums the observables need for n units, modes or jobs
int observables_part_rows(int n);
// step observables into row *obs_row of obs (then the counter advances): a first
// pass writes fixed-order partial sums into part (part_rows rows of 8 doubles,
// at least observables_part_rows(max(n_units, n_modes, n_jobs)), else
// hipErrorInvalidValue), a one-workgroup second pass totals them in fixed order
hipError_t launch_observables(int n_units, int n_atoms, int n_modes, const int32_t* unit_off,
                              const double* mass, const double* p, const double* energy,
                              const double* qm, const double* pm, const double* omega, const double* lam,
                              const double* F, const double* mu_pol, const int32_t* status,
                              const int32_t* job_iters, int n_jobs, double* part, int part_rows, double* obs,
                              unsigned int* obs_row, hipStream_t s);
// ---- real-space cavity (one photon pair per cell) ----
hipError_t launch_rs_photon_kick(int n, const double* mu_pol, double eta, double dt, double* pn, hipStream_t s);
hipError_t launch_rs_field(int n, const double* q, const double* mu_pol, double eta, double w0, double* field,
                           hipStream_t s);
hipError_t launch_rs_init(int n, const double* mu_pol, double eta, double w0, double* q, double* pn, hipStream_t s);
// adds to (q_n, p_n) the real-space image of the k-space fluctuation q_k = sqrt(kT) xi_k / omega_k,
// p_k = sqrt(kT) xi_{N+k} (xi: 2N standard normals); buf0, buf1: [n] transform buffers
hipError_t launch_rs_thermal(int n, const double* wk, double w0, double kT, const double* xi, double* q, double* pn,
                             double2* buf0, double2* buf1, hipStream_t s);
// Steps 2-4: transform to k-space, rotate by omega_k dt (recording q_k when qk_rec
// is not null), transform back; buf0 / buf1 hold n complex values each
hipError_t launch_rs_photon_step(int n, const double* wk, double w0, double dt, double* q, double* pn,
                                 double2* buf0, double2* buf1, double* qk, double* pk, double* qk_rec,
                                 hipStream_t s);
hipError_t launch_rs_observables(int n_units, const int32_t* unit_off, const double* mass, const double* p,
                                 const double* energy, const double* q, const double* mu_pol, const double* qk,
                                 const double* pk, const double* wk, double eta, double w0, const int32_t* status,
                                 const int32_t* job_iters, double* part, int part_rows, double* obs,
                                 unsigned int* obs_row, hipStream_t s);
// reorders `order` (n units of a bucket) by the cost of their last evaluation,
// iters[j] cost_scale[order[j]] with cost_scale[u] = (orbitals / bucket nmax)^3,
// largest first; tmp: [n] scratch
hipError_t launch_order_by_cost(int n, int32_t* order, const int32_t* iters, const float* cost_scale, int32_t* tmp,
                                hipStream_t s);
// *c = v by a one-thread kernel (a kernel node, not a memset, inside captured graphs)
hipError_t launch_set_u32(unsigned int* c, unsigned int v, hipStream_t s);

// ---- surrogate kernels (sg_kernels.hip) ----
hipError_t launch_sg_features(int n_atoms, const int32_t* atom_unit, const int32_t* unit_off, const int8_t* species,
                              const double* pos, double* feat, double* frames, hipStream_t s);
hipError_t launch_sg_prep(int n, int width, const int32_t* idx, const double* v, const float* norm, float* x,
                          hipStream_t s);
hipError_t launch_sg_forward(const float* P, const float* x, int n, float* y, float* act, hipStream_t s);
hipError_t launch_sg_backward(const float* P, const float* x, const float* act, const float* dy, int n, float* grad,
                              float* work, hipStream_t s);
hipError_t launch_sg_mse(const float* y, const float* t, int count, float* dy, float* loss, float* work,
                         hipStream_t s);
hipError_t launch_sg_adam(float* w, const float* g, float* m, float* v, int count, float lr, float b1, float b2,
                          float eps, int step, hipStream_t s);
hipError_t launch_sg_gather(const float* src, const int32_t* idx, int n, int width, float* dst, hipStream_t s);
hipError_t launch_sg_moments(const double* x, const int32_t* idx, int n, int width, float* out, hipStream_t s);
hipError_t launch_sg_to_local(int n, const int32_t* idx, const double* frames, const double* born,
                              const double* charges, double* out, hipStream_t s);
hipError_t launch_sg_combine(int n_atoms, const int8_t* species, const int32_t* pos_in_species,
                             const int32_t* n_species, const float* ybuf, const float* norm, const double* frames,
                             const double* charges, double* born, double* std, hipStream_t s);
hipError_t launch_sg_asr_flag(int n_units, const int32_t* unit_off, double* born, const double* std, double thr,
                              int32_t* flag, unsigned long long* n_flagged, hipStream_t s);
hipError_t launch_zpol_from_born(int n, const double* born, const double pol[3], double* zp, hipStream_t s);
hipError_t launch_fd_compact(int n_units_b, const int32_t* units_b, const int32_t* unit_off, const int32_t* flag,
                             int field, int32_t* job_unit, int32_t* job_disp, int32_t* job0, int32_t* n_jobs,
                             hipStream_t s);

}  // namespace cavdftb
