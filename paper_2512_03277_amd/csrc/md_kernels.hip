// Cavity coupling and integrator kernels (gfx950).
//
// Mode-space form of the paper's light-matter Hamiltonian (Theory, Eq.
// hlm_bigin with real standing-wave mode functions phi_m(X) = sin(k_m X +
// theta_m)):  F_m = sum_n phi_m(X_n) e.mu_n ;  the field felt by cell n is
// E_n = sum_m lambda_m omega_m phi_m(X_n) (q_m + lambda_m F_m / omega_m); the
// nuclear coupling force is -E_n e.Z_A and the photon coupling force
// -lambda_m omega_m F_m (Eq. dpj).  The integrator follows Step 1 (Eq. pj1) and
// the exact free rotation of Step 3 (Eq. qknk).  Mode functions are recomputed
// with sin() rather than streamed (M x U table is up to 1 GB), and every sum
// runs in a fixed order (no floating-point atomics).
#include <math.h>

#include <algorithm>

#include "internal.h"

namespace cavdftb {
namespace {

constexpr int kNT = 256;

__device__ double wg_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = kNT / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// e . mu_n; a unit whose evaluation set a status bit enters the mode sums as zero
// (its dipole is not that of a converged density, and one runaway unit must not
// drive every F_m)
__global__ __launch_bounds__(kNT) void mu_pol_kernel(const double* __restrict__ dip, double e0, double e1, double e2,
                                                     int n, const int32_t* __restrict__ status,
                                                     double* __restrict__ out) {
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (i < n) {
    const double v = e0 * dip[i * 3] + e1 * dip[i * 3 + 1] + e2 * dip[i * 3 + 2];
    out[i] = (!status || status[i] == 0) && isfinite(v) ? v : 0.0;
  }
}

// one workgroup per mode: F_m = sum_n phi_m(X_n) mu_n ; fq_m = -lambda omega F_m
__global__ __launch_bounds__(kNT) void scatter_kernel(const CavArgs c, const double* __restrict__ mu_pol,
                                                      double* __restrict__ F, double* __restrict__ fq) {
  __shared__ double red[kNT];
  const int m = blockIdx.x;
  const double km = c.k[m], th = c.theta[m];
  double acc = 0.0;
  for (int n = threadIdx.x; n < c.n_units; n += kNT) acc += sin(km * c.unit_x[n] + th) * mu_pol[n];
  const double f = wg_sum(acc, red);
  if (threadIdx.x == 0) {
    if (F) F[m] = f;
    if (fq) fq[m] = -c.lam[m] * c.omega[m] * f;
  }
}

// E_n = sum_m phi_m(X_n) g_m with g_m = lambda omega (q + lambda F / omega): one
// wave per cell, lane l taking the modes m = l (mod 64), then a fixed butterfly
// over the wave (enough waves to fill the chip for a few thousand cells)
__global__ __launch_bounds__(kNT) void gather_kernel(const CavArgs c, const double* __restrict__ q,
                                                     const double* __restrict__ F, double* __restrict__ field) {
  const int lane = threadIdx.x & 63;
  const int n = blockIdx.x * (kNT / 64) + (threadIdx.x >> 6);
  if (n >= c.n_units) return;  // whole waves
  const double x = c.unit_x[n];
  double acc = 0.0;
  for (int m = lane; m < c.n_modes; m += 64) {
    const double g = c.lam[m] * c.omega[m] * (q[m] + c.lam[m] * F[m] / c.omega[m]);
    acc += sin(c.k[m] * x + c.theta[m]) * g;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if (lane == 0) field[n] = acc;
}

__global__ __launch_bounds__(kNT) void init_photons_kernel(const CavArgs c, const double* __restrict__ F,
                                                           double* __restrict__ qm, double* __restrict__ pm) {
  const int m = blockIdx.x * kNT + threadIdx.x;
  if (m < c.n_modes) {
    qm[m] = -c.lam[m] * F[m] / c.omega[m];
    pm[m] = 0.0;
  }
}

// thermal start: the classical Boltzmann fluctuation of each mode about the
// relaxed start, q_m += sqrt(kT) xi_m / omega_m, p_m = sqrt(kT) xi_{M+m}
__global__ __launch_bounds__(kNT) void photon_thermal_kernel(int n_modes, const double* __restrict__ omega,
                                                             double kT, const double* __restrict__ xi,
                                                             double* __restrict__ qm, double* __restrict__ pm) {
  const int m = blockIdx.x * kNT + threadIdx.x;
  if (m >= n_modes) return;
  const double s = sqrt(kT);
  qm[m] += s * xi[m] / omega[m];
  pm[m] = s * xi[n_modes + m];
}

__global__ __launch_bounds__(kNT) void born_mulliken_kernel(const double* __restrict__ q, int n,
                                                            double* __restrict__ born) {
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (i < n)
    for (int e = 0; e < 9; ++e) born[(int64_t)i * 9 + e] = (e % 4 == 0) ? q[i] : 0.0;
}

__global__ __launch_bounds__(kNT) void zpol_mulliken_kernel(const double* __restrict__ q, double e0, double e1,
                                                            double e2, int n, double* __restrict__ zp) {
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (i < n) {
    zp[i * 3] = q[i] * e0;
    zp[i * 3 + 1] = q[i] * e1;
    zp[i * 3 + 2] = q[i] * e2;
  }
}

// one workgroup per unit, one thread per atom: Z[a][al][b] = (mu+_al - mu-_al) / 2h from the
// displaced jobs of the unit (job order (atom*3 + dir)*2 + (minus)).
__global__ __launch_bounds__(256) void born_fd_kernel(const int32_t* __restrict__ unit_off,
                                                      const int32_t* __restrict__ fd_unit,
                                                      const int32_t* __restrict__ fd_job0, int n_fd_units,
                                                      const double* __restrict__ mu_job, double h, double e0,
                                                      double e1, double e2, const int32_t* __restrict__ mask,
                                                      double* __restrict__ born, double* __restrict__ zpol) {
  const int w = blockIdx.x;
  if (w >= n_fd_units) return;
  const int u = fd_unit[w];
  if (mask && !mask[u]) return;
  const int a0 = unit_off[u], na = unit_off[u + 1] - a0;
  const int64_t j0 = fd_job0[w];
  for (int loc = threadIdx.x; loc < na; loc += blockDim.x) {
    double Z[3][3];
    for (int b = 0; b < 3; ++b) {
      const int64_t jp = j0 + (int64_t)((loc * 3 + b) * 2);
      for (int al = 0; al < 3; ++al) Z[al][b] = (mu_job[jp * 3 + al] - mu_job[(jp + 1) * 3 + al]) / (2.0 * h);
    }
    const int64_t A = a0 + loc;
    if (born)
      for (int al = 0; al < 3; ++al)
        for (int b = 0; b < 3; ++b) born[A * 9 + al * 3 + b] = Z[al][b];
    if (zpol)
      for (int b = 0; b < 3; ++b) zpol[A * 3 + b] = e0 * Z[0][b] + e1 * Z[1][b] + e2 * Z[2][b];
  }
}

// one workgroup per fd unit: Z[A][al][b] = (mu_al(+h e_Ab) - mu_al(R)) / h from the
// unit's 3 n_a forward jobs (atom-major, then b) and its undisplaced dipole
__global__ __launch_bounds__(256) void born_fd_forward_kernel(const int32_t* __restrict__ unit_off,
                                                              const int32_t* __restrict__ fd_unit,
                                                              const int32_t* __restrict__ fd_job0, int n_fd_units,
                                                              const double* __restrict__ mu_job,
                                                              const double* __restrict__ dipole, double h, double e0,
                                                              double e1, double e2, double* __restrict__ born,
                                                              double* __restrict__ zpol) {
  const int w = blockIdx.x;
  if (w >= n_fd_units) return;
  const int u = fd_unit[w];
  const int a0 = unit_off[u], na = unit_off[u + 1] - a0;
  const int64_t j0 = fd_job0[w];
  const double m0[3] = {dipole[u * 3], dipole[u * 3 + 1], dipole[u * 3 + 2]};
  for (int loc = threadIdx.x; loc < na; loc += blockDim.x) {
    double Z[3][3];
    for (int b = 0; b < 3; ++b) {
      const int64_t jp = j0 + (int64_t)(loc * 3 + b);
      for (int al = 0; al < 3; ++al) Z[al][b] = (mu_job[jp * 3 + al] - m0[al]) / h;
    }
    const int64_t A = a0 + loc;
    if (born)
      for (int al = 0; al < 3; ++al)
        for (int b = 0; b < 3; ++b) born[A * 9 + al * 3 + b] = Z[al][b];
    if (zpol)
      for (int b = 0; b < 3; ++b) zpol[A * 3 + b] = e0 * Z[0][b] + e1 * Z[1][b] + e2 * Z[2][b];
  }
}

// one thread per atom: Z[A][al][b] = (F_Ab(+e e_al) - F_Ab(-e e_al)) / 2e from the
// forces of the six field jobs of the atom's unit (Maxwell relation d mu_al / d R_Ab
// = d F_Ab / d field_al); the unit's first atom ORs the field-job status into the
// unit status.
__global__ __launch_bounds__(kNT) void born_field_kernel(int n, const int32_t* __restrict__ atom_unit,
                                                         const int32_t* __restrict__ unit_off,
                                                         const double* __restrict__ f_job, double e, double e0,
                                                         double e1, double e2, const int32_t* __restrict__ f_status,
                                                         const int32_t* __restrict__ mask,
                                                         double* __restrict__ born, double* __restrict__ zpol,
                                                         int32_t* __restrict__ status) {
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (i >= n) return;
  const int u = atom_unit[i];
  if (mask && !mask[u]) return;
  double Z[3][3];
  for (int al = 0; al < 3; ++al)
    for (int b = 0; b < 3; ++b)
      Z[al][b] = (f_job[((int64_t)(2 * al) * n + i) * 3 + b] - f_job[((int64_t)(2 * al + 1) * n + i) * 3 + b]) /
                 (2.0 * e);
  if (born)
    for (int al = 0; al < 3; ++al)
      for (int b = 0; b < 3; ++b) born[(int64_t)i * 9 + al * 3 + b] = Z[al][b];
  if (zpol)
    for (int b = 0; b < 3; ++b) zpol[(int64_t)i * 3 + b] = e0 * Z[0][b] + e1 * Z[1][b] + e2 * Z[2][b];
  if (status && f_status && i == unit_off[u]) {
    int st = status[u];
    for (int c = 0; c < 6; ++c) st |= f_status[(int64_t)u * 6 + c];
    status[u] = st;
  }
}

// OR the displaced-job status into the unit status, one thread per fd unit
__global__ __launch_bounds__(kNT) void born_fd_status_kernel(const int32_t* __restrict__ unit_off,
                                                             const int32_t* __restrict__ fd_unit,
                                                             const int32_t* __restrict__ fd_job0, int n_fd_units,
                                                             const int32_t* __restrict__ job_status,
                                                             const int32_t* __restrict__ mask, int per_atom,
                                                             int32_t* __restrict__ status) {
  const int w = blockIdx.x * kNT + threadIdx.x;
  if (w >= n_fd_units) return;
  const int u = fd_unit[w];
  if (mask && !mask[u]) return;
  const int na = unit_off[u + 1] - unit_off[u];
  int st = status[u];
  for (int j = 0; j < per_atom * na; ++j) st |= job_status[fd_job0[w] + j];
  status[u] = st;
}

// p += dt/2 (F - E_n e.Z) ; optionally r += dt p / m
__global__ __launch_bounds__(kNT) void kick_drift_kernel(int n, const int32_t* __restrict__ atom_unit,
                                                         const double* __restrict__ inv_mass,
                                                         const double* __restrict__ f,
                                                         const double* __restrict__ zp,
                                                         const double* __restrict__ field, double dt,
                                                         double* __restrict__ r, double* __restrict__ p,
                                                         int drift, const int32_t* __restrict__ status) {
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (i >= n) return;
  const int u = atom_unit[i];
  const double e = status && status[u] != 0 ? 0.0 : field[u];  // flagged units feel no cavity force
  for (int g = 0; g < 3; ++g) {
    const double pn = p[i * 3 + g] + 0.5 * dt * (f[i * 3 + g] - e * zp[i * 3 + g]);
    p[i * 3 + g] = pn;
    if (drift) r[i * 3 + g] += dt * pn * inv_mass[i];
  }
}

// p_m -= dt/2 lambda omega F_m ; optionally exact rotation by omega dt
__global__ __launch_bounds__(kNT) void photon_kernel(int nm, const double* __restrict__ omega,
                                                     const double* __restrict__ lam, const double* __restrict__ F,
                                                     double dt, double* __restrict__ pm, int rotate,
                                                     double* __restrict__ qm) {
  const int m = blockIdx.x * kNT + threadIdx.x;
  if (m >= nm) return;
  const double w = omega[m];
  double p = pm[m] - 0.5 * dt * lam[m] * w * F[m];
  if (rotate) {
    const double q = qm[m];
    const double c = cos(w * dt), s = sin(w * dt);
    qm[m] = q * c + p * s / w;
    p = p * c - w * q * s;
  }
  pm[m] = p;
}

// kinetic energy and the temperature term of unit u: 2 (K - K_com) / (dof k_B)
__device__ inline void unit_kinetic(int u, const int32_t* __restrict__ uoff, const double* __restrict__ mass,
                                    const double* __restrict__ p, double& ke, double& tterm) {
  const int a0 = uoff[u], a1 = uoff[u + 1];
  double pc[3] = {0.0, 0.0, 0.0}, mt = 0.0, k2 = 0.0;
  for (int a = a0; a < a1; ++a) {
    mt += mass[a];
    for (int g = 0; g < 3; ++g) {
      pc[g] += p[a * 3 + g];
      k2 += p[a * 3 + g] * p[a * 3 + g] / (2.0 * mass[a]);
    }
  }
  ke = k2;
  const double kcm = (pc[0] * pc[0] + pc[1] * pc[1] + pc[2] * pc[2]) / (2.0 * mt);
  const int dof = 3 * (a1 - a0) - 3;
  tterm = dof > 0 ? 2.0 * (k2 - kcm) / (dof * 3.166811563e-6) : 0.0;
}

// first pass of the step observables: workgroup b takes units, modes and jobs
// b*kNT .. b*kNT + kNT - 1 (one each per thread) and writes its fixed-order
// partial sums (kinetic, matter, photon, temperature term, flagged units, SCC
// iterations, e.mu) to part[b][0..6]
__global__ __launch_bounds__(kNT) void observables_part_kernel(int nu, int nm, const int32_t* __restrict__ uoff,
                                                               const double* __restrict__ mass,
                                                               const double* __restrict__ p,
                                                               const double* __restrict__ energy,
                                                               const double* __restrict__ qm,
                                                               const double* __restrict__ pm,
                                                               const double* __restrict__ omega,
                                                               const double* __restrict__ lam,
                                                               const double* __restrict__ F,
                                                               const double* __restrict__ mu_pol,
                                                               const int32_t* __restrict__ status,
                                                               const int32_t* __restrict__ iters, int n_jobs,
                                                               double* __restrict__ part) {
  __shared__ double red[kNT];
  const int i = blockIdx.x * kNT + threadIdx.x;
  double ke = 0.0, v = 0.0, eph = 0.0, tsum = 0.0, nbad = 0.0, its = 0.0, mus = 0.0;
  if (i < nu) {
    unit_kinetic(i, uoff, mass, p, ke, tsum);
    v = energy[i];
    nbad = status[i] != 0 ? 1.0 : 0.0;
    mus = mu_pol[i];
  }
  if (i < nm) {
    const double x = qm[i] + lam[i] * F[i] / omega[i];
    eph = 0.5 * pm[i] * pm[i] + 0.5 * omega[i] * omega[i] * x * x;
  }
  if (i < n_jobs) its = iters[i];
  const double vals[7] = {ke, v, eph, tsum, nbad, its, mus};
  for (int q = 0; q < 7; ++q) {
    const double t = wg_sum(vals[q], red);
    if (threadIdx.x == 0) part[blockIdx.x * 8 + q] = t;
  }
}

// second pass, one workgroup: totals over the n_part partial rows in a fixed
// order, written to row *obs_row of obs; the row counter then advances (one
// launch per MD step, so the same launches can be replayed from a captured graph)
__global__ __launch_bounds__(kNT) void observables_finish_kernel(int n_part, int nu, const double* __restrict__ part,
                                                                 double* __restrict__ obs,
                                                                 unsigned int* __restrict__ obs_row) {
  __shared__ double red[kNT];
  double tot[7];
  for (int q = 0; q < 7; ++q) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < n_part; b += kNT) acc += part[b * 8 + q];
    tot[q] = wg_sum(acc, red);
  }
  if (threadIdx.x == 0) {
    const unsigned int row = *obs_row;
    double* o = obs + (size_t)row * 8;
    o[0] = tot[0];
    o[1] = tot[1];
    o[2] = tot[2];
    o[3] = tot[0] + tot[1] + tot[2];
    o[4] = tot[3] / nu;
    o[5] = tot[4];
    o[6] = tot[5];
    o[7] = tot[6];
    *obs_row = row + 1u;
  }
}

// ---- real-space cavity (one photon pair per cell, coupling local in real space)
// p_n -= dt/2 eta mu_n
__global__ __launch_bounds__(kNT) void rs_photon_kick_kernel(int n, const double* __restrict__ mu_pol, double eta,
                                                             double dt, double* __restrict__ pn) {
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (i < n) pn[i] -= 0.5 * dt * eta * mu_pol[i];
}

// field felt by the nuclei of cell n: eta q_n + eta^2 mu_n / omega_0^2
__global__ __launch_bounds__(kNT) void rs_field_kernel(int n, const double* __restrict__ q,
                                                       const double* __restrict__ mu_pol, double eta, double w0,
                                                       double* __restrict__ field) {
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (i < n) field[i] = eta * q[i] + eta * eta * mu_pol[i] / (w0 * w0);
}

// z_n = sqrt(omega_0 / 2N) (q_n + i p_n / omega_0)
__global__ __launch_bounds__(kNT) void rs_pack_kernel(int n, const double* __restrict__ q,
                                                      const double* __restrict__ pn, double w0,
                                                      double2* __restrict__ z) {
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (i >= n) return;
  const double s = sqrt(w0 / (2.0 * n));
  z[i] = make_double2(s * q[i], s * pn[i] / w0);
}

// a_k -> (q_k, p_k), exact rotation by omega_k dt, optional record of q_k, and
// c_k = sqrt(omega_k / 2N) (q_k + i p_k / omega_k) for the inverse transform
__global__ __launch_bounds__(kNT) void rs_kspace_kernel(int n, const double* __restrict__ wk, double dt,
                                                        double2* __restrict__ a, double* __restrict__ qk_out,
                                                        double* __restrict__ pk_out, double* __restrict__ qk_rec) {
  const int k = blockIdx.x * kNT + threadIdx.x;
  if (k >= n) return;
  const double w = wk[k];
  const double2 v = a[k];
  const double q0 = 2.0 * v.x / sqrt(2.0 * w), p0 = sqrt(2.0 * w) * v.y;
  const double c = cos(w * dt), s = sin(w * dt);
  const double q = q0 * c + p0 * s / w, p = p0 * c - w * q0 * s;
  if (qk_out) qk_out[k] = q;
  if (pk_out) pk_out[k] = p;
  if (qk_rec) qk_rec[k] = q;
  const double sc = sqrt(w / (2.0 * n));
  a[k] = make_double2(sc * q, sc * p / w);
}

// a_n -> q_n = 2 Re a_n / sqrt(2 omega_0), p_n = sqrt(2 omega_0) Im a_n
__global__ __launch_bounds__(kNT) void rs_unpack_kernel(int n, const double2* __restrict__ a, double w0,
                                                        double* __restrict__ q, double* __restrict__ pn) {
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (i >= n) return;
  q[i] = 2.0 * a[i].x / sqrt(2.0 * w0);
  pn[i] = sqrt(2.0 * w0) * a[i].y;
}

// free-field thermal fluctuation in k-space, q_k = sqrt(kT) xi_k / omega_k and
// p_k = sqrt(kT) xi_{N+k}, as c_k = sqrt(omega_k / 2N) (q_k + i p_k / omega_k)
__global__ __launch_bounds__(kNT) void rs_thermal_kernel(int n, const double* __restrict__ wk, double kT,
                                                         const double* __restrict__ xi, double2* __restrict__ c) {
  const int k = blockIdx.x * kNT + threadIdx.x;
  if (k >= n) return;
  const double w = wk[k], s = sqrt(kT);
  const double q = s * xi[k] / w, p = s * xi[n + k];
  const double sc = sqrt(w / (2.0 * n));
  c[k] = make_double2(sc * q, sc * p / w);
}

// a_n -> (q_n, p_n) as in rs_unpack_kernel, added to the current values
__global__ __launch_bounds__(kNT) void rs_unpack_add_kernel(int n, const double2* __restrict__ a, double w0,
                                                            double* __restrict__ q, double* __restrict__ pn) {
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (i >= n) return;
  q[i] += 2.0 * a[i].x / sqrt(2.0 * w0);
  pn[i] += sqrt(2.0 * w0) * a[i].y;
}

// q_n = -eta mu_n / omega_0^2, p_n = 0
__global__ __launch_bounds__(kNT) void rs_init_kernel(int n, const double* __restrict__ mu_pol, double eta, double w0,
                                                      double* __restrict__ q, double* __restrict__ pn) {
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (i >= n) return;
  q[i] = -eta * mu_pol[i] / (w0 * w0);
  pn[i] = 0.0;
}

// one radix-2 Stockham stage of X_k = sum_n x_n e^{sign 2 pi i k n / N} (N a power
// of two, natural order in and out): butterflies j < N/2 with span ns
__global__ __launch_bounds__(kNT) void fft_stage_kernel(int n, int ns, double sign, const double2* __restrict__ x,
                                                        double2* __restrict__ y) {
  const int j = blockIdx.x * kNT + threadIdx.x;
  const int half = n >> 1;
  if (j >= half) return;
  const int k = j & (ns - 1);
  double sn, cs;
  sincospi(sign * (double)k / (double)ns, &sn, &cs);
  const double2 v0 = x[j], u = x[j + half];
  const double2 v1 = make_double2(u.x * cs - u.y * sn, u.x * sn + u.y * cs);
  const int d = ((j - k) << 1) + k;
  y[d] = make_double2(v0.x + v1.x, v0.y + v1.y);
  y[d + ns] = make_double2(v0.x - v1.x, v0.y - v1.y);
}

// the same transform term by term for any N: one thread per output, angle from
// the exact residue (k n) mod N
__global__ __launch_bounds__(kNT) void dft_direct_kernel(int n, double sign, const double2* __restrict__ x,
                                                         double2* __restrict__ y) {
  const int k = blockIdx.x * kNT + threadIdx.x;
  if (k >= n) return;
  double re = 0.0, im = 0.0;
  long long r = 0;  // (k m) mod n
  for (int m = 0; m < n; ++m) {
    double sn, cs;
    sincospi(sign * 2.0 * (double)r / (double)n, &sn, &cs);
    const double2 v = x[m];
    re += v.x * cs - v.y * sn;
    im += v.x * sn + v.y * cs;
    r += k;
    if (r >= n) r -= n;
  }
  y[k] = make_double2(re, im);
}

// first pass of the observables of the real-space scheme (same partial rows as
// observables_part_kernel), the photon term of cell n being its free part in
// k-space, (p_k^2 + omega_k^2 q_k^2)/2 at k = n, plus the local coupling and the
// dipole self-energy of cell n
__global__ __launch_bounds__(kNT) void rs_observables_part_kernel(int nu, const int32_t* __restrict__ uoff,
                                                                  const double* __restrict__ mass,
                                                                  const double* __restrict__ p,
                                                                  const double* __restrict__ energy,
                                                                  const double* __restrict__ q,
                                                                  const double* __restrict__ mu_pol,
                                                                  const double* __restrict__ qk,
                                                                  const double* __restrict__ pk,
                                                                  const double* __restrict__ wk, double eta, double w0,
                                                                  const int32_t* __restrict__ status,
                                                                  const int32_t* __restrict__ iters,
                                                                  double* __restrict__ part) {
  __shared__ double red[kNT];
  const int u = blockIdx.x * kNT + threadIdx.x;
  double ke = 0.0, v = 0.0, eph = 0.0, tsum = 0.0, nbad = 0.0, its = 0.0, mus = 0.0;
  if (u < nu) {
    unit_kinetic(u, uoff, mass, p, ke, tsum);
    v = energy[u];
    nbad = status[u] != 0 ? 1.0 : 0.0;
    its = iters[u];
    mus = mu_pol[u];
    eph = 0.5 * (pk[u] * pk[u] + wk[u] * wk[u] * qk[u] * qk[u]) + eta * q[u] * mu_pol[u] +
          eta * eta * mu_pol[u] * mu_pol[u] / (2.0 * w0 * w0);
  }
  const double vals[7] = {ke, v, eph, tsum, nbad, its, mus};
  for (int c = 0; c < 7; ++c) {
    const double t = wg_sum(vals[c], red);
    if (threadIdx.x == 0) part[blockIdx.x * 8 + c] = t;
  }
}

__global__ void set_u32_kernel(unsigned int* c, unsigned int v) {
  if (threadIdx.x == 0) c[0] = v;
}

inline int nblk(int n) { return (n + kNT - 1) / kNT; }

}  // namespace

hipError_t launch_mu_pol(const double* dipole, const double pol[3], int n_units, const int32_t* status,
                         double* mu_pol, hipStream_t s) {
  if (n_units <= 0) return hipSuccess;
  hipLaunchKernelGGL(mu_pol_kernel, dim3(nblk(n_units)), dim3(kNT), 0, s, dipole, pol[0], pol[1], pol[2], n_units,
                     status, mu_pol);
  return hipGetLastError();
}

hipError_t launch_cav_scatter(const CavArgs& c, const double* mu_pol, double* F, double* fq, hipStream_t s) {
  if (c.n_modes <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_kernel, dim3(c.n_modes), dim3(kNT), 0, s, c, mu_pol, F, fq);
  return hipGetLastError();
}

hipError_t launch_cav_gather(const CavArgs& c, const double* q, const double* F, double* field, hipStream_t s) {
  if (c.n_units <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3((c.n_units + kNT / 64 - 1) / (kNT / 64)), dim3(kNT), 0, s, c, q, F, field);
  return hipGetLastError();
}

hipError_t launch_init_photons(const CavArgs& c, const double* F, double* qm, double* pm, hipStream_t s) {
  if (c.n_modes <= 0) return hipSuccess;
  hipLaunchKernelGGL(init_photons_kernel, dim3(nblk(c.n_modes)), dim3(kNT), 0, s, c, F, qm, pm);
  return hipGetLastError();
}

hipError_t launch_photon_thermal(const CavArgs& c, double kT, const double* xi, double* qm, double* pm,
                                 hipStream_t s) {
  if (c.n_modes <= 0) return hipSuccess;
  hipLaunchKernelGGL(photon_thermal_kernel, dim3(nblk(c.n_modes)), dim3(kNT), 0, s, c.n_modes, c.omega, kT, xi, qm,
                     pm);
  return hipGetLastError();
}

hipError_t launch_born_mulliken(const double* charges, int n_atoms, double* born, hipStream_t s) {
  hipLaunchKernelGGL(born_mulliken_kernel, dim3(nblk(n_atoms)), dim3(kNT), 0, s, charges, n_atoms, born);
  return hipGetLastError();
}

hipError_t launch_zpol_mulliken(const double* charges, const double pol[3], int n_atoms, double* zpol,
                                hipStream_t s) {
  hipLaunchKernelGGL(zpol_mulliken_kernel, dim3(nblk(n_atoms)), dim3(kNT), 0, s, charges, pol[0], pol[1], pol[2],
                     n_atoms, zpol);
  return hipGetLastError();
}

hipError_t launch_born_fd_assemble(const int32_t* unit_off, const int32_t* fd_unit, const int32_t* fd_job0,
                                   int n_fd_units, const double* mu_job, double h, const double pol[3],
                                   const int32_t* job_status, const int32_t* unit_mask, double* born, double* zpol,
                                   int32_t* status, hipStream_t s) {
  if (n_fd_units <= 0) return hipSuccess;
  hipLaunchKernelGGL(born_fd_kernel, dim3(n_fd_units), dim3(256), 0, s, unit_off, fd_unit, fd_job0, n_fd_units,
                     mu_job, h, pol[0], pol[1], pol[2], unit_mask, born, zpol);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (status && job_status) {
    hipLaunchKernelGGL(born_fd_status_kernel, dim3(nblk(n_fd_units)), dim3(kNT), 0, s, unit_off, fd_unit, fd_job0,
                       n_fd_units, job_status, unit_mask, 6, status);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_born_fd_forward_assemble(const int32_t* unit_off, const int32_t* fd_unit, const int32_t* fd_job0,
                                           int n_fd_units, const double* mu_job, const double* dipole, double h,
                                           const double pol[3], const int32_t* job_status, double* born,
                                           double* zpol, int32_t* status, hipStream_t s) {
  if (n_fd_units <= 0) return hipSuccess;
  hipLaunchKernelGGL(born_fd_forward_kernel, dim3(n_fd_units), dim3(256), 0, s, unit_off, fd_unit, fd_job0,
                     n_fd_units, mu_job, dipole, h, pol[0], pol[1], pol[2], born, zpol);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (status && job_status) {
    hipLaunchKernelGGL(born_fd_status_kernel, dim3(nblk(n_fd_units)), dim3(kNT), 0, s, unit_off, fd_unit, fd_job0,
                       n_fd_units, job_status, nullptr, 3, status);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_born_field_assemble(int n_atoms, const int32_t* atom_unit, const int32_t* unit_off,
                                      const double* f_job, double e, const double pol[3], const int32_t* f_status,
                                      const int32_t* unit_mask, double* born, double* zpol, int32_t* status,
                                      hipStream_t s) {
  hipLaunchKernelGGL(born_field_kernel, dim3(nblk(n_atoms)), dim3(kNT), 0, s, n_atoms, atom_unit, unit_off, f_job, e,
                     pol[0], pol[1], pol[2], f_status, unit_mask, born, zpol, status);
  return hipGetLastError();
}

hipError_t launch_kick_drift(int n_atoms, const int32_t* atom_unit, const double* inv_mass, const double* forces,
                             const double* zpol, const double* field, double dt, double* r, double* p,
                             int do_drift, const int32_t* status, hipStream_t s) {
  hipLaunchKernelGGL(kick_drift_kernel, dim3(nblk(n_atoms)), dim3(kNT), 0, s, n_atoms, atom_unit, inv_mass, forces,
                     zpol, field, dt, r, p, do_drift, status);
  return hipGetLastError();
}

hipError_t launch_photon_kick(int n_modes, const double* omega, const double* lam, const double* F, double dt,
                              double* pm, int rotate, double* qm, hipStream_t s) {
  if (n_modes <= 0) return hipSuccess;
  hipLaunchKernelGGL(photon_kernel, dim3(nblk(n_modes)), dim3(kNT), 0, s, n_modes, omega, lam, F, dt, pm, rotate,
                     qm);
  return hipGetLastError();
}

int observables_part_rows(int n) { return nblk(n > 0 ? n : 1); }

hipError_t launch_observables(int n_units, int n_atoms, int n_modes, const int32_t* unit_off, const double* mass,
                              const double* p, const double* energy, const double* qm, const double* pm,
                              const double* omega, const double* lam, const double* F, const double* mu_pol,
                              const int32_t* status, const int32_t* job_iters, int n_jobs, double* part,
                              int part_rows, double* obs, unsigned int* obs_row, hipStream_t s) {
  (void)n_atoms;
  const int g = observables_part_rows(std::max(n_units, std::max(n_modes, n_jobs)));
  if (g > part_rows) return hipErrorInvalidValue;
  hipLaunchKernelGGL(observables_part_kernel, dim3(g), dim3(kNT), 0, s, n_units, n_modes, unit_off, mass, p, energy,
                     qm, pm, omega, lam, F, mu_pol, status, job_iters, n_jobs, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(observables_finish_kernel, dim3(1), dim3(kNT), 0, s, g, n_units, part, obs, obs_row);
  return hipGetLastError();
}

// job order of the next MD evaluation of a bucket: the units of `order` sorted by
// the cost of their last evaluation, iterations x cost_scale = (orbitals / nmax)^3, largest
// first (longest-processing-time order for the device job queue).  One
// workgroup: a 256-bin histogram, bin starts, then a scatter by LDS atomics
// (order within a bin is immaterial: every unit's result is independent of
// when it runs).
__global__ __launch_bounds__(1024) void order_by_cost_kernel(int n, const int32_t* __restrict__ order,
                                                            const int32_t* __restrict__ iters,
                                                            const float* __restrict__ cost_scale,
                                                            int32_t* __restrict__ out) {
  __shared__ int cnt[256];
  __shared__ int start[256];
  const int tid = threadIdx.x;
  for (int b = tid; b < 256; b += 1024) cnt[b] = 0;
  __syncthreads();
  auto bin = [&](int j) {
    const float cost = (float)iters[j] * cost_scale[order[j]];  // iterations at the bucket's nmax orbitals
    const int k = (int)(cost * 2.5f);
    return k < 0 ? 0 : (k > 255 ? 255 : k);
  };
  for (int j = tid; j < n; j += 1024) atomicAdd(&cnt[bin(j)], 1);
  __syncthreads();
  if (tid == 0) {
    int s = 0;
    for (int k = 255; k >= 0; --k) {
      start[k] = s;
      s += cnt[k];
    }
  }
  __syncthreads();
  for (int j = tid; j < n; j += 1024) out[atomicAdd(&start[bin(j)], 1)] = order[j];
}

__global__ __launch_bounds__(kNT) void copy_i32_kernel(int n, const int32_t* __restrict__ src,
                                                       int32_t* __restrict__ dst) {
  const int i = blockIdx.x * kNT + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t launch_order_by_cost(int n, int32_t* order, const int32_t* iters, const float* cost_scale, int32_t* tmp,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(order_by_cost_kernel, dim3(1), dim3(1024), 0, s, n, order, iters, cost_scale, tmp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(copy_i32_kernel, dim3(nblk(n)), dim3(kNT), 0, s, n, tmp, order);
  return hipGetLastError();
}

hipError_t launch_set_u32(unsigned int* c, unsigned int v, hipStream_t s) {
  hipLaunchKernelGGL(set_u32_kernel, dim3(1), dim3(64), 0, s, c, v);
  return hipGetLastError();
}

hipError_t launch_rs_photon_kick(int n, const double* mu_pol, double eta, double dt, double* pn, hipStream_t s) {
  hipLaunchKernelGGL(rs_photon_kick_kernel, dim3(nblk(n)), dim3(kNT), 0, s, n, mu_pol, eta, dt, pn);
  return hipGetLastError();
}

hipError_t launch_rs_field(int n, const double* q, const double* mu_pol, double eta, double w0, double* field,
                           hipStream_t s) {
  hipLaunchKernelGGL(rs_field_kernel, dim3(nblk(n)), dim3(kNT), 0, s, n, q, mu_pol, eta, w0, field);
  return hipGetLastError();
}

hipError_t launch_rs_init(int n, const double* mu_pol, double eta, double w0, double* q, double* pn, hipStream_t s) {
  hipLaunchKernelGGL(rs_init_kernel, dim3(nblk(n)), dim3(kNT), 0, s, n, mu_pol, eta, w0, q, pn);
  return hipGetLastError();
}

// X = sum_m x_m e^{sign 2 pi i k m / n} into one of buf0 / buf1 (returned); x may
// alias buf0.  Powers of two by Stockham stages, any other n term by term.
hipError_t launch_dft(int n, double sign, const double2* x, double2* buf0, double2* buf1, double2** result,
                      hipStream_t s) {
  if ((n & (n - 1)) != 0) {
    hipLaunchKernelGGL(dft_direct_kernel, dim3(nblk(n)), dim3(kNT), 0, s, n, sign, x, buf1);
    *result = buf1;
    return hipGetLastError();
  }
  const double2* src = x;
  double2* dst = (x == buf1) ? buf0 : buf1;
  if (n == 1) {
    *result = const_cast<double2*>(x);
    return hipSuccess;
  }
  for (int ns = 1; ns < n; ns <<= 1) {
    hipLaunchKernelGGL(fft_stage_kernel, dim3(nblk(n / 2)), dim3(kNT), 0, s, n, ns, sign, src, dst);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    src = dst;
    dst = (dst == buf1) ? buf0 : buf1;
  }
  *result = const_cast<double2*>(src);
  return hipSuccess;
}

hipError_t launch_rs_thermal(int n, const double* wk, double w0, double kT, const double* xi, double* q, double* pn,
                             double2* buf0, double2* buf1, hipStream_t s) {
  hipLaunchKernelGGL(rs_thermal_kernel, dim3(nblk(n)), dim3(kNT), 0, s, n, wk, kT, xi, buf0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double2* b = nullptr;
  e = launch_dft(n, 1.0, buf0, buf0, buf1, &b, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rs_unpack_add_kernel, dim3(nblk(n)), dim3(kNT), 0, s, n, b, w0, q, pn);
  return hipGetLastError();
}

hipError_t launch_rs_photon_step(int n, const double* wk, double w0, double dt, double* q, double* pn,
                                 double2* buf0, double2* buf1, double* qk, double* pk, double* qk_rec,
                                 hipStream_t s) {
  hipLaunchKernelGGL(rs_pack_kernel, dim3(nblk(n)), dim3(kNT), 0, s, n, q, pn, w0, buf0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double2* a = nullptr;
  e = launch_dft(n, -1.0, buf0, buf0, buf1, &a, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rs_kspace_kernel, dim3(nblk(n)), dim3(kNT), 0, s, n, wk, dt, a, qk, pk, qk_rec);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  double2* b = nullptr;
  e = launch_dft(n, 1.0, a, a == buf0 ? buf0 : buf1, a == buf0 ? buf1 : buf0, &b, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rs_unpack_kernel, dim3(nblk(n)), dim3(kNT), 0, s, n, b, w0, q, pn);
  return hipGetLastError();
}

hipError_t launch_rs_observables(int n_units, const int32_t* unit_off, const double* mass, const double* p,
                                 const double* energy, const double* q, const double* mu_pol, const double* qk,
                                 const double* pk, const double* wk, double eta, double w0, const int32_t* status,
                                 const int32_t* job_iters, double* part, int part_rows, double* obs,
                                 unsigned int* obs_row, hipStream_t s) {
  const int g = observables_part_rows(n_units);
  if (g > part_rows) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rs_observables_part_kernel, dim3(g), dim3(kNT), 0, s, n_units, unit_off, mass, p, energy, q,
                     mu_pol, qk, pk, wk, eta, w0, status, job_iters, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(observables_finish_kernel, dim3(1), dim3(kNT), 0, s, g, n_units, part, obs, obs_row);
  return hipGetLastError();
}

}  // namespace cavdftb
