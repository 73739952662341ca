"""Real-space / reciprocal-space photon propagation of the paper (oracle).

Test infrastructure: plain numpy, written from the paper's Theory section and
its propagation Steps 1-4; only tests/ and the benchmark's CPU leg use it.

One photon coordinate pair (q_n, p_n) per cell n = 0..N-1, cells at R_n = n a.
With the coupling taken at omega_0 for every k, the light-matter Hamiltonian is
local in real space (Eq. hlm3): each cell carries eta q_n mu_n plus the dipole
self-energy eta^2 mu_n^2 / (2 omega_0^2), mu_n = e . mu of the cell.  Forces
(Eq. dpj):
    nuclear  F_nj = -grad V_n - (eta q_n + eta^2 mu_n / omega_0^2) e . Z_nj
    photon   F_n  = -eta mu_n        (the free photon part is done in k-space)
One MD step (Steps 1-4):
  1. p_n += dt/2 F_n(t); nuclear velocity Verlet with q_n(t) held fixed in both
     half-kicks; p_n += dt/2 F_n(t + dt);
  2. a_k = sum_n sqrt(omega_0 / 2N) (q_n + i p_n / omega_0) e^{-i k R_n},
     q_k = (a_k + a_k*) / sqrt(2 omega_k),  p_k = i sqrt(omega_k / 2) (a_k* - a_k);
  3. exact rotation of (q_k, p_k) by omega_k dt (Eq. qknk);
  4. a_n = sum_k sqrt(omega_k / 2N) (q_k + i p_k / omega_k) e^{i k R_n},
     q_n = (a_n + a_n*) / sqrt(2 omega_0),  p_n = i sqrt(omega_0 / 2) (a_n* - a_n).
k = 2 pi j / (N a) on the symmetric grid j = -floor((N-1)/2) .. floor(N/2) (the
DFT index j mod N), dispersion omega_k = c sqrt((pi / L)^2 + k^2) with
omega_0 = c pi / L the k = 0 frequency (Theory).  The sums of Steps 2 and 4 are
discrete Fourier transforms (numpy's FFT serves as that step).

Photon start: q_n = -eta mu_n / omega_0^2, p_n = 0 (the minimum of the local
term at frozen matter).  A thermal start adds the Boltzmann fluctuation of the
free field at temperature T: q_k = sqrt(kT) xi_k / omega_k, p_k = sqrt(kT) xi'_k
(standard normal draws passed in), carried to real space by Step 4's transform.

Pinned by (tests/test_oracle_realspace.py): Steps 2 -> 4 with no rotation is the
identity in both directions; Parseval for a flat dispersion; one cell with
harmonic matter has the normal modes of its 2 x 2 mass-weighted Hessian; free
photons (eta = 0) rotate exactly with omega_k; the k = 0 polariton splitting of
harmonic cells is linear in eta; a thermal start has kT/2 per quadratic term.
"""
import numpy as np


def k_grid(n_cells, cell_a):
    """In-plane wavevectors by DFT index: k[idx] = 2 pi j / (N a), j = idx or idx - N."""
    idx = np.arange(n_cells)
    j = np.where(idx <= n_cells // 2, idx, idx - n_cells)
    return 2.0 * np.pi * j / (n_cells * cell_a)


def dispersion(n_cells, omega0, c, cell_a):
    """omega_k = sqrt(omega_0^2 + c^2 k^2) (= c sqrt((pi/L)^2 + k^2), omega_0 = c pi / L)."""
    k = k_grid(n_cells, cell_a)
    return np.sqrt(omega0 ** 2 + (c * k) ** 2)


def to_kspace(q, p, omega0, omega_k):
    N = len(q)
    a = np.fft.fft(np.sqrt(omega0 / (2.0 * N)) * (q + 1j * p / omega0))  # sum_n ... e^{-2 pi i j n / N}
    return 2.0 * a.real / np.sqrt(2.0 * omega_k), np.sqrt(2.0 * omega_k) * a.imag


def to_realspace(qk, pk, omega0, omega_k):
    N = len(qk)
    c = np.sqrt(omega_k / (2.0 * N)) * (qk + 1j * pk / omega_k)
    a = N * np.fft.ifft(c)  # sum_k ... e^{+2 pi i j n / N}
    return 2.0 * a.real / np.sqrt(2.0 * omega0), np.sqrt(2.0 * omega0) * a.imag


class RealSpaceCavity:
    def __init__(self, eta, omega0, omega_k, pol):
        self.eta = float(eta)
        self.omega0 = float(omega0)
        self.omega_k = np.asarray(omega_k, dtype=np.float64)
        self.pol = np.asarray(pol, dtype=np.float64)


def _zpol(Z, pol):
    return np.einsum("a,jab->jb", pol, Z)


def thermal_offset(kT, xi, omega0, omega_k):
    """Real-space (q_n, p_n) of the free-field fluctuation q_k = sqrt(kT) xi_k / omega_k,
    p_k = sqrt(kT) xi'_k, with xi of length 2N (xi[:N] for q_k, xi[N:] for p_k)."""
    N = len(omega_k)
    xi = np.asarray(xi, dtype=np.float64)
    return to_realspace(np.sqrt(kT) * xi[:N] / omega_k, np.sqrt(kT) * xi[N:2 * N], omega0, omega_k)


def init_state(backend, cav, r, p, masses, atom_unit, kT=0.0, xi=None):
    """Photons at the minimum of the local photon term at frozen matter:
    q_n = -eta mu_n / omega_0^2, p_n = 0; with xi given, plus the thermal
    free-field fluctuation at kT (thermal_offset)."""
    ev = backend.evaluate(r)
    mu = ev["mu"] @ cav.pol
    q = -cav.eta * mu / cav.omega0 ** 2
    pn = np.zeros_like(mu)
    if xi is not None:
        dq, dp = thermal_offset(kT, xi, cav.omega0, cav.omega_k)
        q, pn = q + dq, pn + dp
    return {"r": np.array(r, dtype=np.float64), "p": np.array(p, dtype=np.float64),
            "q": q, "pn": pn, "ev": ev,
            "masses": np.asarray(masses, dtype=np.float64), "atom_unit": np.asarray(atom_unit)}


def step(st, backend, cav, dt):
    eta, w0 = cav.eta, cav.omega0
    au, m = st["atom_unit"], st["masses"]
    mu = st["ev"]["mu"] @ cav.pol
    pn = st["pn"] - 0.5 * dt * eta * mu
    field = eta * st["q"] + eta ** 2 * mu / w0 ** 2
    p = st["p"] + 0.5 * dt * (st["ev"]["forces"] - field[au][:, None] * _zpol(st["ev"]["Z"], cav.pol))
    r = st["r"] + dt * p / m[:, None]
    ev = backend.evaluate(r)
    mu1 = ev["mu"] @ cav.pol
    field1 = eta * st["q"] + eta ** 2 * mu1 / w0 ** 2
    p = p + 0.5 * dt * (ev["forces"] - field1[au][:, None] * _zpol(ev["Z"], cav.pol))
    pn = pn - 0.5 * dt * eta * mu1
    qk, pk = to_kspace(st["q"], pn, w0, cav.omega_k)
    c, s = np.cos(cav.omega_k * dt), np.sin(cav.omega_k * dt)
    qk, pk = qk * c + pk * s / cav.omega_k, pk * c - cav.omega_k * qk * s
    q, pn = to_realspace(qk, pk, w0, cav.omega_k)
    st.update({"r": r, "p": p, "q": q, "pn": pn, "ev": ev, "qk": qk, "pk": pk})
    return st


def photon_energy(q, pn, mu, cav):
    """sum_k (p_k^2 + omega_k^2 q_k^2) / 2 + sum_n (eta q_n mu_n + eta^2 mu_n^2 / (2 omega_0^2))."""
    qk, pk = to_kspace(q, pn, cav.omega0, cav.omega_k)
    free = 0.5 * float(np.sum(pk ** 2 + cav.omega_k ** 2 * qk ** 2))
    return free + float(np.sum(cav.eta * q * mu + cav.eta ** 2 * mu ** 2 / (2.0 * cav.omega0 ** 2)))
