"""ctypes binding of libcavdftb (argument marshalling only).

Every method forwards to the C function of the same name in include/cavdftb.h;
torch CUDA (HIP) tensors supply device memory and the current stream.  No
arithmetic of the method happens here.  The library must be built (see
__graft_entry__.build); importing this module without it raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcavdftb.so")

OK, EINVAL, ENOMEM, EHIP = 0, -1, -2, -3
SG_NOALLOC_MAX_ROWS = 8192
ST_NOT_CONVERGED, ST_NOT_PD, ST_DEGENERATE, ST_NAN = 1, 2, 4, 8
BORN_MULLIKEN, BORN_FD, BORN_SURROGATE, BORN_FIELD, BORN_FD_FORWARD = 0, 1, 2, 3, 4
SG_N_IN, SG_N_HID, SG_N_OUT, SG_MEMBERS, SG_N_PARAM, SG_N_NORM = 80, 128, 9, 4, 28041, 178
N_OBS = 8
WORK_MU_POL, WORK_DIPOLE, WORK_ENERGY, WORK_CHARGES, WORK_FORCES, WORK_FIELD = range(6)
EIG_AUTO, EIG_FULL, EIG_JACOBI = 0, 1, 2
BUCKETS = (8, 16, 32, 48, 64, 96, 128, 192)
OBS_NAMES = ("kinetic", "potential", "photon", "total", "temperature", "n_bad_units", "scc_iterations",
             "sum_mu_pol")

_c_d = ctypes.c_double
_c_i32 = ctypes.c_int32
_vp = ctypes.c_void_p


class Params(ctypes.Structure):
    _fields_ = [("sk", (_c_d * 4) * 7), ("onsite", (_c_d * 2) * 2), ("hubbard_u", _c_d * 2), ("q0", _c_d * 2),
                ("rep_a", _c_d * 3), ("rep_alpha", _c_d * 3), ("mass", _c_d * 2)]


class Layout(ctypes.Structure):
    _fields_ = [("n_units", _c_i32), ("n_atoms", _c_i32), ("n_modes", _c_i32), ("unit_atom_off", _vp),
                ("species", _vp), ("unit_x", _vp), ("omega", _vp), ("k", _vp), ("theta", _vp), ("lam", _vp),
                ("pol", _c_d * 3)]


class Counters(ctypes.Structure):
    _fields_ = [("scc_jobs", ctypes.c_int64), ("scc_iterations", ctypes.c_int64), ("scc_flops", _c_d),
                ("scc_kernel_ms", _c_d), ("scc_launches", ctypes.c_int64), ("jacobi_sweeps", ctypes.c_int64),
                ("surrogate_fallback_units", ctypes.c_int64), ("jacobi_iterations", ctypes.c_int64),
                ("graph_replays", ctypes.c_int64), ("graph_captures", ctypes.c_int64),
                ("tridiagonal_solves", ctypes.c_int64), ("tridiagonal_fallbacks", ctypes.c_int64)]


SYMBOLS = {
    "cavdftb_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(Layout), _vp, ctypes.POINTER(_vp)]),
    "cavdftb_destroy": (ctypes.c_int, [_vp]),
    "cavdftb_set_scc": (ctypes.c_int, [_vp, _c_d, _c_i32, _c_d]),
    "cavdftb_set_tuning": (ctypes.c_int, [_vp, _c_d, _c_i32]),
    "cavdftb_set_warm_start": (ctypes.c_int, [_vp, _c_i32]),
    "cavdftb_reset_warm_start": (ctypes.c_int, [_vp]),
    "cavdftb_eval_units": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cavdftb_born_charges": (ctypes.c_int, [_vp, _vp, _c_i32, _c_d, _vp, _vp, _vp]),
    "cavdftb_cavity_forces": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "cavdftb_init_photons": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "cavdftb_init_photons_thermal": (ctypes.c_int, [_vp, _vp, _vp, _vp, _c_d, _vp]),
    "cavdftb_set_surrogate": (ctypes.c_int, [_vp, _vp, _vp, _c_d]),
    "cavdftb_set_fallback": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "cavdftb_set_schedule": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32]),
    "cavdftb_set_eigensolver": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "cavdftb_set_bucket_schedule": (ctypes.c_int, [_vp, _c_i32, _c_i32, _c_i32, _c_i32]),
    "cavdftb_set_bucket_streams": (ctypes.c_int, [_vp, _c_i32]),
    "cavdftb_bucket_info": (ctypes.c_int, [_vp, _c_i32, ctypes.POINTER(_c_i32), ctypes.POINTER(_c_i32),
                                           ctypes.POINTER(_c_i32)]),
    "cavdftb_load_launch_table": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "cavdftb_set_graph": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "cavdftb_set_born_interval": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "cavdftb_set_realspace_cavity": (ctypes.c_int, [_vp, _c_d, _c_d, _c_d, _c_d]),
    "cavdftb_init_photons_realspace": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "cavdftb_init_photons_realspace_thermal": (ctypes.c_int, [_vp, _vp, _vp, _vp, _c_d, _vp]),
    "cavdftb_step_realspace": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_int32, _c_d, ctypes.c_int32, _c_d,
                                              _vp, _vp]),
    "cavdftb_read_work": (ctypes.c_int, [_vp, ctypes.c_int32, _vp]),
    "cavdftb_sg_features": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "cavdftb_sg_prep": (ctypes.c_int, [_vp, _vp, _c_i32, _c_i32, _vp, _vp, _vp]),
    "cavdftb_sg_forward": (ctypes.c_int, [_vp, _vp, _c_i32, _vp, _vp, _vp]),
    "cavdftb_sg_backward": (ctypes.c_int, [_vp, _vp, _vp, _vp, _c_i32, _vp, _vp, _vp]),
    "cavdftb_sg_backward_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _vp, _c_i32, _vp, _vp]),
    "cavdftb_sg_mse": (ctypes.c_int, [_vp, _vp, _c_i32, _vp, _vp, _vp, _vp]),
    "cavdftb_sg_adam": (ctypes.c_int, [_vp, _vp, _vp, _vp, _c_i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_float, _c_i32, _vp]),
    "cavdftb_sg_gather": (ctypes.c_int, [_vp, _vp, _c_i32, _c_i32, _vp, _vp]),
    "cavdftb_sg_moments": (ctypes.c_int, [_vp, _vp, _c_i32, _c_i32, _vp, _vp]),
    "cavdftb_sg_to_local": (ctypes.c_int, [_vp, _vp, _vp, _vp, _c_i32, _vp, _vp]),
    "cavdftb_step": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _c_i32, _c_d, _c_i32, _c_d, _vp]),
    "cavdftb_invalidate": (ctypes.c_int, [_vp]),
    "cavdftb_sync": (ctypes.c_int, [_vp, ctypes.POINTER(_c_i32)]),
    "cavdftb_enable_timing": (ctypes.c_int, [_vp, _c_i32]),
    "cavdftb_read_counters": (ctypes.c_int, [_vp, ctypes.POINTER(Counters)]),
    "cavdftb_reset_counters": (ctypes.c_int, [_vp]),
    "cavdftb_last_error": (ctypes.c_char_p, [_vp]),
    "cavdftb_version": (ctypes.c_char_p, []),
}

_lib = None


def load_library():
    """Load libcavdftb.so from the package directory (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SYMBOLS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class CavdftbError(RuntimeError):
    pass


def _ptr(t, dtype=None, numel=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (or None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise CavdftbError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise CavdftbError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise CavdftbError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise CavdftbError(f"{name} must have {numel} elements, got {t.numel()}")
    return t.data_ptr()


def params_struct(p):
    s = Params()
    for t in range(7):
        for j in range(4):
            s.sk[t][j] = float(p["sk"][t][j])
    for a in range(2):
        for b in range(2):
            s.onsite[a][b] = float(p["onsite"][a][b])
        s.hubbard_u[a] = float(p["hubbard_u"][a])
        s.q0[a] = float(p["q0"][a])
        s.mass[a] = float(p["mass"][a])
    for t in range(3):
        s.rep_a[t] = float(p["rep_a"][t])
        s.rep_alpha[t] = float(p["rep_alpha"][t])
    return s


class Context:
    """A library context for one batch layout (units, species, cavity modes)."""

    def __init__(self, params, species, unit_off, unit_x, omega, k, theta, lam, pol, stream=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        self._host = {
            "unit_off": np.ascontiguousarray(unit_off, dtype=np.int32),
            "species": np.ascontiguousarray(species, dtype=np.int8),
            "unit_x": np.ascontiguousarray(unit_x, dtype=np.float64),
            "omega": np.ascontiguousarray(omega, dtype=np.float64),
            "k": np.ascontiguousarray(k, dtype=np.float64),
            "theta": np.ascontiguousarray(theta, dtype=np.float64),
            "lam": np.ascontiguousarray(lam, dtype=np.float64),
        }
        h = self._host
        self.n_units = len(h["unit_off"]) - 1
        self.n_atoms = int(h["unit_off"][-1])
        self.n_modes = len(h["omega"])
        L = Layout()
        L.n_units, L.n_atoms, L.n_modes = self.n_units, self.n_atoms, self.n_modes
        for key in ("unit_off", "species", "unit_x", "omega", "k", "theta", "lam"):
            setattr(L, "unit_atom_off" if key == "unit_off" else key, h[key].ctypes.data)
        for g in range(3):
            L.pol[g] = float(pol[g])
        self.stream = torch.cuda.current_stream() if stream is None else stream
        P = params_struct(params)
        out = _vp()
        rc = self.lib.cavdftb_create(ctypes.byref(P), ctypes.byref(L), _vp(self.stream.cuda_stream), ctypes.byref(out))
        if rc != OK:
            raise CavdftbError(f"cavdftb_create failed with code {rc}")
        self.ctx = out

    def _check(self, rc, what):
        if rc != OK:
            msg = self.lib.cavdftb_last_error(self.ctx)
            raise CavdftbError(f"{what} failed ({rc}): {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.cavdftb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- entry points (same names as the C ABI without the prefix)
    def set_scc(self, tol, max_iter=200, mix_alpha=0.6):
        self._check(self.lib.cavdftb_set_scc(self.ctx, float(tol), int(max_iter), float(mix_alpha)), "set_scc")

    def set_tuning(self, jacobi_res_factor=1e-3, keep_mixer_history=True):
        self._check(self.lib.cavdftb_set_tuning(self.ctx, float(jacobi_res_factor), int(bool(keep_mixer_history))),
                    "set_tuning")

    def set_schedule(self, job_queue=True, max_wg_per_cu=0):
        self._check(self.lib.cavdftb_set_schedule(self.ctx, int(bool(job_queue)), int(max_wg_per_cu)), "set_schedule")

    def set_eigensolver(self, mode):
        self._check(self.lib.cavdftb_set_eigensolver(self.ctx, int(mode)), "set_eigensolver")

    def set_bucket_schedule(self, bucket, wg_per_cu=0, eig_mode=-1, job_queue=-1):
        self._check(self.lib.cavdftb_set_bucket_schedule(self.ctx, int(bucket), int(wg_per_cu), int(eig_mode),
                                                         int(job_queue)), "set_bucket_schedule")

    def set_bucket_streams(self, n_streams):
        self._check(self.lib.cavdftb_set_bucket_streams(self.ctx, int(n_streams)), "set_bucket_streams")

    def bucket_info(self, bucket):
        """(units, largest resident workgroups per CU, current) of one orbital bucket."""
        nu, mx, cur = _c_i32(), _c_i32(), _c_i32()
        self._check(self.lib.cavdftb_bucket_info(self.ctx, int(bucket), ctypes.byref(nu), ctypes.byref(mx),
                                                 ctypes.byref(cur)), "bucket_info")
        return nu.value, mx.value, cur.value

    def load_launch_table(self, path):
        """Entries applied (the library reads and parses the file)."""
        rc = self.lib.cavdftb_load_launch_table(self.ctx, os.fsencode(path))
        if rc < 0:
            self._check(rc, "load_launch_table")
        return rc

    def read_work(self, which, dst):
        """Device copy of a work array (WORK_MU_POL ... WORK_FIELD) into dst."""
        sizes = {WORK_MU_POL: self.n_units, WORK_DIPOLE: 3 * self.n_units, WORK_ENERGY: self.n_units,
                 WORK_CHARGES: self.n_atoms, WORK_FORCES: 3 * self.n_atoms, WORK_FIELD: self.n_units}
        if which not in sizes:
            raise CavdftbError(f"read_work: unknown array {which}")
        self._check(self.lib.cavdftb_read_work(self.ctx, int(which), _ptr(dst, self.torch.float64, sizes[which], "dst")),
                    "read_work")

    def set_realspace_cavity(self, eta, omega0, c_medium, cell_a):
        self._check(self.lib.cavdftb_set_realspace_cavity(self.ctx, float(eta), float(omega0), float(c_medium),
                                                          float(cell_a)), "set_realspace_cavity")

    def init_photons_realspace(self, r, qn, pn):
        t = self.torch
        U = self.n_units
        self._check(self.lib.cavdftb_init_photons_realspace(
            self.ctx, _ptr(r, t.float64, self.n_atoms * 3, "r"), _ptr(qn, t.float64, U, "qn"),
            _ptr(pn, t.float64, U, "pn")), "init_photons_realspace")

    def init_photons_realspace_thermal(self, r, qn, pn, kT, xi):
        """xi: device [2 n_units] standard normal draws (q_k first, then p_k)."""
        t = self.torch
        U = self.n_units
        self._check(self.lib.cavdftb_init_photons_realspace_thermal(
            self.ctx, _ptr(r, t.float64, self.n_atoms * 3, "r"), _ptr(qn, t.float64, U, "qn"),
            _ptr(pn, t.float64, U, "pn"), float(kT), _ptr(xi, t.float64, 2 * U, "xi")),
            "init_photons_realspace_thermal")

    def step_realspace(self, r, p, qn, pn, n_steps, dt, born_mode=BORN_MULLIKEN, h_fd=1e-3, obs=None, qk_record=None):
        t = self.torch
        NA, U = self.n_atoms, self.n_units
        self._check(self.lib.cavdftb_step_realspace(
            self.ctx, _ptr(r, t.float64, NA * 3, "r"), _ptr(p, t.float64, NA * 3, "p"), _ptr(qn, t.float64, U, "qn"),
            _ptr(pn, t.float64, U, "pn"), int(n_steps), float(dt), int(born_mode), float(h_fd),
            _ptr(obs, t.float64, int(n_steps) * N_OBS, "obs"),
            _ptr(qk_record, t.float64, int(n_steps) * U, "qk_record")), "step_realspace")

    def set_born_interval(self, every):
        self._check(self.lib.cavdftb_set_born_interval(self.ctx, int(every)), "set_born_interval")

    def set_graph(self, enable=True):
        self._check(self.lib.cavdftb_set_graph(self.ctx, int(bool(enable))), "set_graph")

    def set_warm_start(self, enable):
        self._check(self.lib.cavdftb_set_warm_start(self.ctx, int(bool(enable))), "set_warm_start")

    def reset_warm_start(self):
        self._check(self.lib.cavdftb_reset_warm_start(self.ctx), "reset_warm_start")

    def eval_units(self, pos, energy=None, forces=None, charges=None, dipole=None, unit_status=None):
        t = self.torch
        U, NA = self.n_units, self.n_atoms
        self._check(self.lib.cavdftb_eval_units(
            self.ctx, _ptr(pos, t.float64, NA * 3, "pos"), _ptr(energy, t.float64, U, "energy"),
            _ptr(forces, t.float64, NA * 3, "forces"), _ptr(charges, t.float64, NA, "charges"),
            _ptr(dipole, t.float64, U * 3, "dipole"), _ptr(unit_status, t.int32, U, "unit_status")), "eval_units")

    def born_charges(self, pos, mode, h, born, unit_status=None, ens_std=None):
        t = self.torch
        self._check(self.lib.cavdftb_born_charges(
            self.ctx, _ptr(pos, t.float64, self.n_atoms * 3, "pos"), int(mode), float(h),
            _ptr(born, t.float64, self.n_atoms * 9, "born"), _ptr(ens_std, t.float64, self.n_atoms, "ens_std"),
            _ptr(unit_status, t.int32, self.n_units, "unit_status")), "born_charges")

    def set_surrogate(self, params, norm, std_threshold=0.05):
        t = self.torch
        self._check(self.lib.cavdftb_set_surrogate(
            self.ctx, _ptr(params, t.float32, 2 * SG_MEMBERS * SG_N_PARAM, "params"),
            _ptr(norm, t.float32, 2 * SG_N_NORM, "norm"), float(std_threshold)), "set_surrogate")

    def set_fallback(self, mode):
        self._check(self.lib.cavdftb_set_fallback(self.ctx, int(mode)), "set_fallback")

    def sg_features(self, pos, feat=None, frames=None):
        t = self.torch
        self._check(self.lib.cavdftb_sg_features(
            self.ctx, _ptr(pos, t.float64, self.n_atoms * 3, "pos"),
            _ptr(feat, t.float64, self.n_atoms * SG_N_IN, "feat"),
            _ptr(frames, t.float64, self.n_atoms * 9, "frames")), "sg_features")

    def cavity_forces(self, mu_pol, q, F=None, field=None, fq=None):
        t = self.torch
        U, M = self.n_units, self.n_modes
        self._check(self.lib.cavdftb_cavity_forces(
            self.ctx, _ptr(mu_pol, t.float64, U, "mu_pol"), _ptr(q, t.float64, M, "q"), _ptr(F, t.float64, M, "F"),
            _ptr(field, t.float64, U, "field"), _ptr(fq, t.float64, M, "fq")), "cavity_forces")

    def init_photons(self, r, qm, pm):
        t = self.torch
        self._check(self.lib.cavdftb_init_photons(
            self.ctx, _ptr(r, t.float64, self.n_atoms * 3, "r"), _ptr(qm, t.float64, self.n_modes, "qm"),
            _ptr(pm, t.float64, self.n_modes, "pm")), "init_photons")

    def init_photons_thermal(self, r, qm, pm, kT, xi):
        """xi: device [2 n_modes] standard normal draws (q first, then p)."""
        t = self.torch
        self._check(self.lib.cavdftb_init_photons_thermal(
            self.ctx, _ptr(r, t.float64, self.n_atoms * 3, "r"), _ptr(qm, t.float64, self.n_modes, "qm"),
            _ptr(pm, t.float64, self.n_modes, "pm"), float(kT), _ptr(xi, t.float64, 2 * self.n_modes, "xi")),
            "init_photons_thermal")

    def step(self, r, p, qm, pm, n_steps, dt, born_mode=BORN_MULLIKEN, h_fd=1e-3, obs=None):
        t = self.torch
        NA, M = self.n_atoms, self.n_modes
        self._check(self.lib.cavdftb_step(
            self.ctx, _ptr(r, t.float64, NA * 3, "r"), _ptr(p, t.float64, NA * 3, "p"),
            _ptr(qm, t.float64, M, "qm"), _ptr(pm, t.float64, M, "pm"), int(n_steps), float(dt), int(born_mode),
            float(h_fd), _ptr(obs, t.float64, int(n_steps) * N_OBS, "obs")), "step")

    def invalidate(self):
        self._check(self.lib.cavdftb_invalidate(self.ctx), "invalidate")

    def sync(self):
        nb = _c_i32(0)
        self._check(self.lib.cavdftb_sync(self.ctx, ctypes.byref(nb)), "sync")
        return nb.value

    def enable_timing(self, enable=True):
        self._check(self.lib.cavdftb_enable_timing(self.ctx, int(bool(enable))), "enable_timing")

    def read_counters(self):
        c = Counters()
        self._check(self.lib.cavdftb_read_counters(self.ctx, ctypes.byref(c)), "read_counters")
        return {k: getattr(c, k) for k, _ in Counters._fields_}

    def reset_counters(self):
        self._check(self.lib.cavdftb_reset_counters(self.ctx), "reset_counters")


def context_from_system(params, system, stream=None):
    """Convenience constructor from a cavgen system dictionary."""
    return Context(params, system["species"], system["unit_off"], system["unit_x"], system["omega"], system["k"],
                   system["theta"], system["lam"], system["pol"], stream=stream)


# ---------------------------------------------------------------- surrogate training calls (no context)
def _stream_handle(stream):
    import torch
    st = torch.cuda.current_stream() if stream is None else stream
    return _vp(st.cuda_stream)


def _rc(rc, what):
    if rc != OK:
        raise CavdftbError(f"{what} failed ({rc})")


def sg_prep(v, idx, n, width, norm, x, stream=None):
    _rc(load_library().cavdftb_sg_prep(_ptr(v, name="v"), _ptr(idx, name="idx"), int(n), int(width),
                                       _ptr(norm, name="norm"), _ptr(x, name="x"), _stream_handle(stream)), "sg_prep")


def sg_forward(params, x, n, y, act=None, stream=None):
    _rc(load_library().cavdftb_sg_forward(_ptr(params, name="params"), _ptr(x, name="x"), int(n), _ptr(y, name="y"),
                                          _ptr(act, name="act"), _stream_handle(stream)), "sg_forward")


def sg_backward(params, x, act, dy, n, grad, work, stream=None):
    _rc(load_library().cavdftb_sg_backward(_ptr(params, name="params"), _ptr(x, name="x"), _ptr(act, name="act"),
                                           _ptr(dy, name="dy"), int(n), _ptr(grad, name="grad"),
                                           _ptr(work, name="work"), _stream_handle(stream)), "sg_backward")


def sg_backward_noalloc(params, x, act, dy, n, grad, stream=None):
    _rc(load_library().cavdftb_sg_backward_noalloc(_ptr(params, name="params"), _ptr(x, name="x"),
                                                   _ptr(act, name="act"), _ptr(dy, name="dy"), int(n),
                                                   _ptr(grad, name="grad"), _stream_handle(stream)),
        "sg_backward_noalloc")


def sg_mse(y, t, count, dy, loss, work, stream=None):
    _rc(load_library().cavdftb_sg_mse(_ptr(y, name="y"), _ptr(t, name="t"), int(count), _ptr(dy, name="dy"),
                                      _ptr(loss, name="loss"), _ptr(work, name="work"), _stream_handle(stream)),
        "sg_mse")


def sg_adam(params, grad, m, v, count, lr, beta1, beta2, eps, step, stream=None):
    _rc(load_library().cavdftb_sg_adam(_ptr(params, name="params"), _ptr(grad, name="grad"), _ptr(m, name="m"),
                                       _ptr(v, name="v"), int(count), float(lr), float(beta1), float(beta2),
                                       float(eps), int(step), _stream_handle(stream)), "sg_adam")


def sg_gather(src, idx, n, width, dst, stream=None):
    _rc(load_library().cavdftb_sg_gather(_ptr(src, name="src"), _ptr(idx, name="idx"), int(n), int(width),
                                         _ptr(dst, name="dst"), _stream_handle(stream)), "sg_gather")


def sg_moments(x, idx, n, width, out, stream=None):
    _rc(load_library().cavdftb_sg_moments(_ptr(x, name="x"), _ptr(idx, name="idx"), int(n), int(width),
                                          _ptr(out, name="out"), _stream_handle(stream)), "sg_moments")


def sg_to_local(frames, born, charges, idx, n, out, stream=None):
    _rc(load_library().cavdftb_sg_to_local(_ptr(frames, name="frames"), _ptr(born, name="born"),
                                           _ptr(charges, name="charges"), _ptr(idx, name="idx"), int(n),
                                           _ptr(out, name="out"), _stream_handle(stream)), "sg_to_local")
