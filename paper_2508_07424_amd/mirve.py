"""ctypes binding of libmirve.so (include/mirve.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  PyTorch supplies the device workspace and the stream.  The
module raises at import if the library has not been built; there is no
fallback path.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmirve.so")

RVE_OK = 0
RVE_EINVAL = -1
RVE_ENOSPC = -2
RVE_EDEVICE = -3
RVE_ENOCONV = -4
RVE_ENUMERIC = -5
RVE_ESTATE = -6
RVE_ENOTDONE = -7
RVE_NOALLOC_SCRATCH_BYTES = 64 << 20   # static device array of rve_apply_green_op_device_noalloc
_NAMES = {0: "RVE_OK", -1: "RVE_EINVAL", -2: "RVE_ENOSPC", -3: "RVE_EDEVICE", -4: "RVE_ENOCONV",
          -5: "RVE_ENUMERIC", -6: "RVE_ESTATE", -7: "RVE_ENOTDONE"}

RVE_PREC_FP64 = 0
RVE_PREC_MIXED = 1
RVE_SPLIT_NONE = 0
RVE_SPLIT_VOLDEV = 1
RVE_PRECOND_FFT = 0
RVE_PRECOND_JACOBI = 1
RVE_PHASE_ISO = 0
RVE_PHASE_CUBIC = 1
RVE_RUN_STOP_AT_FRACTURE = 1
RVE_RUN_KEEP = 2
WHY = {0: "none", 1: "stagger", 2: "cg", 3: "pcg", 4: "arclength", 5: "split", 6: "breakdown",
       7: "anderson", 8: "gmres", 9: "newton"}

FIELDS = {"phi": 0, "hist": 1, "psi_ini": 2, "eps1": 3, "sig1": 4, "psi1": 5, "phi_ini": 6}

# every function declared in include/mirve.h
EXPORTS = ["rve_default_config", "rve_query_workspace", "rve_create", "rve_destroy",
           "rve_set_microstructure", "rve_set_microstructure_slot", "rve_step_dissipation",
           "rve_step_dissipation_slots", "rve_step_dissipation_batch", "rve_batch_size",
           "rve_release_slot", "rve_effective_toughness", "rve_effective_toughness_slot",
           "rve_get_field", "rve_set_field", "rve_get_field_slot", "rve_set_field_slot",
           "rve_get_scalars", "rve_set_scalars", "rve_get_scalars_slot", "rve_set_scalars_slot",
           "rve_apply_green_op", "rve_apply_green_op_device", "rve_solve_mechanics",
           "rve_solve_damage", "rve_dissipation", "rve_profile_pass", "rve_autotune",
           "rve_last_error", "rve_version", "rve_run_slots", "rve_state_bytes", "rve_save_state",
           "rve_load_state", "rve_apply_green_op_device_noalloc", "rve_run_stats", "rve_run_budget",
           "rve_newton_default_opts", "rve_newton_workspace", "rve_step_newton",
           "rve_set_microstructure_euler"]


class rve_config(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double), ("ell", C.c_double),
                ("k_res", C.c_double), ("f", C.c_double * 6), ("split", C.c_int),
                ("history", C.c_int), ("precision", C.c_int), ("tol", C.c_double),
                ("tol_cg", C.c_double), ("tol_pcg", C.c_double), ("tol_al", C.c_double),
                ("max_stagger", C.c_int), ("max_halvings", C.c_int), ("stall_window", C.c_int),
                ("max_cg", C.c_int), ("max_pcg", C.c_int),
                ("anderson_depth", C.c_int), ("frac_threshold", C.c_double), ("A_g", C.c_double),
                ("max_materials", C.c_int), ("batch", C.c_int), ("damage_precond", C.c_int),
                ("graphs", C.c_int), ("streaming", C.c_int)]


class rve_phase(C.Structure):
    _fields_ = [("kind", C.c_int), ("E", C.c_double), ("nu", C.c_double), ("C11", C.c_double),
                ("C12", C.c_double), ("C44", C.c_double), ("Gc", C.c_double), ("beta", C.c_double),
                ("n", C.c_double * 3)]


class rve_step_info(C.Structure):
    _fields_ = [("E", C.c_double), ("Sigma", C.c_double), ("D", C.c_double),
                ("Gamma", C.c_double), ("tau", C.c_double), ("T", C.c_double),
                ("n_stagger", C.c_int), ("n_cg", C.c_int), ("n_pcg", C.c_int),
                ("n_greenop", C.c_int), ("res_R1", C.c_double), ("res_R2", C.c_double),
                ("res_R3", C.c_double), ("fractured", C.c_int), ("step", C.c_int),
                ("n_steps", C.c_int), ("n_substeps", C.c_int), ("reason", C.c_int),
                ("G_inst", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class rve_newton_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("krylov_tol", C.c_double), ("theta", C.c_double),
                ("restart", C.c_int), ("max_cycles", C.c_int), ("max_newton", C.c_int),
                ("relax", C.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmirve.so is not built; run `python -m paper_2508_07424_amd.build`")
    # torch first: the library then binds to the HIP runtime torch has
    # loaded, so that its workspaces and streams belong to the same runtime
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P, I, D, S = C.c_void_p, C.c_int, C.c_double, C.c_size_t
    dp = C.POINTER(C.c_double)
    sig = {
        "rve_default_config": (I, [C.POINTER(rve_config)]),
        "rve_query_workspace": (I, [C.POINTER(rve_config), C.POINTER(C.c_size_t)]),
        "rve_create": (I, [C.POINTER(rve_config), P, S, P, C.POINTER(P)]),
        "rve_destroy": (I, [P]),
        "rve_set_microstructure": (I, [P, P, C.POINTER(rve_phase), I, P, P, P, D]),
        "rve_set_microstructure_slot": (I, [P, I, P, C.POINTER(rve_phase), I, P, P, P, D]),
        "rve_step_dissipation_slots": (I, [P, dp, C.POINTER(rve_step_info), C.POINTER(C.c_int)]),
        "rve_run_slots": (I, [P, dp, C.POINTER(C.c_int), I, C.POINTER(rve_step_info),
                              C.POINTER(C.c_int)]),
        "rve_state_bytes": (I, [P, C.POINTER(C.c_size_t)]),
        "rve_save_state": (I, [P, I, P, S]),
        "rve_load_state": (I, [P, I, P, S]),
        "rve_batch_size": (I, [P]),
        "rve_run_stats": (I, [P, dp]),
        "rve_run_budget": (I, [P, dp, C.POINTER(C.c_int), C.c_longlong, I, C.POINTER(rve_step_info),
                               C.POINTER(C.c_int)]),
        "rve_newton_default_opts": (None, [C.POINTER(rve_newton_opts)]),
        "rve_set_microstructure_euler": (I, [P, I, P, C.POINTER(rve_phase), I, P, P, P, D]),
        "rve_newton_workspace": (I, [P, I, C.POINTER(C.c_size_t)]),
        "rve_step_newton": (I, [P, I, D, C.POINTER(rve_newton_opts), P, S, C.POINTER(rve_step_info)]),
        "rve_release_slot": (I, [P, I]),
        "rve_effective_toughness_slot": (I, [P, I, dp]),
        "rve_get_field_slot": (I, [P, I, I, dp, S]),
        "rve_set_field_slot": (I, [P, I, I, dp, S]),
        "rve_get_scalars_slot": (I, [P, I, dp]),
        "rve_set_scalars_slot": (I, [P, I, dp]),
        "rve_step_dissipation": (I, [P, D, C.POINTER(rve_step_info)]),
        "rve_step_dissipation_batch": (I, [C.POINTER(P), I, dp, C.POINTER(rve_step_info),
                                           C.POINTER(C.c_int)]),
        "rve_effective_toughness": (I, [P, dp]),
        "rve_get_field": (I, [P, I, dp, S]),
        "rve_set_field": (I, [P, I, dp, S]),
        "rve_get_scalars": (I, [P, dp]),
        "rve_set_scalars": (I, [P, dp]),
        "rve_apply_green_op": (I, [P, dp, dp]),
        "rve_apply_green_op_device": (I, [P, P, P, I]),
        "rve_apply_green_op_device_noalloc": (I, [P, P, P, I]),
        "rve_solve_mechanics": (I, [P, C.POINTER(C.c_int), dp]),
        "rve_solve_damage": (I, [P, D, dp, C.POINTER(C.c_int), I]),
        "rve_dissipation": (I, [P, dp, dp]),
        "rve_profile_pass": (I, [P, I, I, dp]),
        "rve_autotune": (I, [P, I, C.POINTER(C.c_int)]),
        "rve_last_error": (C.c_char_p, [P]),
        "rve_version": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class MirveError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_NAMES.get(code, "?"), code, msg))
        self.code = code


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def default_config():
    c = rve_config()
    lib.rve_default_config(C.byref(c))
    return c


def make_config(n, h=1.0, ell=1.5, k=1e-6, f=None, precision=RVE_PREC_FP64, **kw):
    """rve_config for grid n = (n_x, n_y[, n_z]) with the library defaults."""
    c = default_config()
    dim = len(n)
    c.dim = dim
    c.n[0], c.n[1] = int(n[0]), int(n[1])
    c.n[2] = int(n[2]) if dim == 3 else 1
    c.h, c.ell, c.k_res = float(h), float(ell), float(k)
    s = 3 if dim == 2 else 6
    ff = np.zeros(6)
    if f is None:
        ff[1] = 1.0
    else:
        ff[:s] = np.asarray(f, dtype=float)[:s]
    for i in range(6):
        c.f[i] = ff[i]
    c.precision = precision          # tolerances left at 0 take the precision's defaults
    for key, v in kw.items():
        setattr(c, key, v)
    return c


def rve_query_workspace(cfg):
    b = C.c_size_t(0)
    rc = lib.rve_query_workspace(C.byref(cfg), C.byref(b))
    if rc != RVE_OK:
        raise MirveError(rc, lib.rve_last_error(None).decode())
    return b.value


def phases_array(phases):
    arr = (rve_phase * len(phases))()
    for i, ph in enumerate(phases):
        nrm = (C.c_double * 3)(*[float(v) for v in ph.get("n", (0.0, 0.0, 1.0))])
        if ph["kind"] == "iso":
            arr[i] = rve_phase(RVE_PHASE_ISO, ph["E"], ph["nu"], 0.0, 0.0, 0.0, ph["Gc"],
                               ph.get("beta", 0.0), nrm)
        else:
            arr[i] = rve_phase(RVE_PHASE_CUBIC, 0.0, 0.0, ph["C11"], ph["C12"], ph["C44"], ph["Gc"],
                               ph.get("beta", 0.0), nrm)
    return arr


class Rve:
    """One RVE handle: device workspace from torch, stream from torch."""

    def __init__(self, cfg, stream=None, device="cuda"):
        import torch
        self.cfg = cfg
        self.nbytes = rve_query_workspace(cfg)
        self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.stream = stream
        sptr = stream.cuda_stream if stream is not None else torch.cuda.current_stream().cuda_stream
        h = C.c_void_p()
        rc = lib.rve_create(C.byref(cfg), C.c_void_p(self.workspace.data_ptr()),
                            C.c_size_t(self.nbytes), C.c_void_p(sptr), C.byref(h))
        if rc != RVE_OK:
            raise MirveError(rc, lib.rve_last_error(None).decode())
        self.h = h
        self.B = int(cfg.batch)
        self.dim = cfg.dim
        self.n = tuple(cfg.n[: cfg.dim])
        self.s = 3 if cfg.dim == 2 else 6
        self.N = int(np.prod(self.n))
        self.shape = tuple(reversed(self.n))

    def _chk(self, rc):
        if rc != RVE_OK:
            raise MirveError(rc, lib.rve_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib.rve_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API with the C names' semantics ------------------------------------
    def rve_set_microstructure(self, phase_id, phases, theta=None, void=None, phi_disc=None,
                               phi_M=0.8, slot=0):
        pid = np.ascontiguousarray(phase_id, dtype=np.uint16).reshape(-1)
        assert pid.size == self.N
        th = None if theta is None else np.ascontiguousarray(theta, dtype=np.float64).reshape(-1)
        vm = None if void is None else np.ascontiguousarray(void, dtype=np.uint8).reshape(-1)
        pd = None if phi_disc is None else np.ascontiguousarray(phi_disc, dtype=np.uint8).reshape(-1)
        arr = phases_array(phases)
        vp = lambda a: None if a is None else C.c_void_p(a.ctypes.data)
        self._chk(lib.rve_set_microstructure_slot(self.h, int(slot), vp(pid), arr, len(phases),
                                                  vp(th), vp(vm), vp(pd), float(phi_M)))

    def rve_set_microstructure_euler(self, phase_id, phases, euler, void=None, phi_disc=None, phi_M=0.8,
                                     slot=0):
        pid = np.ascontiguousarray(phase_id, dtype=np.uint16).reshape(-1)
        assert pid.size == self.N
        eu = np.ascontiguousarray(euler, dtype=np.float64).reshape(-1)
        assert eu.size == 3 * self.N
        vm = None if void is None else np.ascontiguousarray(void, dtype=np.uint8).reshape(-1)
        pd = None if phi_disc is None else np.ascontiguousarray(phi_disc, dtype=np.uint8).reshape(-1)
        arr = phases_array(phases)
        vp = lambda a: None if a is None else C.c_void_p(a.ctypes.data)
        self._chk(lib.rve_set_microstructure_euler(self.h, int(slot), vp(pid), arr, len(phases), vp(eu),
                                                   vp(vm), vp(pd), float(phi_M)))

    def set_workload(self, w, slot=0):
        if getattr(w, "euler", None) is not None:
            self.rve_set_microstructure_euler(w.phase_id, w.phases, w.euler, void=w.void,
                                              phi_disc=w.phi_disc, phi_M=w.phi_M, slot=slot)
            return
        self.rve_set_microstructure(w.phase_id, w.phases, theta=w.theta, void=w.void,
                                    phi_disc=w.phi_disc, phi_M=w.phi_M, slot=slot)

    def rve_step_dissipation_slots(self, dtaus):
        """One lockstep step; dtaus[b] > 0 steps slot b.  Returns (infos, status)."""
        dt = np.ascontiguousarray(dtaus, dtype=np.float64)
        assert dt.size == self.B
        infos = (rve_step_info * self.B)()
        status = (C.c_int * self.B)()
        lib.rve_step_dissipation_slots(self.h, _dptr(dt), infos, status)
        return [infos[i].as_dict() for i in range(self.B)], [status[i] for i in range(self.B)]

    def rve_run_slots(self, dtaus, max_steps, stop_at_fracture=False):
        """Up to max_steps[b] steps of dtaus[b] per slot, each slot at its own
        pace.  Returns (infos, status)."""
        dt = np.ascontiguousarray(dtaus, dtype=np.float64)
        ms = np.ascontiguousarray(max_steps, dtype=np.int32)
        assert dt.size == self.B and ms.size == self.B
        infos = (rve_step_info * self.B)()
        status = (C.c_int * self.B)()
        lib.rve_run_slots(self.h, _dptr(dt), ms.ctypes.data_as(C.POINTER(C.c_int)),
                          RVE_RUN_STOP_AT_FRACTURE if stop_at_fracture else 0, infos, status)
        return [infos[i].as_dict() for i in range(self.B)], [status[i] for i in range(self.B)]

    def rve_run_budget(self, dtaus, total_steps, stop_at_fracture=False, keep=False, max_steps=None):
        """Steps at each slot's own pace until the slots together committed
        total_steps (keep: steps in flight at the end stay for the next
        keep call).  Returns (infos, status)."""
        dt = np.ascontiguousarray(dtaus, dtype=np.float64)
        assert dt.size == self.B
        ms = None
        if max_steps is not None:
            ms = np.ascontiguousarray(max_steps, dtype=np.int32)
            assert ms.size == self.B
        infos = (rve_step_info * self.B)()
        status = (C.c_int * self.B)()
        flags = (RVE_RUN_STOP_AT_FRACTURE if stop_at_fracture else 0) | (RVE_RUN_KEEP if keep else 0)
        lib.rve_run_budget(self.h, _dptr(dt), None if ms is None else ms.ctypes.data_as(C.POINTER(C.c_int)),
                           int(total_steps), flags, infos, status)
        return [infos[i].as_dict() for i in range(self.B)], [status[i] for i in range(self.B)]

    def rve_step_newton(self, dtau, slot=0, **opts):
        """One step by the monolithic Newton-Raphson solver; opts override the
        fields of rve_newton_opts.  The Krylov workspace is a device buffer
        kept per restart length."""
        import torch
        o = rve_newton_opts()
        lib.rve_newton_default_opts(C.byref(o))
        for key, v in opts.items():
            setattr(o, key, v)
        nb = C.c_size_t(0)
        self._chk(lib.rve_newton_workspace(self.h, o.restart, C.byref(nb)))
        ws = getattr(self, "_newton_ws", None)
        if ws is None or ws.numel() < nb.value:
            ws = self._newton_ws = torch.empty(nb.value, dtype=torch.uint8, device=self.workspace.device)
        info = rve_step_info()
        self._chk(lib.rve_step_newton(self.h, int(slot), float(dtau), C.byref(o), C.c_void_p(ws.data_ptr()),
                                      C.c_size_t(nb.value), C.byref(info)))
        return info.as_dict()

    def rve_run_stats(self):
        """(rounds, mean fraction of the slots each round covered) of the last
        rve_run_slots or rve_run_budget call."""
        out = np.zeros(2)
        self._chk(lib.rve_run_stats(self.h, _dptr(out)))
        return int(out[0]), float(out[1])

    def rve_save_state(self, slot=0):
        n = C.c_size_t(0)
        self._chk(lib.rve_state_bytes(self.h, C.byref(n)))
        buf = np.zeros(n.value, dtype=np.uint8)
        self._chk(lib.rve_save_state(self.h, int(slot), C.c_void_p(buf.ctypes.data), n.value))
        return buf

    def rve_load_state(self, blob, slot=0):
        b = np.ascontiguousarray(blob, dtype=np.uint8)
        self._chk(lib.rve_load_state(self.h, int(slot), C.c_void_p(b.ctypes.data), b.size))

    def rve_release_slot(self, slot):
        self._chk(lib.rve_release_slot(self.h, int(slot)))

    def rve_step_dissipation(self, dtau):
        info = rve_step_info()
        self._chk(lib.rve_step_dissipation(self.h, float(dtau), C.byref(info)))
        return info.as_dict()

    def rve_effective_toughness(self, slot=0):
        g = C.c_double(0.0)
        self._chk(lib.rve_effective_toughness_slot(self.h, int(slot), C.byref(g)))
        return g.value

    def rve_get_field(self, name, slot=0):
        which = FIELDS[name]
        cnt = self.N * (self.s if name in ("eps1", "sig1") else 1)
        out = np.empty(cnt, dtype=np.float64)
        self._chk(lib.rve_get_field_slot(self.h, int(slot), which, _dptr(out), cnt))
        if name in ("eps1", "sig1"):
            return out.reshape((self.s,) + self.shape)
        return out.reshape(self.shape)

    def rve_set_field(self, name, arr, slot=0):
        a = np.ascontiguousarray(arr, dtype=np.float64).reshape(-1)
        self._chk(lib.rve_set_field_slot(self.h, int(slot), FIELDS[name], _dptr(a), a.size))

    def rve_get_scalars(self, slot=0):
        o = np.zeros(8)
        self._chk(lib.rve_get_scalars_slot(self.h, int(slot), _dptr(o)))
        return dict(E=o[0], Sigma=o[1], T=o[2], tau=o[3], tau0=o[4], step=int(o[5]),
                    fractured=bool(o[6]), A_g=o[7])

    def rve_set_scalars(self, d, slot=0):
        a = np.array([d["E"], d["Sigma"], d["T"], d["tau"], d["tau0"], d["step"]], dtype=float)
        self._chk(lib.rve_set_scalars_slot(self.h, int(slot), _dptr(a)))

    def rve_apply_green_op(self, eps):
        e = np.ascontiguousarray(eps, dtype=np.float64).reshape(-1)
        assert e.size == self.s * self.N
        out = np.empty_like(e)
        self._chk(lib.rve_apply_green_op(self.h, _dptr(e), _dptr(out)))
        return out.reshape((self.s,) + self.shape)

    def rve_apply_green_op_device(self, eps_dev, out_dev, repeat=1):
        self._chk(lib.rve_apply_green_op_device(self.h, C.c_void_p(eps_dev.data_ptr()),
                                                C.c_void_p(out_dev.data_ptr()), int(repeat)))

    def rve_apply_green_op_device_noalloc(self, eps_dev, out_dev, repeat=1):
        """rve_apply_green_op_device with the spectrum and partial sums in the
        library's static device array (allocates nothing)."""
        self._chk(lib.rve_apply_green_op_device_noalloc(self.h, C.c_void_p(eps_dev.data_ptr()),
                                                        C.c_void_p(out_dev.data_ptr()), int(repeat)))

    def rve_solve_mechanics(self):
        it = C.c_int(0)
        s1 = C.c_double(0.0)
        self._chk(lib.rve_solve_mechanics(self.h, C.byref(it), C.byref(s1)))
        return it.value, s1.value

    def rve_solve_damage(self, E, commit=False):
        D = C.c_double(0.0)
        it = C.c_int(0)
        self._chk(lib.rve_solve_damage(self.h, float(E), C.byref(D), C.byref(it), int(commit)))
        return D.value, it.value

    def rve_dissipation(self):
        D = C.c_double(0.0)
        G = C.c_double(0.0)
        self._chk(lib.rve_dissipation(self.h, C.byref(D), C.byref(G)))
        return D.value, G.value


    def rve_autotune(self, repeat=20):
        """Pick the fastest launch shapes for this handle; returns
        (rows per x block, y lines per block, z columns per tile,
        1 if the Krylov vectors are streamed non-temporally)."""
        out = (C.c_int * 4)()
        self._chk(lib.rve_autotune(self.h, int(repeat), out))
        return tuple(out)

    def rve_profile_pass(self, which, repeat=1):
        b = C.c_double(0.0)
        self._chk(lib.rve_profile_pass(self.h, int(which), int(repeat), C.byref(b)))
        return b.value


def rve_step_dissipation_batch(rves, dtaus):
    n = len(rves)
    hs = (C.c_void_p * n)(*[r.h for r in rves])
    dt = np.ascontiguousarray(dtaus, dtype=np.float64)
    infos = (rve_step_info * n)()
    status = (C.c_int * n)()
    lib.rve_step_dissipation_batch(hs, n, _dptr(dt), infos, status)
    return [infos[i].as_dict() for i in range(n)], [status[i] for i in range(n)]


def rve_version():
    return lib.rve_version().decode()


def from_workload(w, precision=RVE_PREC_FP64, stream=None, **kw):
    """Create a handle for a workloads.Workload and set its microstructure."""
    cfg = make_config(w.n, h=w.h, ell=w.ell, k=w.k, f=w.f, precision=precision, **kw)
    r = Rve(cfg, stream=stream)
    r.set_workload(w)
    return r


def from_workloads(ws, precision=RVE_PREC_FP64, stream=None, **kw):
    """One batched handle holding the workloads (same grid, l, h, k, f) in
    slots 0..len(ws)-1."""
    w0 = ws[0]
    for w in ws:
        assert tuple(w.n) == tuple(w0.n) and w.ell == w0.ell and w.h == w0.h and w.k == w0.k
        assert np.array_equal(np.asarray(w.f), np.asarray(w0.f))
    kw.setdefault("max_materials", max(4096, max(len(w.phases) * 2 for w in ws)))
    cfg = make_config(w0.n, h=w0.h, ell=w0.ell, k=w0.k, f=w0.f, precision=precision,
                      batch=len(ws), **kw)
    r = Rve(cfg, stream=stream)
    for i, w in enumerate(ws):
        r.set_workload(w, slot=i)
    return r
