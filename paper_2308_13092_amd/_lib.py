"""ctypes binding of libecpic.so (argument marshalling only).

Every step of the method runs in the HIP library; this module converts
Python dictionaries and numpy arrays to the C structures of
``include/ecpic.h`` and back, and holds the torch-allocated device arena.
There is no fallback: without the built library every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libecpic.so")

PIC_OK, PIC_EINVAL, PIC_ENOMEM, PIC_ECAPACITY, PIC_ENONFINITE, PIC_EGROWTH, PIC_EDEVICE, PIC_ESTATE = range(8)
STATUS_NAMES = ["PIC_OK", "PIC_EINVAL", "PIC_ENOMEM", "PIC_ECAPACITY", "PIC_ENONFINITE",
                "PIC_EGROWTH", "PIC_EDEVICE", "PIC_ESTATE"]


class pic_config(C.Structure):
    _fields_ = [
        ("n_cells", C.c_int32), ("bc", C.c_int32), ("nodes", C.POINTER(C.c_double)),
        ("gap_m", C.c_double), ("v_rf", C.c_double), ("f_rf", C.c_double), ("phase", C.c_double),
        ("p_pa", C.c_double), ("t_gas_k", C.c_double), ("n0_m3", C.c_double), ("te_ev", C.c_double),
        ("ti_ev", C.c_double), ("n_per_species", C.c_int64), ("capacity", C.c_int64),
        ("weight_m2", C.c_double), ("dt_s", C.c_double), ("gather", C.c_int32),
        ("precision", C.c_int32), ("gamma_see", C.c_double), ("t_see_ev", C.c_double),
        ("seed", C.c_uint64), ("sort_interval", C.c_int32), ("n_species", C.c_int32),
        ("collisions", C.c_int32), ("pullback", C.c_int32), ("nu_max_e", C.c_double),
        ("nu_max_i", C.c_double), ("avg_start", C.c_int64), ("avg_every", C.c_int32),
        ("eedf_every", C.c_int32), ("eedf_bins", C.c_int32), ("eedf_emax_ev", C.c_double),
        ("eedf_width_m", C.c_double), ("k_stop", C.c_int64), ("growth_limit", C.c_double),
        ("impact_bins", C.c_int32), ("impact_angle_bins", C.c_int32), ("impact_emax_ev", C.c_double),
        ("moments", C.c_int32), ("rebalance_ppc", C.c_int32), ("rebalance_every", C.c_int32),
        ("rebalance_dv_e", C.c_double), ("rebalance_dv_i", C.c_double),
    ]


class pic_diag(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("time_s", C.c_double), ("status", C.c_int32),
        ("n_samples", C.c_int32), ("eedf_samples", C.c_int32), ("reserved0", C.c_int32),
        ("n_live", C.c_int64 * 2), ("extent", C.c_int64 * 2), ("deposit_total", C.c_int64 * 2),
        ("kinetic_j_m2", C.c_double * 2), ("field_j_m2", C.c_double),
        ("absorbed", (C.c_int64 * 2) * 2), ("absorbed_energy_ev", (C.c_double * 2) * 2),
        ("see_emitted", C.c_int64), ("ionisations", C.c_int64), ("excitations", C.c_int64),
        ("elastic", C.c_int64), ("charge_exchange", C.c_int64), ("candidates", C.c_int64 * 2),
        ("bound_violations", C.c_int64), ("particle_steps", C.c_int64), ("ne_max_m3", C.c_double),
        ("wpe_dt_max", C.c_double), ("vmax_dt_over_dxmin", C.c_double),
        ("lambda_de_over_dxmin", C.c_double), ("nu_max", C.c_double * 2),
        ("merges", C.c_int64 * 2), ("splits", C.c_int64 * 2),
    ]


class pic_state_view(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("x", C.POINTER(C.c_double)), ("cell", C.POINTER(C.c_int32)),
        ("off", C.POINTER(C.c_float)), ("vx", C.c_void_p), ("vy", C.c_void_p), ("vz", C.c_void_p),
        ("id", C.POINTER(C.c_uint64)), ("knext", C.POINTER(C.c_int32)),
        ("wclass", C.POINTER(C.c_uint8)),
    ]


class pic_tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("blocks_per_cu", C.c_int32), ("sort_interval", C.c_int32),
                ("use_graph", C.c_int32), ("inline_drain", C.c_int32)]


class pic_kernel_time(C.Structure):
    _fields_ = [("field_ms", C.c_double), ("field_launches", C.c_int64),
                ("particle_ms", C.c_double), ("particle_launches", C.c_int64),
                ("drain_ms", C.c_double), ("drain_launches", C.c_int64),
                ("sort_ms", C.c_double), ("sort_launches", C.c_int64)]


# (name, restype, argtypes) of every entry point declared in include/ecpic.h.
_CTX = C.c_void_p
SIGNATURES = [
    ("pic_abi_version", C.c_int32, []),
    ("pic_status_string", C.c_char_p, [C.c_int]),
    ("pic_footprint", C.c_size_t, [C.POINTER(pic_config), C.c_int32]),
    ("pic_init", C.c_int, [C.POINTER(pic_config), C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                           C.POINTER(_CTX)]),
    ("pic_deposit", C.c_int, [_CTX]),
    ("pic_poisson", C.c_int, [_CTX]),
    ("pic_gather_push", C.c_int, [_CTX]),
    ("pic_mcc", C.c_int, [_CTX]),
    ("pic_step", C.c_int, [_CTX, C.c_int32]),
    ("pic_sort", C.c_int, [_CTX]),
    ("pic_rebalance", C.c_int, [_CTX]),
    ("pic_diagnostics", C.c_int, [_CTX, C.c_int32, C.POINTER(pic_diag)]),
    ("pic_diagnostics_noalloc", C.c_int, [_CTX, C.POINTER(C.c_int32), C.c_int32, C.POINTER(pic_diag)]),
    ("pic_get_state", C.c_int, [_CTX, C.c_int32, C.c_int32, C.POINTER(pic_state_view)]),
    ("pic_set_state", C.c_int, [_CTX, C.c_int32, C.c_int32, C.POINTER(pic_state_view)]),
    ("pic_set_step", C.c_int, [_CTX, C.c_int32, C.c_int64]),
    ("pic_get_fields", C.c_int, [_CTX, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p]),
    ("pic_profiles", C.c_int, [_CTX, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pic_impacts", C.c_int, [_CTX, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    ("pic_moments", C.c_int, [_CTX, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("pic_checkpoint_bytes", C.c_int, [_CTX, C.c_int32, C.POINTER(C.c_size_t)]),
    ("pic_checkpoint_save", C.c_int, [_CTX, C.c_int32, C.c_void_p, C.c_size_t]),
    ("pic_checkpoint_load", C.c_int, [_CTX, C.c_int32, C.c_void_p, C.c_size_t]),
    ("pic_slot_reset", C.c_int, [_CTX, C.c_int32, C.POINTER(pic_config)]),
    ("pic_slot_release", C.c_int, [_CTX, C.c_int32]),
    ("pic_slot_bytes", C.c_size_t, [C.POINTER(pic_config)]),
    ("pic_pool_free", C.c_size_t, [_CTX]),
    ("pic_set_tuning", C.c_int, [_CTX, C.POINTER(pic_tuning)]),
    ("pic_get_tuning", C.c_int, [_CTX, C.POINTER(pic_tuning)]),
    ("pic_kernel_times", C.c_int, [_CTX, C.c_int32, C.POINTER(pic_kernel_time)]),
    ("pic_grid_refined", C.c_int32, [C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.POINTER(C.c_double), C.c_int32]),
    ("pic_destroy", None, [_CTX]),
    ("pic_last_error", C.c_char_p, [_CTX]),
]

_lib = None


def load(path=LIB_PATH):
    """Load libecpic.so (raises if it has not been built).

    torch is imported first: it brings its own HIP runtime, and the library
    must bind to that same runtime (its soname is already loaded then), since
    the device arena and the stream it is given come from torch.
    """
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with python -m paper_2308_13092_amd.build")
        import torch  # noqa: F401  (one HIP runtime per process: torch's)
        lib = C.CDLL(path)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class PicError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {msg}")


CONFIG_KEYS = [f[0] for f in pic_config._fields_ if f[0] != "nodes"]


def make_config(d, keep):
    """dict -> pic_config; node arrays are appended to ``keep`` to stay alive."""
    c = pic_config()
    for k in CONFIG_KEYS:
        if k in d and d[k] is not None:
            setattr(c, k, d[k])
    nodes = d.get("nodes")
    if nodes is not None:
        arr = np.ascontiguousarray(nodes, dtype=np.float64)
        keep.append(arr)
        c.nodes = arr.ctypes.data_as(C.POINTER(C.c_double))
        c.n_cells = len(arr) - 1
    return c


def grid_refined(L, dx_min, dx_max, L_buff):
    """Nodes of the Section 3c refined grid, built by the library."""
    lib = load()
    n = lib.pic_grid_refined(L, dx_min, dx_max, L_buff, None, 0)
    if n < 0:
        raise ValueError("bad refined-grid arguments")
    out = np.empty(n + 1, dtype=np.float64)
    lib.pic_grid_refined(L, dx_min, dx_max, L_buff, out.ctypes.data_as(C.POINTER(C.c_double)), n + 1)
    return out


def footprint(cfgs):
    lib = load()
    keep = []
    arr = (pic_config * len(cfgs))(*[make_config(d, keep) for d in cfgs])
    return int(lib.pic_footprint(arr, len(cfgs)))


def slot_bytes(cfg):
    keep = []
    c = make_config(cfg, keep)
    return int(load().pic_slot_bytes(C.byref(c)))


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


class Context:
    """One library context over a torch-allocated device arena.

    ``cfgs`` is a list of configuration dicts (keys of ``pic_config``; an
    entry with n_cells == 0 is an empty slot); ``pool_bytes`` extra arena bytes
    are left for ``slot_reset``.
    """

    def __init__(self, cfgs, pool_bytes=0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the EC-PIC library needs a GPU")
        self.lib = load()
        self._keep = []
        self.cfgs = [dict(c) for c in cfgs]
        arr = (pic_config * len(cfgs))(*[make_config(d, self._keep) for d in cfgs])
        need = int(self.lib.pic_footprint(arr, len(cfgs)))
        if need == 0:
            raise PicError(PIC_EINVAL, "bad configuration list")
        self.nbytes = need + int(pool_bytes)
        self.arena = torch.empty(self.nbytes, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ctx = C.c_void_p()
        st = self.lib.pic_init(arr, len(cfgs), C.c_void_p(self.arena.data_ptr()), self.nbytes,
                               C.c_void_p(self.stream.cuda_stream), C.byref(self.ctx))
        if st != PIC_OK:
            msg = self.lib.pic_last_error(None)
            raise PicError(st, "pic_init: " + (msg.decode() if msg else ""))
        self.n_inst = len(cfgs)
        # the library's rule: the first discharge's form, else (all slots
        # empty) the first entry's
        first = int(cfgs[0].get("precision", 0)) if cfgs else 0
        self.prec = next((int(c.get("precision", 0)) for c in cfgs if c.get("n_cells", 0)), first)

    # -- plumbing -----------------------------------------------------------
    def _check(self, st, what, allow=()):
        if st != PIC_OK and st not in allow:
            msg = self.lib.pic_last_error(self.ctx)
            raise PicError(st, f"{what}: {msg.decode() if msg else ''}")
        return st

    def close(self):
        if self.ctx:
            self.lib.pic_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the step -------------------------------------------------------------
    def deposit(self):
        self._check(self.lib.pic_deposit(self.ctx), "pic_deposit")

    def poisson(self):
        self._check(self.lib.pic_poisson(self.ctx), "pic_poisson")

    def gather_push(self):
        self._check(self.lib.pic_gather_push(self.ctx), "pic_gather_push")

    def mcc(self):
        self._check(self.lib.pic_mcc(self.ctx), "pic_mcc")

    def step(self, n=1):
        self._check(self.lib.pic_step(self.ctx, int(n)), "pic_step")

    def sort(self):
        self._check(self.lib.pic_sort(self.ctx), "pic_sort")

    def rebalance(self):
        self._check(self.lib.pic_rebalance(self.ctx), "pic_rebalance")

    # -- results --------------------------------------------------------------
    def diagnostics(self, inst=0, allow_error=False):
        d = pic_diag()
        st = self.lib.pic_diagnostics(self.ctx, inst, C.byref(d))
        if not allow_error:
            self._check(st, "pic_diagnostics")
        out = {}
        for name, _ in pic_diag._fields_:
            v = getattr(d, name)
            if isinstance(v, C.Array):
                v = np.array([list(r) if isinstance(r, C.Array) else r for r in v])
            out[name] = v
        out["return_status"] = st
        return out

    @staticmethod
    def _diag_dict(d):
        out = {}
        for name, _ in pic_diag._fields_:
            v = getattr(d, name)
            if isinstance(v, C.Array):
                v = np.array([list(r) if isinstance(r, C.Array) else r for r in v])
            out[name] = v
        return out

    def diagnostics_noalloc(self, insts):
        """pic_diagnostics_noalloc over a list of instances: one dict per
        instance, as ``diagnostics`` gives."""
        n = len(insts)
        ids = (C.c_int32 * max(n, 1))(*[int(i) for i in insts])
        outs = (pic_diag * max(n, 1))()
        st = self.lib.pic_diagnostics_noalloc(self.ctx, ids, n, outs)
        self._check(st, "pic_diagnostics_noalloc")
        res = []
        for i in range(n):
            d = self._diag_dict(outs[i])
            d["return_status"] = st
            res.append(d)
        return res

    def get_state(self, inst, species):
        d = self.diagnostics(inst, allow_error=True)
        n = int(d["extent"][species])
        out = {}
        v = pic_state_view()
        v.n = n
        if self.prec == 1:
            out["cell"] = np.empty(n, np.int32)
            out["off"] = np.empty(n, np.float32)
            vt = np.float32
            v.cell = out["cell"].ctypes.data_as(C.POINTER(C.c_int32))
            v.off = out["off"].ctypes.data_as(C.POINTER(C.c_float))
        else:
            out["x"] = np.empty(n, np.float64)
            vt = np.float64
            v.x = out["x"].ctypes.data_as(C.POINTER(C.c_double))
        for f in ("vx", "vy", "vz"):
            out[f] = np.empty(n, vt)
            setattr(v, f, out[f].ctypes.data)
        out["id"] = np.empty(n, np.uint64)
        out["knext"] = np.empty(n, np.int32)
        v.id = out["id"].ctypes.data_as(C.POINTER(C.c_uint64))
        v.knext = out["knext"].ctypes.data_as(C.POINTER(C.c_int32))
        if self.prec == 1:
            out["wc"] = np.empty(n, np.uint8)
            v.wclass = out["wc"].ctypes.data_as(C.POINTER(C.c_uint8))
        st = self.lib.pic_get_state(self.ctx, inst, species, C.byref(v))
        self._check(st, "pic_get_state", allow=(PIC_ECAPACITY, PIC_ENONFINITE, PIC_EGROWTH))
        m = int(v.n)
        return {k: a[:m].copy() for k, a in out.items()}

    def set_state(self, inst, species, st):
        v = pic_state_view()
        n = len(st["id"])
        v.n = n
        keep = {}
        vt = np.float32 if self.prec == 1 else np.float64
        if self.prec == 1:
            keep["cell"] = np.ascontiguousarray(st["cell"], np.int32)
            keep["off"] = np.ascontiguousarray(st["off"], np.float32)
            v.cell = keep["cell"].ctypes.data_as(C.POINTER(C.c_int32))
            v.off = keep["off"].ctypes.data_as(C.POINTER(C.c_float))
        else:
            keep["x"] = np.ascontiguousarray(st["x"], np.float64)
            v.x = keep["x"].ctypes.data_as(C.POINTER(C.c_double))
        for f in ("vx", "vy", "vz"):
            keep[f] = np.ascontiguousarray(st[f], vt)
            setattr(v, f, keep[f].ctypes.data)
        keep["id"] = np.ascontiguousarray(st["id"], np.uint64)
        keep["knext"] = np.ascontiguousarray(np.minimum(st["knext"], 2 ** 31 - 1), np.int32)
        v.id = keep["id"].ctypes.data_as(C.POINTER(C.c_uint64))
        v.knext = keep["knext"].ctypes.data_as(C.POINTER(C.c_int32))
        if self.prec == 1 and st.get("wc") is not None:
            keep["wc"] = np.ascontiguousarray(st["wc"], np.uint8)
            v.wclass = keep["wc"].ctypes.data_as(C.POINTER(C.c_uint8))
        self._check(self.lib.pic_set_state(self.ctx, inst, species, C.byref(v)), "pic_set_state")

    def set_step(self, inst, k):
        self._check(self.lib.pic_set_step(self.ctx, inst, int(k)), "pic_set_step")

    def fields(self, inst=0):
        cfg = self.cfgs[inst]
        N = int(cfg["n_cells"]) if cfg.get("nodes") is None else len(cfg["nodes"]) - 1
        ne = N + int(cfg.get("gather", 0))     # EC cells, MC nodes, or EC2 centres + 2 ghosts
        out = dict(A_e=np.zeros(N + 1, np.int64), A_i=np.zeros(N + 1, np.int64),
                   phi=np.zeros(N + 1), E=np.zeros(ne), E32=np.zeros(ne, np.float32))
        st = self.lib.pic_get_fields(self.ctx, inst, _ptr(out["A_e"]), _ptr(out["A_i"]),
                                     _ptr(out["phi"]), _ptr(out["E"]), _ptr(out["E32"]))
        self._check(st, "pic_get_fields", allow=(PIC_ECAPACITY, PIC_ENONFINITE, PIC_EGROWTH))
        return out

    def profiles(self, inst=0):
        cfg = self.cfgs[inst]
        N = int(cfg["n_cells"]) if cfg.get("nodes") is None else len(cfg["nodes"]) - 1
        bins = int(cfg.get("eedf_bins", 0) or 200)
        out = dict(ne=np.zeros(N + 1), ni=np.zeros(N + 1), phi=np.zeros(N + 1),
                   eedf=np.zeros(bins, np.int64))
        st = self.lib.pic_profiles(self.ctx, inst, _ptr(out["ne"]), _ptr(out["ni"]),
                                   _ptr(out["phi"]), _ptr(out["eedf"]))
        self._check(st, "pic_profiles", allow=(PIC_ECAPACITY, PIC_ENONFINITE, PIC_EGROWTH))
        return out

    def moments(self, inst, species):
        """Averaged mean x-velocity and x-temperature at the nodes and power
        density per cell of one species."""
        cfg = self.cfgs[inst]
        N = int(cfg["n_cells"]) if cfg.get("nodes") is None else len(cfg["nodes"]) - 1
        out = dict(ux=np.zeros(N + 1), tx=np.zeros(N + 1), power=np.zeros(N))
        st = self.lib.pic_moments(self.ctx, inst, species, _ptr(out["ux"]), _ptr(out["tx"]),
                                  _ptr(out["power"]))
        self._check(st, "pic_moments", allow=(PIC_ECAPACITY, PIC_ENONFINITE, PIC_EGROWTH))
        return out

    def impacts(self, inst, species, wall):
        """Energy (bins + overflow) and angle counts of particles of ``species``
        absorbed at ``wall`` (0: x = 0, 1: x = L) over the averaged steps."""
        cfg = self.cfgs[inst]
        nb = int(cfg.get("impact_bins", 0) or 200)
        na = int(cfg.get("impact_angle_bins", 0) or 90)
        out = dict(energy=np.zeros(nb + 1, np.int64), angle=np.zeros(na, np.int64))
        st = self.lib.pic_impacts(self.ctx, inst, species, wall, _ptr(out["energy"]), _ptr(out["angle"]))
        self._check(st, "pic_impacts", allow=(PIC_ECAPACITY, PIC_ENONFINITE, PIC_EGROWTH))
        return out

    # -- checkpoint and resume -------------------------------------------------
    def checkpoint(self, inst):
        """The instance's restorable state as bytes (pic_checkpoint_save)."""
        n = C.c_size_t()
        self._check(self.lib.pic_checkpoint_bytes(self.ctx, inst, C.byref(n)), "pic_checkpoint_bytes")
        buf = np.empty(n.value, dtype=np.uint8)
        st = self.lib.pic_checkpoint_save(self.ctx, inst, C.c_void_p(buf.ctypes.data), n.value)
        self._check(st, "pic_checkpoint_save", allow=(PIC_ECAPACITY, PIC_ENONFINITE, PIC_EGROWTH))
        return buf.tobytes()

    def restore(self, inst, data):
        """Load a checkpoint into slot ``inst`` (pic_checkpoint_load)."""
        buf = np.frombuffer(data, dtype=np.uint8)
        self._check(self.lib.pic_checkpoint_load(self.ctx, inst, C.c_void_p(buf.ctypes.data), len(buf)),
                    "pic_checkpoint_load")

    # -- slots, tuning, timing ------------------------------------------------
    def slot_reset(self, inst, cfg):
        keep = []
        c = make_config(cfg, keep)
        st = self.lib.pic_slot_reset(self.ctx, inst, C.byref(c))
        if st == PIC_OK:
            self.cfgs[inst] = dict(cfg)
        return self._check(st, "pic_slot_reset", allow=(PIC_ENOMEM,))

    def slot_release(self, inst):
        self._check(self.lib.pic_slot_release(self.ctx, inst), "pic_slot_release")

    def pool_free(self):
        return int(self.lib.pic_pool_free(self.ctx))

    def tuning(self):
        t = pic_tuning()
        self._check(self.lib.pic_get_tuning(self.ctx, C.byref(t)), "pic_get_tuning")
        return dict(block=t.block, blocks_per_cu=t.blocks_per_cu, sort_interval=t.sort_interval,
                    use_graph=t.use_graph, inline_drain=t.inline_drain)

    def set_tuning(self, **kw):
        cur = self.tuning()
        cur.update(kw)
        t = pic_tuning(**cur)
        self._check(self.lib.pic_set_tuning(self.ctx, C.byref(t)), "pic_set_tuning")

    def kernel_times(self, enable):
        kt = pic_kernel_time()
        self._check(self.lib.pic_kernel_times(self.ctx, int(enable), C.byref(kt)), "pic_kernel_times")
        return {name: getattr(kt, name) for name, _ in pic_kernel_time._fields_}
