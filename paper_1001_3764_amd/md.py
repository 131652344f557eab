"""ctypes binding of the C ABI declared in ``include/md.h`` (argument marshalling only).

PyTorch supplies device memory and the HIP stream; every step of the simulation runs in
the library's HIP kernels.  If ``libmd_gfx950.so`` is missing this module raises: there
is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

LIB_PATH = os.environ.get("PAPER_1001_3764_AMD_LIB") or os.path.join(
    os.path.dirname(os.path.abspath(__file__)), "libmd_gfx950.so")

MD_OK, MD_ERR_ARG, MD_ERR_BOX_TOO_SMALL, MD_ERR_NONFINITE = 0, -1, -2, -3
MD_ERR_WORKSPACE, MD_ERR_HIP, MD_ERR_STATE, MD_ERR_NLIST = -4, -6, -7, -8
MD_PREC_FP64, MD_PREC_MIXED = 0, 1
MD_LJ_AUTO, MD_LJ_ATOM, MD_LJ_CELLTILE, MD_LJ_CELLTILE_NB, MD_LJ_NLIST, MD_LJ_NLIST_TILE = 0, 1, 2, 3, 4, 5
MD_LJ_HALFSHELL = 6
MD_INT_VERLET_BERENDSEN, MD_INT_LEAPFROG_NH = 0, 1

_D, _I32, _I64, _P = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p


class md_forcefield(ctypes.Structure):
    _fields_ = [("mass", _D * 2), ("sigma", _D * 2), ("epsilon", _D * 2), ("kb", _D), ("b0", _D),
                ("ka", _D), ("theta0_deg", _D), ("kphi", _D), ("phis_deg", _D), ("n_dih", _I32),
                ("rc", _D), ("excl_depth", _I32)]


class md_config(ctypes.Structure):
    _fields_ = [("n_boxes", _I32), ("chain_len", _I32), ("n_chains", ctypes.POINTER(_I32)),
                ("box", ctypes.POINTER(_D)), ("T0", ctypes.POINTER(_D)), ("dt_fs", _D), ("tau_fs", _D),
                ("precision", _I32), ("cell_div", _I32), ("lj_kernel", _I32), ("use_graph", _I32),
                ("nl_skin", _D), ("nl_every", _I32), ("integrator", _I32), ("remove_com", _I32),
                ("tile_homes", _I32)]


class md_energy(ctypes.Structure):
    _fields_ = [("e_lj", _D), ("e_lj_shifted", _D), ("e_bond", _D), ("e_angle", _D), ("e_dih", _D),
                ("e_kin", _D), ("temperature", _D), ("virial", _D), ("step", _I64), ("nh_xi", _D),
                ("e_thermostat", _D)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class md_obs_config(ctypes.Structure):
    _fields_ = [("rdf_bins", _I32), ("rdf_rmax", _D), ("dih_bins", _I32)]


MD_OBS_MAX_BINS = 2048


class MDError(RuntimeError):
    def __init__(self, status, what, detail=""):
        self.status = status
        super().__init__("%s failed: %s (%d)%s" % (what, _status_string(status), status,
                                                    (": " + detail) if detail else ""))


_LIB = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmd_gfx950.so not found at %s; build it with __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    S = ctypes.c_int
    sig = {
        "md_workspace_bytes": (S, [_P, _P, ctypes.POINTER(ctypes.c_size_t)]),
        "md_init_system": (S, [_P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
        "md_init_system_static": (S, [_P, _P, _P, _P, _P, _P, ctypes.POINTER(_P)]),
        "md_rebuild_bins": (S, [_P]),
        "md_compute_forces": (S, [_P, _I32]),
        "md_step": (S, [_P, _I32]),
        "md_energies": (S, [_P, _P]),
        "md_step_timed": (S, [_P, _I32, _P]),
        "md_bins": (S, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.POINTER(_I64)]),
        "md_grid": (S, [_P, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
        "md_forces": (S, [_P, ctypes.POINTER(_P), ctypes.POINTER(_I32)]),
        "md_forces_lj": (S, [_P, ctypes.POINTER(_P), ctypes.POINTER(_I32)]),
        "md_tuning": (S, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
        "md_destroy": (S, [_P]),
        "md_observables": (S, [_P, _P, _P, _P, _P]),
        "md_ree_reference": (S, [_P]),
        "md_ree_acf": (S, [_P, _P]),
        "md_list_builds": (S, [_P, ctypes.POINTER(_I64)]),
        "md_status_string": (ctypes.c_char_p, [S]),
        "md_last_error": (ctypes.c_char_p, [_P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


def _status_string(s):
    try:
        return load().md_status_string(s).decode()
    except Exception:
        return "status"


def _check(status, what, ctx=None):
    if status != MD_OK:
        detail = ""
        if ctx:
            detail = load().md_last_error(ctx).decode(errors="replace")
        raise MDError(status, what, detail)


def make_forcefield(ff: dict) -> md_forcefield:
    s = md_forcefield()
    s.mass[:] = ff["mass"]
    s.sigma[:] = ff["sigma"]
    s.epsilon[:] = ff["epsilon"]
    for k in ("kb", "b0", "ka", "theta0_deg", "kphi", "phis_deg", "rc"):
        setattr(s, k, float(ff[k]))
    s.n_dih = int(ff["n_dih"])
    s.excl_depth = int(ff["excl_depth"])
    return s


class _Config:
    """md_config plus the host arrays it points to (kept alive together)."""

    def __init__(self, n_chains, boxes, T0, chain_len, dt, tau, precision, cell_div, lj_kernel, use_graph,
                 nl_skin=0.0, nl_every=1, integrator=MD_INT_VERLET_BERENDSEN, remove_com=False, tile_homes=0):
        self.n_chains = np.ascontiguousarray(n_chains, dtype=np.int32)
        self.box = np.ascontiguousarray(np.asarray(boxes, dtype=np.float64).reshape(-1, 3))
        self.T0 = np.ascontiguousarray(T0, dtype=np.float64)
        c = md_config()
        c.n_boxes = self.n_chains.size
        c.chain_len = int(chain_len)
        c.n_chains = self.n_chains.ctypes.data_as(ctypes.POINTER(_I32))
        c.box = self.box.ctypes.data_as(ctypes.POINTER(_D))
        c.T0 = self.T0.ctypes.data_as(ctypes.POINTER(_D))
        c.dt_fs = float(dt)
        c.tau_fs = float(tau)
        c.precision = MD_PREC_MIXED if precision in ("mixed", MD_PREC_MIXED) else MD_PREC_FP64
        c.cell_div = int(cell_div)
        c.lj_kernel = int(lj_kernel)
        c.use_graph = int(bool(use_graph))
        c.nl_skin = float(nl_skin)
        c.nl_every = int(nl_every)
        c.integrator = int(integrator)
        c.remove_com = int(bool(remove_com))
        c.tile_homes = int(tile_homes)
        self.c = c


def md_workspace_bytes(ff: md_forcefield, cfg: md_config) -> int:
    n = ctypes.c_size_t()
    _check(load().md_workspace_bytes(ctypes.byref(ff), ctypes.byref(cfg), ctypes.byref(n)), "md_workspace_bytes")
    return n.value


def md_init_system(ff, cfg, pos, vel, types, workspace, stream):
    ctx = _P()
    _check(load().md_init_system(ctypes.byref(ff), ctypes.byref(cfg), pos.data_ptr(), vel.data_ptr(),
                                 types.data_ptr(), workspace.data_ptr(), workspace.numel(), stream,
                                 ctypes.byref(ctx)), "md_init_system")
    return ctx


def md_init_system_static(ff, cfg, pos, vel, types, stream):
    ctx = _P()
    _check(load().md_init_system_static(ctypes.byref(ff), ctypes.byref(cfg), pos.data_ptr(), vel.data_ptr(),
                                        types.data_ptr(), stream, ctypes.byref(ctx)), "md_init_system_static")
    return ctx


MD_STATIC_WORKSPACE_BYTES = 64 << 20


def md_rebuild_bins(ctx):
    _check(load().md_rebuild_bins(ctx), "md_rebuild_bins", ctx)


def md_compute_forces(ctx, with_energy=True):
    _check(load().md_compute_forces(ctx, int(bool(with_energy))), "md_compute_forces", ctx)


def md_step(ctx, n_steps):
    _check(load().md_step(ctx, int(n_steps)), "md_step", ctx)


MD_N_PHASES = 8
PHASES = ("integrate_bin", "scan", "scatter", "rank_payload", "lj", "bonded_kick", "reduce", "nlist_build")


def md_step_timed(ctx, n_steps):
    ms = (_D * MD_N_PHASES)()
    _check(load().md_step_timed(ctx, int(n_steps), ms), "md_step_timed", ctx)
    return dict(zip(PHASES, ms[:]))


def md_energies(ctx, n_boxes):
    out = (md_energy * n_boxes)()
    _check(load().md_energies(ctx, out), "md_energies", ctx)
    return [e.as_dict() for e in out]


def md_bins(ctx):
    cs, ca, n = _P(), _P(), _I64()
    _check(load().md_bins(ctx, ctypes.byref(cs), ctypes.byref(ca), ctypes.byref(n)), "md_bins", ctx)
    return cs.value, ca.value, n.value


def md_grid(ctx, box):
    M = (_I32 * 3)()
    co, ao = _I64(), _I64()
    _check(load().md_grid(ctx, int(box), M, ctypes.byref(co), ctypes.byref(ao)), "md_grid", ctx)
    return np.array(M[:], dtype=np.int32), co.value, ao.value


def md_forces(ctx):
    f, fp32 = _P(), _I32()
    _check(load().md_forces(ctx, ctypes.byref(f), ctypes.byref(fp32)), "md_forces", ctx)
    return f.value, bool(fp32.value)


def md_forces_lj(ctx):
    f, fp32 = _P(), _I32()
    _check(load().md_forces_lj(ctx, ctypes.byref(f), ctypes.byref(fp32)), "md_forces_lj", ctx)
    return f.value, bool(fp32.value)


def md_tuning(ctx, homes=False):
    """(cell_div, lj_kernel), or (cell_div, lj_kernel, tile_homes) with homes=True."""
    r, k, h = _I32(), _I32(), _I32()
    _check(load().md_tuning(ctx, ctypes.byref(r), ctypes.byref(k), ctypes.byref(h)), "md_tuning", ctx)
    return (r.value, k.value, h.value) if homes else (r.value, k.value)


def md_ree_reference(ctx):
    _check(load().md_ree_reference(ctx), "md_ree_reference", ctx)


def md_ree_acf(ctx, out):
    _check(load().md_ree_acf(ctx, out.data_ptr()), "md_ree_acf", ctx)


def md_list_builds(ctx):
    n = _I64()
    _check(load().md_list_builds(ctx, ctypes.byref(n)), "md_list_builds", ctx)
    return n.value


def md_destroy(ctx):
    _check(load().md_destroy(ctx), "md_destroy")


_HIP = None


def _hip_copy_to_host(dst, src, nbytes):
    """hipMemcpy device -> host (synchronous) for device memory that no torch tensor owns."""
    global _HIP
    if _HIP is None:
        _HIP = ctypes.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.restype = ctypes.c_int
        _HIP.hipMemcpy.argtypes = [_P, _P, ctypes.c_size_t, ctypes.c_int]
    rc = _HIP.hipMemcpy(dst, src, nbytes, 2)   # hipMemcpyDeviceToHost
    if rc != 0:
        raise RuntimeError("hipMemcpy device to host failed (%d)" % rc)


class MDSystem:
    """One or more periodic boxes on one GPU: torch owns the device buffers, the HIP
    library owns every computation on them."""

    def __init__(self, ff: dict, n_chains, boxes, T0, pos, vel, types, chain_len=300, dt=1.0, tau=100.0,
                 precision="mixed", cell_div=1, lj_kernel=None, use_graph=False, device="cuda:0",
                 nl_skin=0.0, nl_every=10, integrator="verlet", remove_com=False, static_workspace=False,
                 tile_homes=0):
        """lj_kernel: an md_lj_kernel; None is MD_LJ_ATOM on the cell path and the autotuner
        (0) in neighbour-list mode.
        static_workspace: set up with md_init_system_static (the library's own device array as
        the workspace; no graph, explicit cell_div and lj_kernel).
        nl_skin > 0: neighbour-list mode (bins and list rebuilt every nl_every steps).
        integrator: "verlet" (velocity Verlet, Berendsen when T0 > 0) or "leapfrog" (leap-frog,
        Nose-Hoover when T0 > 0, tau the thermostat period; vel holds half-step velocities).
        remove_com: subtract each box's centre-of-mass velocity after every step."""
        load()
        self.device = torch.device(device)
        self.ff = make_forcefield(ff)
        integ = {"verlet": MD_INT_VERLET_BERENDSEN, "leapfrog": MD_INT_LEAPFROG_NH}.get(integrator, integrator)
        if lj_kernel is None:
            lj_kernel = MD_LJ_AUTO if nl_skin > 0 else MD_LJ_ATOM
        self.cfg = _Config(n_chains, boxes, T0, chain_len, dt, tau, precision, cell_div, lj_kernel, use_graph,
                           nl_skin, nl_every, integ, remove_com, tile_homes)
        self.n_boxes = self.cfg.c.n_boxes
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        vel = np.ascontiguousarray(vel, dtype=np.float64)
        self.N = pos.shape[1]
        assert pos.shape == (3, self.N) and vel.shape == (3, self.N)
        assert self.N == int(self.cfg.n_chains.sum()) * chain_len
        self.pos = torch.from_numpy(pos).to(self.device).contiguous()
        self.vel = torch.from_numpy(vel).to(self.device).contiguous()
        self.types = torch.from_numpy(np.ascontiguousarray(types, dtype=np.uint8)).to(self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = None
        if static_workspace:
            self.workspace = None
            self.ctx = md_init_system_static(self.ff, self.cfg.c, self.pos, self.vel, self.types,
                                             self.stream.cuda_stream)
        else:
            nbytes = md_workspace_bytes(self.ff, self.cfg.c)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.ctx = md_init_system(self.ff, self.cfg.c, self.pos, self.vel, self.types, self.workspace,
                                      self.stream.cuda_stream)

    # --- the C ABI, one call each ---
    def rebuild_bins(self):
        md_rebuild_bins(self.ctx)

    def compute_forces(self, with_energy=True):
        md_compute_forces(self.ctx, with_energy)

    def step(self, n):
        md_step(self.ctx, n)

    def step_timed(self, n):
        return md_step_timed(self.ctx, n)

    def energies(self):
        return md_energies(self.ctx, self.n_boxes)

    def tuning(self, homes=False):
        return md_tuning(self.ctx, homes)

    def list_builds(self):
        return md_list_builds(self.ctx)

    def ree_reference(self):
        md_ree_reference(self.ctx)

    def ree_acf(self):
        """End-to-end vector autocorrelation of each box against the reference (md_ree_acf)."""
        out = torch.zeros(self.n_boxes, dtype=torch.float64, device=self.device)
        md_ree_acf(self.ctx, out)
        torch.cuda.synchronize(self.device)
        return out.cpu().numpy()

    def grid(self, box=0):
        return md_grid(self.ctx, box)

    def observables(self, rdf_bins=105, rdf_rmax=10.5, dih_bins=72, pairs=True, dihedrals=True, shape=True):
        """Section 5 observables of the current positions (md_observables): a dict of numpy
        arrays pair_counts [n_boxes, rdf_bins], dihedral_hist [n_boxes, dih_bins],
        dihedral_classes [n_boxes, 3] (trans, gauche+, gauche-) and chain_shape
        [n_chains, 4] (R_g^2, end-to-end vector)."""
        nb, nch = self.n_boxes, int(self.cfg.n_chains.sum())
        cfg = md_obs_config(rdf_bins=int(rdf_bins), rdf_rmax=float(rdf_rmax), dih_bins=int(dih_bins))
        # never empty, so a bad bin count reaches the library's own check rather than a null pointer
        pc = torch.zeros(max(nb * rdf_bins, 1), dtype=torch.int64, device=self.device)
        dc = torch.zeros(max(nb * (dih_bins + 3), 1), dtype=torch.int64, device=self.device)
        cs = torch.zeros(nch * 4, dtype=torch.float64, device=self.device)
        _check(load().md_observables(self.ctx, ctypes.byref(cfg), pc.data_ptr() if pairs else None,
                                     dc.data_ptr() if dihedrals else None, cs.data_ptr() if shape else None),
               "md_observables", self.ctx)
        torch.cuda.synchronize(self.device)
        out = {}
        if pairs:
            out["pair_counts"] = pc.cpu().numpy().view(np.uint64).reshape(nb, rdf_bins)
        if dihedrals:
            d = dc.cpu().numpy().view(np.uint64).reshape(nb, dih_bins + 3)
            out["dihedral_hist"], out["dihedral_classes"] = d[:, :dih_bins], d[:, dih_bins:]
        if shape:
            out["chain_shape"] = cs.cpu().numpy().reshape(nch, 4)
        return out

    # --- device views copied to host ---
    def _ws_view(self, ptr, count, dtype):
        """A host copy of count elements at device address ptr inside the workspace."""
        itemsize = torch.empty(0, dtype=dtype).element_size()
        if self.workspace is None:   # the library's own array: copy with the HIP runtime
            out = torch.empty(count, dtype=dtype)
            _hip_copy_to_host(out.data_ptr(), ptr, count * itemsize)
            return out
        off = ptr - self.workspace.data_ptr()
        assert 0 <= off and off + count * itemsize <= self.workspace.numel()
        return self.workspace[off:off + count * itemsize].view(dtype)

    def bins(self):
        cs, ca, n_cells = md_bins(self.ctx)
        torch.cuda.synchronize(self.device)
        start = self._ws_view(cs, n_cells + 1, torch.int32).cpu().numpy()
        atoms = self._ws_view(ca, self.N, torch.int32).cpu().numpy()
        return start, atoms

    def forces(self, lj_only=False):
        ptr, fp32 = (md_forces_lj if lj_only else md_forces)(self.ctx)
        torch.cuda.synchronize(self.device)
        t = self._ws_view(ptr, 3 * self.N, torch.float32 if fp32 else torch.float64)
        return t.cpu().numpy().astype(np.float64).reshape(3, self.N)

    def state(self):
        torch.cuda.synchronize(self.device)
        return self.pos.cpu().numpy().copy(), self.vel.cpu().numpy().copy()

    def close(self):
        if self.ctx:
            md_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
