"""Python binding of the MI355X plane-wave Kohn-Sham energy/force engine.

Argument marshalling only: every step of the computation runs in the HIP
kernels of libsgo.so (built by `paper_1603_02732_amd.build`).  Importing the
package fails loudly if the library is missing; there is no CPU fallback.

Names mirror include/sgo.h.  `Context` wraps one structure (sgo_ctx),
`Batch` a population of candidates solved together (sgo_batch).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgo.so")

SGO_OK, SGO_EINVAL, SGO_ENOMEM, SGO_EDEVICE, SGO_ENOTCONV, SGO_ENUMERIC, SGO_ESTATE = \
    0, -1, -2, -3, -4, -5, -6
SGO_FP64, SGO_FP32, SGO_FP32_BF16PROJ = 0, 1, 2
SGO_LOCAL_AH, SGO_LOCAL_GAUSS = 0, 1
SGO_OCC_FIXED, SGO_OCC_FERMI = 0, 1
SGO_DE_TRIANGLE, SGO_DE_CLASSIC = 0, 1
SGO_DE_PLANE, SGO_DE_SPHERE = 0, 1
_STATUS = {0: "SGO_OK", -1: "SGO_EINVAL", -2: "SGO_ENOMEM", -3: "SGO_EDEVICE",
           -4: "SGO_ENOTCONV", -5: "SGO_ENUMERIC", -6: "SGO_ESTATE"}


class SgoError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_STATUS.get(code, code), msg))
        self.code = code


class sgo_species(ctypes.Structure):
    _fields_ = [("Z", ctypes.c_double), ("local_kind", ctypes.c_int),
                ("p", ctypes.c_double * 3), ("nkb", ctypes.c_int),
                ("kb_l", ctypes.c_int * 4), ("kb_r", ctypes.c_double * 4),
                ("kb_h", ctypes.c_double * 4), ("rho0_width", ctypes.c_double)]


class sgo_scf_opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("ncg", ctypes.c_int), ("ncg_first", ctypes.c_int),
                ("tol_e", ctypes.c_double), ("tol_rho", ctypes.c_double),
                ("mix_alpha", ctypes.c_double), ("kerker_q0", ctypes.c_double),
                ("history", ctypes.c_int), ("seed", ctypes.c_uint), ("use_graph", ctypes.c_int),
                ("cg_tol", ctypes.c_double)]


class sgo_scf_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("de", ctypes.c_double), ("drho", ctypes.c_double)]


class sgo_energy_terms(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("total", "kinetic", "nonlocal", "local", "hartree", "xc", "ewald", "entropy",
                 "band", "fermi")]


_lib = None


# caller allocator hooks: void* alloc(size_t bytes, void* user); void dealloc(void* p, void* user)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class sgo_de_opts(ctypes.Structure):
    _fields_ = [("mutation", ctypes.c_int), ("crossover", ctypes.c_int), ("F", ctypes.c_double),
                ("fitness_shift", ctypes.c_int), ("relax_steps", ctypes.c_int),
                ("dmin", ctypes.c_double), ("sim_tol", ctypes.c_double), ("attempts", ctypes.c_int)]


class sgo_de_draw(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int * 3), ("normal", ctypes.c_double * 3),
                ("axis", ctypes.c_double * 3), ("offset", ctypes.c_double * 3),
                ("radius", ctypes.c_double)]


class TorchArenas:
    """Allocator hooks that take the structures' device arenas from PyTorch's
    caching allocator (uint8 tensors kept alive until the library frees them).
    Keep the object alive as long as the handle uses it."""

    def __init__(self, device=0):
        import torch
        self._torch = torch
        self.device = device
        self.live = {}
        self.error = None
        # initialise PyTorch's device state here, not inside a callback
        torch.zeros(1, device="cuda:%d" % device)
        self.alloc = ALLOC_FN(self._alloc)
        self.free = FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        # an exception must not cross the C boundary: NULL reports failure
        try:
            t = self._torch.empty(int(nbytes) + 256, dtype=self._torch.uint8,
                                  device="cuda:%d" % self.device)
        except Exception as e:  # out of memory, no device
            self.error = e
            return None
        p = (t.data_ptr() + 255) // 256 * 256
        self.live[p] = t
        return p

    def _free(self, p, user):
        self.live.pop(p, None)


def load_library(path=None):
    """Load libsgo.so (raises OSError if it is not built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise OSError("libsgo.so not built; run python -m paper_1603_02732_amd.build")
    # One HIP runtime per process: PyTorch carries its own copy of the HIP
    # runtime under the same soname, and whichever is loaded first serves
    # both.  Loading PyTorch's first (when it is installed) lets tensors,
    # streams and allocator hooks be shared with this library in any import
    # order; importing torch does not initialise a device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(p)
    P, I, D, U = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    sig = {
        "sgo_default_opts": (None, [ctypes.POINTER(sgo_scf_opts)]),
        "sgo_version": (ctypes.c_char_p, []),
        "sgo_create": (I, [ctypes.POINTER(P), I, I]),
        "sgo_destroy": (I, [P]),
        "sgo_set_stream": (I, [P, P]),
        "sgo_set_species": (I, [P, I, ctypes.POINTER(sgo_species)]),
        "sgo_set_cell": (I, [P, dp]),
        "sgo_set_atoms": (I, [P, I, ip, dp]),
        "sgo_set_cutoff": (I, [P, D, ip, I, I, D]),
        "sgo_scf": (I, [P, ctypes.POINTER(sgo_scf_opts), ctypes.POINTER(sgo_scf_info)]),
        "sgo_energy": (I, [P, dp, ctypes.POINTER(sgo_energy_terms)]),
        "sgo_forces": (I, [P, dp]),
        "sgo_stress": (I, [P, dp, dp]),
        "sgo_eigenvalues": (I, [P, dp, dp]),
        "sgo_adjoint": (I, [P, D, dp, dp]),
        "sgo_reset": (I, [P]),
        "sgo_basis_size": (I, [P, ip, ip]),
        "sgo_basis_millers": (I, [P, ip]),
        "sgo_apply_h": (I, [P, dp, I, dp, dp]),
        "sgo_get_density": (I, [P, dp, dp]),
        "sgo_last_error": (ctypes.c_char_p, [P]),
        "sgo_grid_info": (I, [P, ip]),
        "sgo_set_tuning": (I, [ctypes.c_char_p, I]),
        "sgo_get_tuning": (I, [ctypes.c_char_p]),
        "sgo_subspace_solve": (I, [I, I, I, dp, dp, dp, dp, I, dp,
                                   ctypes.POINTER(ctypes.c_longlong)]),
        "sgo_subspace_solve_noalloc": (I, [I, I, I, P, P, P, P, P, P]),
        "sgo_profile_begin": (I, [ctypes.c_char_p]),
        "sgo_profile_end": (I, [ip, dp, ctypes.POINTER(ctypes.c_longlong),
                                ctypes.POINTER(ctypes.c_longlong), dp]),
        "sgo_batch_create": (I, [ctypes.POINTER(P), I, I, I]),
        "sgo_batch_destroy": (I, [P]),
        "sgo_batch_set_stream": (I, [P, P]),
        "sgo_batch_set_species": (I, [P, I, ctypes.POINTER(sgo_species)]),
        "sgo_batch_add": (I, [P, dp, I, ip, dp, D, ip, I, I, D, ip]),
        "sgo_batch_set_atoms": (I, [P, I, dp]),
        "sgo_batch_scf": (I, [P, ctypes.POINTER(sgo_scf_opts), dp, dp, ip]),
        "sgo_batch_info": (I, [P, I, ctypes.POINTER(sgo_scf_info)]),
        "sgo_batches_scf": (I, [ctypes.POINTER(P), I, ctypes.POINTER(sgo_scf_opts), dp, dp, ip]),
        "sgo_batch_size": (I, [P, ip]),
        "sgo_set_allocator": (I, [P, ALLOC_FN, FREE_FN, P]),
        "sgo_batch_set_allocator": (I, [P, ALLOC_FN, FREE_FN, P]),
        "sgo_batch_stress": (I, [P, dp]),
        "sgo_batch_reset": (I, [P]),
        "sgo_batch_relax_cg": (I, [P, I, ctypes.POINTER(sgo_scf_opts), dp, dp, dp, ip]),
        "sgo_batch_get_state": (I, [P, I, ip, ip, dp, dp, dp, dp, dp,
                                    ctypes.POINTER(sgo_energy_terms)]),
        "sgo_set_kpoints": (I, [P, I, dp, dp]),
        "sgo_kpoint_eigenvalues": (I, [P, dp, dp]),
        "sgo_batch_get_input_density": (I, [P, I, dp]),
        "sgo_batch_last_error": (ctypes.c_char_p, [P]),
        "sgo_de_mutate": (I, [I, dp, dp, dp, D, D, D, I, D, dp]),
        "sgo_de_cross_plane": (I, [I, ip, dp, dp, dp, dp, dp, ip, dp]),
        "sgo_de_cross_sphere": (I, [I, ip, dp, dp, dp, D, dp, ip]),
        "sgo_de_min_distance": (I, [dp, I, dp, dp]),
        "sgo_de_similarity": (I, [dp, I, dp, dp, dp]),
        "sgo_de_init_positions": (I, [dp, I, I, dp, D, dp, I, dp, ip]),
        "sgo_de_select": (I, [I, dp, dp, ip, ip]),
        "sgo_de_jitter_cell": (I, [dp, D, dp, dp]),
        "sgo_batch_relax_pcg": (I, [P, I, I, ctypes.POINTER(sgo_scf_opts), dp, dp, dp, dp, ip]),
        "sgo_ff_morse": (I, [dp, I, dp, dp, dp, dp]),
        "sgo_ff_hessian": (I, [dp, I, dp, dp, dp]),
        "sgo_ff_fit": (I, [dp, I, I, dp, dp, dp]),
        "sgo_ff_preconditioner": (I, [I, dp, dp]),
        "sgo_ff_guided_curve": (I, [dp, I, dp, dp, I, dp, ip]),
        "sgo_batch_relax_cls": (I, [P, I, ctypes.POINTER(sgo_scf_opts), dp, dp, dp, dp, ip]),
        "sgo_batch_de_generation": (I, [P, ctypes.POINTER(sgo_de_opts),
                                        ctypes.POINTER(sgo_scf_opts), dp, dp,
                                        ctypes.POINTER(sgo_de_draw), dp, ip, dp, dp, dp, ip, ip]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def default_opts(**kw):
    o = sgo_scf_opts()
    load_library().sgo_default_opts(ctypes.byref(o))
    names = {n for n, _ in sgo_scf_opts._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError("unknown SCF option %r" % k)
        setattr(o, k, v)
    return o


def make_species(params):
    """sgo_species from a species parameter dict (see workloads.species)."""
    s = sgo_species()
    s.Z = params["Z"]
    loc = params["local"]
    if loc["kind"] == "ah":
        s.local_kind = SGO_LOCAL_AH
        s.p[0], s.p[1], s.p[2] = loc["alpha"], loc["v1"], loc["v2"]
    else:
        s.local_kind = SGO_LOCAL_GAUSS
        s.p[0], s.p[1], s.p[2] = loc["rloc"], loc["c1"], loc["c2"]
    s.nkb = len(params["kb"])
    for k, ch in enumerate(params["kb"]):
        s.kb_l[k], s.kb_r[k], s.kb_h[k] = ch["l"], ch["r"], ch["h"]
    s.rho0_width = params.get("rho0_width", 0.5)
    return s


def _occ(system):
    occ = system["occupation"]
    if occ["kind"] == "fixed":
        return SGO_OCC_FIXED, 0.0
    return SGO_OCC_FERMI, float(occ["sigma"])


class Context:
    """One structure (sgo_ctx)."""

    def __init__(self, device=0, precision=SGO_FP64):
        self._lib = load_library()
        h = ctypes.c_void_p()
        self._check(self._lib.sgo_create(ctypes.byref(h), device, precision), None)
        self._h = h
        self.natoms = 0
        self.species_ids = {}
        # bumped by every call that changes the structure or the held state,
        # so that a deferred adjoint can tell whether its solve is still held
        self.generation = 0

    def _check(self, rc, h=-1, allow=()):
        if rc != SGO_OK and rc not in allow:
            msg = self._lib.sgo_last_error(self._h if h == -1 else h)
            raise SgoError(rc, (msg or b"").decode())
        return rc

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sgo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream_ptr):
        self._check(self._lib.sgo_set_stream(self._h, ctypes.c_void_p(stream_ptr)))

    def set_species(self, sid, params):
        self.generation += 1
        sp = make_species(params)
        self._check(self._lib.sgo_set_species(self._h, sid, ctypes.byref(sp)))

    def set_allocator(self, hooks):
        """Route the arena allocations through `hooks` (e.g. TorchArenas());
        None restores hipMalloc."""
        self._hooks = hooks
        if hooks is None:
            self._check(self._lib.sgo_set_allocator(self._h, ALLOC_FN(), FREE_FN(), None))
        else:
            self._check(self._lib.sgo_set_allocator(self._h, hooks.alloc, hooks.free, None))

    def set_cell(self, lattice):
        self.generation += 1
        a = np.ascontiguousarray(lattice, dtype=np.float64).reshape(9)
        self._check(self._lib.sgo_set_cell(self._h, _dptr(a)))

    def set_atoms(self, species, positions):
        self.generation += 1
        s = np.ascontiguousarray(species, dtype=np.int32)
        p = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1)
        self._check(self._lib.sgo_set_atoms(self._h, len(s), _iptr(s), _dptr(p)))
        self.natoms = len(s)
        self.atom_species = s.copy()

    def set_cutoff(self, ecut, grid, nbands, occ_kind=SGO_OCC_FIXED, sigma=0.0):
        self.generation += 1
        g = np.ascontiguousarray(grid, dtype=np.int32)
        self._check(self._lib.sgo_set_cutoff(self._h, float(ecut), _iptr(g), int(nbands),
                                             int(occ_kind), float(sigma)))
        self.nbands = int(nbands)
        self.grid = tuple(int(x) for x in grid)

    def load_system(self, system):
        """Species, cell, atoms and cutoff from a workloads system dict."""
        names = sorted(system["species"])
        self.species_ids = {n: i for i, n in enumerate(names)}
        for n in names:
            self.set_species(self.species_ids[n], system["species"][n])
        self.set_cell(system["lattice"])
        self.set_atoms([self.species_ids[s] for s in system["symbols"]], system["positions"])
        kind, sigma = _occ(system)
        self.set_cutoff(system["ecut"], system["grid"], system["nbands"], kind, sigma)
        return self

    def scf(self, opts=None, allow_notconv=False, **kw):
        o = opts if opts is not None else default_opts(**kw)
        info = sgo_scf_info()
        allow = (SGO_ENOTCONV,) if allow_notconv else ()
        self.generation += 1
        rc = self._check(self._lib.sgo_scf(self._h, ctypes.byref(o), ctypes.byref(info)),
                         allow=allow)
        return {"status": rc, "iterations": info.iterations, "converged": bool(info.converged),
                "de": info.de, "drho": info.drho}

    def set_kpoints(self, kfrac, weights):
        """k-point sampling (FP64 handles): kfrac (nk, 3) in units of the
        reciprocal lattice vectors, weights (nk,); an empty list returns to
        the Gamma-point path."""
        k = np.ascontiguousarray(np.asarray(kfrac, dtype=np.float64).reshape(-1, 3))
        w = np.ascontiguousarray(np.asarray(weights, dtype=np.float64).reshape(-1))
        if len(k) != len(w):
            raise ValueError("one weight per k-point")
        self.generation += 1
        self.nk = len(k)
        self._check(self._lib.sgo_set_kpoints(self._h, len(k), _dptr(k) if len(k) else None,
                                              _dptr(w) if len(w) else None))

    def kpoint_eigenvalues(self):
        """(eigenvalues, occupations), each (nk, nbands), of the last k-point solve."""
        nb = self.geometry()["nbands"]
        e = np.zeros((self.nk, nb))
        o = np.zeros((self.nk, nb))
        self._check(self._lib.sgo_kpoint_eigenvalues(self._h, _dptr(e), _dptr(o)))
        return e, o

    def energy(self):
        e = ctypes.c_double()
        t = sgo_energy_terms()
        self._check(self._lib.sgo_energy(self._h, ctypes.byref(e), ctypes.byref(t)))
        return e.value, {n: getattr(t, n) for n, _ in sgo_energy_terms._fields_}

    def forces(self):
        f = np.zeros((self.natoms, 3))
        self._check(self._lib.sgo_forces(self._h, _dptr(f)))
        return f

    def adjoint(self, gE=1.0, lattice=False):
        """gE * dE/dR [natoms, 3]; with lattice=True also gE * dE/dA [3, 3]
        (Cartesian positions and Miller set fixed)."""
        g = np.zeros((self.natoms, 3))
        if not lattice:
            self._check(self._lib.sgo_adjoint(self._h, float(gE), _dptr(g), None))
            return g
        gl = np.zeros((3, 3))
        self._check(self._lib.sgo_adjoint(self._h, float(gE), _dptr(g), _dptr(gl)))
        return g, gl

    def stress(self, parts=False):
        """Fixed-basis stress [3, 3] (Ha/bohr^3); with parts=True also a dict
        of the kinetic, nonlocal, hartree, local, xc and ewald parts."""
        s = np.zeros((3, 3))
        if not parts:
            self._check(self._lib.sgo_stress(self._h, _dptr(s), None))
            return s
        p = np.zeros((6, 3, 3))
        self._check(self._lib.sgo_stress(self._h, _dptr(s), _dptr(p)))
        names = ("kinetic", "nonlocal", "hartree", "local", "xc", "ewald")
        return s, {n: p[k] for k, n in enumerate(names)}

    def eigenvalues(self):
        e = np.zeros(self.nbands)
        o = np.zeros(self.nbands)
        self._check(self._lib.sgo_eigenvalues(self._h, _dptr(e), _dptr(o)))
        return e, o

    def basis(self):
        n = ctypes.c_int()
        npj = ctypes.c_int()
        self._check(self._lib.sgo_basis_size(self._h, ctypes.byref(n), ctypes.byref(npj)))
        m = np.zeros((n.value, 3), dtype=np.int32)
        self._check(self._lib.sgo_basis_millers(self._h, _iptr(m)))
        return m, npj.value

    def apply_h(self, veff_zyx, psi):
        """H[V] psi for packed bands psi (nb, 2*npw_half); veff indexed [z][y][x]."""
        self.generation += 1  # the library drops the held solve
        v = np.ascontiguousarray(veff_zyx, dtype=np.float64)
        x = np.ascontiguousarray(psi, dtype=np.float64)
        out = np.zeros_like(x)
        self._check(self._lib.sgo_apply_h(self._h, _dptr(v), x.shape[0], _dptr(x), _dptr(out)))
        return out

    def density(self):
        n = int(np.prod(self.grid))
        rho = np.zeros(n)
        veff = np.zeros(n)
        self._check(self._lib.sgo_get_density(self._h, _dptr(rho), _dptr(veff)))
        shape = (self.grid[2], self.grid[1], self.grid[0])
        return rho.reshape(shape), veff.reshape(shape)

    def reset(self):
        self.generation += 1
        self._check(self._lib.sgo_reset(self._h))

    def geometry(self):
        v = np.zeros(10, dtype=np.int32)
        self._check(self._lib.sgo_grid_info(self._h, _iptr(v)))
        keys = ("N1", "N2", "N3", "ntot", "npw_half", "nbands", "npair", "nst", "nsp", "nproj")
        return {k: int(x) for k, x in zip(keys, v)}

    def profile_begin(self, kernel):
        return profile_begin(kernel)

    def profile_end(self):
        return profile_end()


def subspace_solve(S, H=None, mode=3, reps=1, device=0, clocks=False):
    """Cholesky orthonormalisation (+ subspace diagonalisation for mode 3) of
    host FP64 matrices on the GPU.  Returns (M, eps, ms_per_call, clocks)."""
    lib = load_library()
    S = np.ascontiguousarray(S, dtype=np.float64)
    n = S.shape[0]
    Hc = None if H is None else np.ascontiguousarray(H, dtype=np.float64)
    M = np.zeros((n, n))
    eps = np.zeros(n)
    ms = ctypes.c_double()
    clk = (ctypes.c_longlong * 6)()
    rc = lib.sgo_subspace_solve(device, n, mode, _dptr(S), _dptr(Hc) if Hc is not None else None,
                                _dptr(M), _dptr(eps), reps, ctypes.byref(ms),
                                clk if clocks else None)
    if rc != SGO_OK:
        raise SgoError(rc, (lib.sgo_last_error(None) or b"").decode())
    return M, eps, ms.value, list(clk) if clocks else None


def subspace_solve_noalloc(S, H, M, eps, n, mode=3, status=None, stream=None, device=0):
    """The subspace step on device arrays with the library's fixed workspace
    (no allocation).  S, H, M, eps, status are device addresses (ints, e.g.
    tensor.data_ptr()); H may be None for mode 1, status None to wait and
    raise on failure.  stream: a hipStream_t address or None."""
    lib = load_library()
    rc = lib.sgo_subspace_solve_noalloc(device, n, mode, S, H, M, eps, status, stream)
    if rc != SGO_OK:
        raise SgoError(rc, (lib.sgo_last_error(None) or b"").decode())


def set_tuning(key, value):
    """Set a launch-schedule parameter (see sgo.h); value <= 0 restores the default."""
    rc = load_library().sgo_set_tuning(key.encode(), int(value))
    if rc != SGO_OK:
        raise SgoError(rc, "unknown tuning key %r" % key)


def get_tuning(key):
    return load_library().sgo_get_tuning(key.encode())


def profile_begin(kernel):
    """Time every launch of `kernel` with HIP events until profile_end()."""
    rc = load_library().sgo_profile_begin(kernel.encode())
    if rc != SGO_OK:
        raise SgoError(rc, "profile_begin")


def profile_end():
    n = ctypes.c_int()
    ms = ctypes.c_double()
    cl = ctypes.c_longlong()
    cr = ctypes.c_longlong()
    um = ctypes.c_double()
    lib = load_library()
    rc = lib.sgo_profile_end(ctypes.byref(n), ctypes.byref(ms), ctypes.byref(cl), ctypes.byref(cr),
                             ctypes.byref(um))
    if rc != SGO_OK:
        raise SgoError(rc, (lib.sgo_last_error(None) or b"").decode())
    return {"launches": n.value, "ms": ms.value, "cand_launches": cl.value, "cand_rows": cr.value,
            "union_ms": um.value}


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a if shape is None else a.reshape(shape)


def de_mutate(x1, x2, x3, f, scheme=SGO_DE_TRIANGLE, F=0.5):
    """Mutant of three donor structures (Eq. 2 triangle, or Eq. 1)."""
    x1, x2, x3 = _f64(x1), _f64(x2), _f64(x3)
    v = np.zeros_like(x1)
    rc = load_library().sgo_de_mutate(x1.size, _dptr(x1), _dptr(x2), _dptr(x3), float(f[0]),
                                      float(f[1]), float(f[2]), int(scheme), float(F), _dptr(v))
    if rc != SGO_OK:
        raise SgoError(rc, "de_mutate")
    return v


def de_cross_plane(p1, p2, species, normal, axis):
    """Plane cut-and-splice: (child, source [natoms, 2], theta) or None when
    no orientation gives P1's composition."""
    p1, p2 = _f64(p1), _f64(p2)
    n = p1.shape[0]
    sp = np.ascontiguousarray(species, dtype=np.int32)
    child = np.zeros((n, 3))
    src = np.zeros((n, 2), dtype=np.int32)
    th = ctypes.c_double()
    rc = load_library().sgo_de_cross_plane(n, _iptr(sp), _dptr(p1), _dptr(p2),
                                           _dptr(_f64(normal)), _dptr(_f64(axis)), _dptr(child),
                                           _iptr(src), ctypes.byref(th))
    if rc == SGO_ENUMERIC:
        return None
    if rc != SGO_OK:
        raise SgoError(rc, "de_cross_plane")
    return child, src, th.value


def de_cross_sphere(p1, p2, species, offset, radius):
    """Sphere cut-and-splice: (child, source [natoms, 2])."""
    p1, p2 = _f64(p1), _f64(p2)
    n = p1.shape[0]
    sp = np.ascontiguousarray(species, dtype=np.int32)
    child = np.zeros((n, 3))
    src = np.zeros((n, 2), dtype=np.int32)
    rc = load_library().sgo_de_cross_sphere(n, _iptr(sp), _dptr(p1), _dptr(p2),
                                            _dptr(_f64(offset)), float(radius), _dptr(child),
                                            _iptr(src))
    if rc != SGO_OK:
        raise SgoError(rc, "de_cross_sphere")
    return child, src


def de_min_distance(lattice, pos):
    pos = _f64(pos)
    d = ctypes.c_double()
    rc = load_library().sgo_de_min_distance(_dptr(_f64(lattice, 9)), pos.shape[0], _dptr(pos),
                                            ctypes.byref(d))
    if rc != SGO_OK:
        raise SgoError(rc, "de_min_distance")
    return d.value


def de_similarity(lattice, pa, pb):
    pa, pb = _f64(pa), _f64(pb)
    d = ctypes.c_double()
    rc = load_library().sgo_de_similarity(_dptr(_f64(lattice, 9)), pa.shape[0], _dptr(pa),
                                          _dptr(pb), ctypes.byref(d))
    if rc != SGO_OK:
        raise SgoError(rc, "de_similarity")
    return d.value


def de_init_positions(lattice, natoms, region, params, dmin, uniforms):
    """Random placement; (positions [natoms, 3], uniforms used) or None when
    the uniforms run out."""
    u = _f64(uniforms)
    par = _f64(list(params) + [0.0])
    pos = np.zeros((natoms, 3))
    used = ctypes.c_int()
    rc = load_library().sgo_de_init_positions(_dptr(_f64(lattice, 9)), int(natoms), int(region),
                                              _dptr(par), float(dmin), _dptr(u), u.size,
                                              _dptr(pos), ctypes.byref(used))
    if rc == SGO_ENUMERIC:
        return None
    if rc != SGO_OK:
        raise SgoError(rc, "de_init_positions")
    return pos, used.value


def de_jitter_cell(lattice, delta, u3):
    """Lattice vectors scaled by 1 + delta (2 u_k - 1)."""
    out = np.zeros(9)
    rc = load_library().sgo_de_jitter_cell(_dptr(_f64(lattice, 9)), float(delta),
                                           _dptr(_f64(u3)), _dptr(out))
    if rc != SGO_OK:
        raise SgoError(rc, "de_jitter_cell")
    return out.reshape(3, 3)


def de_select(e_parent, e_child, child_status=None):
    ep, ec = _f64(e_parent), _f64(e_child)
    take = np.zeros(ep.size, dtype=np.int32)
    st = None if child_status is None else np.ascontiguousarray(child_status, dtype=np.int32)
    rc = load_library().sgo_de_select(ep.size, _dptr(ep), _dptr(ec),
                                      None if st is None else _iptr(st), _iptr(take))
    if rc != SGO_OK:
        raise SgoError(rc, "de_select")
    return take


def ff_morse(lattice, pos, params):
    """Morse pair energy and forces (the PCG preconditioner's force field)."""
    pos = _f64(pos)
    e = ctypes.c_double()
    F = np.zeros_like(pos)
    rc = load_library().sgo_ff_morse(_dptr(_f64(lattice, 9)), pos.shape[0], _dptr(pos),
                                     _dptr(_f64(params)), ctypes.byref(e), _dptr(F))
    if rc != SGO_OK:
        raise SgoError(rc, "ff_morse")
    return e.value, F


def ff_hessian(lattice, pos, params):
    pos = _f64(pos)
    m = pos.size
    H = np.zeros((m, m))
    rc = load_library().sgo_ff_hessian(_dptr(_f64(lattice, 9)), pos.shape[0], _dptr(pos),
                                       _dptr(_f64(params)), _dptr(H))
    if rc != SGO_OK:
        raise SgoError(rc, "ff_hessian")
    return H


def ff_fit(lattice, positions, forces):
    """(D, a, r0) fitted to lists of [natoms, 3] positions and forces."""
    X = np.ascontiguousarray(np.stack([np.asarray(p, dtype=np.float64) for p in positions]))
    F = np.ascontiguousarray(np.stack([np.asarray(f, dtype=np.float64) for f in forces]))
    prm = np.zeros(3)
    rc = load_library().sgo_ff_fit(_dptr(_f64(lattice, 9)), X.shape[1], X.shape[0], _dptr(X),
                                   _dptr(F), _dptr(prm))
    if rc != SGO_OK:
        raise SgoError(rc, "ff_fit")
    return prm


def ff_preconditioner(H):
    H = _f64(H)
    P = np.zeros_like(H)
    rc = load_library().sgo_ff_preconditioner(H.shape[0], _dptr(H), _dptr(P))
    if rc != SGO_OK:
        raise SgoError(rc, "ff_preconditioner")
    return P


def ff_guided_curve(lattice, pos, params):
    """Nodes [K, natoms, 3] of the CLS guided curve."""
    pos = _f64(pos)
    nodes = np.zeros((201,) + pos.shape)
    k = ctypes.c_int()
    rc = load_library().sgo_ff_guided_curve(_dptr(_f64(lattice, 9)), pos.shape[0],
                                            _dptr(_f64(params)), _dptr(pos), 201, _dptr(nodes),
                                            ctypes.byref(k))
    if rc != SGO_OK:
        raise SgoError(rc, "ff_guided_curve")
    return nodes[:k.value].copy()


def batches_scf(batches, opts=None, **kw):
    """Solve several Batch objects at once, each from its own host thread on
    its own stream (set_stream each to a distinct stream first).  Returns
    energies, forces (list of (natoms, 3)) and status concatenated in batch
    order."""
    o = opts if opts is not None else default_opts(**kw)
    lib = load_library()
    hs = (ctypes.c_void_p * len(batches))(*[b._h.value for b in batches])
    n = sum(len(b.natoms) for b in batches)
    nat = [na for b in batches for na in b.natoms]
    e = np.zeros(n)
    f = np.zeros(3 * sum(nat))
    st = np.zeros(n, dtype=np.int32)
    rc = lib.sgo_batches_scf(hs, len(batches), ctypes.byref(o), _dptr(e), _dptr(f), _iptr(st))
    if rc not in (SGO_OK, SGO_ENOTCONV, SGO_ENUMERIC):
        raise SgoError(rc, "; ".join((lib.sgo_batch_last_error(b._h) or b"").decode() for b in batches))
    forces, off = [], 0
    for na in nat:
        forces.append(f[off:off + 3 * na].reshape(na, 3))
        off += 3 * na
    return e, forces, st


def de_opts(mutation=SGO_DE_TRIANGLE, crossover=SGO_DE_PLANE, F=0.5, fitness_shift=1,
            relax_steps=5, dmin=2.0, sim_tol=0.0, attempts=4):
    o = sgo_de_opts()
    o.mutation, o.crossover, o.F, o.fitness_shift = mutation, crossover, F, fitness_shift
    o.relax_steps, o.dmin, o.sim_tol, o.attempts = relax_steps, dmin, sim_tol, attempts
    return o


def de_draws(d):
    """sgo_de_draw array [n * attempts] from a dict of arrays: r [n, a, 3],
    normal, axis, offset [n, a, 3], radius [n, a]."""
    r = np.asarray(d["r"])
    n, a = r.shape[:2]
    arr = (sgo_de_draw * (n * a))()
    for i in range(n):
        for k in range(a):
            e = arr[i * a + k]
            for c in range(3):
                e.r[c] = int(r[i, k, c])
                e.normal[c] = float(d["normal"][i][k][c])
                e.axis[c] = float(d["axis"][i][k][c])
                e.offset[c] = float(d["offset"][i][k][c])
            e.radius = float(d["radius"][i][k])
    return arr


class Batch:
    """A population of candidates solved together (sgo_batch)."""

    def __init__(self, capacity, device=0, precision=SGO_FP32):
        self._lib = load_library()
        h = ctypes.c_void_p()
        rc = self._lib.sgo_batch_create(ctypes.byref(h), device, precision, capacity)
        if rc != SGO_OK:
            raise SgoError(rc, (self._lib.sgo_batch_last_error(None) or b"").decode())
        self._h = h
        self.natoms = []
        self.species_ids = {}

    def _check(self, rc, allow=()):
        if rc != SGO_OK and rc not in allow:
            raise SgoError(rc, (self._lib.sgo_batch_last_error(self._h) or b"").decode())
        return rc

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sgo_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_allocator(self, hooks):
        """Route the candidates' arena allocations through `hooks`."""
        self._hooks = hooks
        if hooks is None:
            self._check(self._lib.sgo_batch_set_allocator(self._h, ALLOC_FN(), FREE_FN(), None))
        else:
            self._check(self._lib.sgo_batch_set_allocator(self._h, hooks.alloc, hooks.free, None))

    def set_stream(self, stream_ptr):
        self._check(self._lib.sgo_batch_set_stream(self._h, ctypes.c_void_p(stream_ptr)))

    def add_system(self, system):
        for n in sorted(system["species"]):
            if n not in self.species_ids:
                sid = len(self.species_ids)
                self.species_ids[n] = sid
                sp = make_species(system["species"][n])
                self._check(self._lib.sgo_batch_set_species(self._h, sid, ctypes.byref(sp)))
        lat = np.ascontiguousarray(system["lattice"], dtype=np.float64).reshape(9)
        spec = np.ascontiguousarray([self.species_ids[s] for s in system["symbols"]],
                                    dtype=np.int32)
        pos = np.ascontiguousarray(system["positions"], dtype=np.float64).reshape(-1)
        grid = np.ascontiguousarray(system["grid"], dtype=np.int32)
        kind, sigma = _occ(system)
        idx = ctypes.c_int()
        self._check(self._lib.sgo_batch_add(self._h, _dptr(lat), len(spec), _iptr(spec),
                                            _dptr(pos), float(system["ecut"]), _iptr(grid),
                                            int(system["nbands"]), kind, sigma,
                                            ctypes.byref(idx)))
        self.natoms.append(len(spec))
        return idx.value

    def set_atoms(self, i, positions):
        p = np.ascontiguousarray(positions, dtype=np.float64).reshape(-1)
        self._check(self._lib.sgo_batch_set_atoms(self._h, int(i), _dptr(p)))

    def scf(self, opts=None, **kw):
        o = opts if opts is not None else default_opts(**kw)
        n = len(self.natoms)
        e = np.zeros(n)
        f = np.zeros(sum(self.natoms) * 3)
        st = np.zeros(n, dtype=np.int32)
        rc = self._lib.sgo_batch_scf(self._h, ctypes.byref(o), _dptr(e), _dptr(f), _iptr(st))
        if rc not in (SGO_OK, SGO_ENOTCONV, SGO_ENUMERIC):
            self._check(rc)
        forces, off = [], 0
        for na in self.natoms:
            forces.append(f[off:off + 3 * na].reshape(na, 3))
            off += 3 * na
        return e, forces, st

    def reset(self):
        self._check(self._lib.sgo_batch_reset(self._h))

    def state(self, i):
        """Converged state of candidate i: sizes, Miller indices, packed bands,
        eigenvalues, occupations, density, V_eff (both [z][y][x]) and energy terms."""
        info = np.zeros(10, dtype=np.int32)
        self._check(self._lib.sgo_batch_get_state(self._h, int(i), _iptr(info), None, None, None,
                                                  None, None, None, None))
        N1, N2, N3, ntot, nh, nb = (int(x) for x in info[:6])
        m = np.zeros((nh, 3), dtype=np.int32)
        psi = np.zeros((nb, 2 * nh))
        eig = np.zeros(nb)
        occ = np.zeros(nb)
        rho = np.zeros(ntot)
        veff = np.zeros(ntot)
        t = sgo_energy_terms()
        self._check(self._lib.sgo_batch_get_state(self._h, int(i), None, _iptr(m), _dptr(psi),
                                                  _dptr(eig), _dptr(occ), _dptr(rho),
                                                  _dptr(veff), ctypes.byref(t)))
        rho_in = np.zeros(ntot)
        self._check(self._lib.sgo_batch_get_input_density(self._h, int(i), _dptr(rho_in)))
        return {"grid": (N1, N2, N3), "millers": m, "psi": psi, "eig": eig, "occ": occ,
                "rho": rho.reshape(N3, N2, N1), "veff": veff.reshape(N3, N2, N1),
                "rho_in": rho_in.reshape(N3, N2, N1),
                "terms": {n: getattr(t, n) for n, _ in sgo_energy_terms._fields_}}

    def relax_cg(self, nsteps, opts=None, **kw):
        """nsteps CG relaxation steps of every candidate; returns energies
        (n, nsteps+1), final forces and positions (lists of (natoms, 3)), status."""
        o = opts if opts is not None else default_opts(**kw)
        n = len(self.natoms)
        e = np.zeros((n, nsteps + 1))
        f = np.zeros(sum(self.natoms) * 3)
        p = np.zeros(sum(self.natoms) * 3)
        st = np.zeros(n, dtype=np.int32)
        rc = self._lib.sgo_batch_relax_cg(self._h, int(nsteps), ctypes.byref(o), _dptr(e), _dptr(f),
                                          _dptr(p), _iptr(st))
        if rc not in (SGO_OK, SGO_ENOTCONV, SGO_ENUMERIC):
            self._check(rc)
        forces, pos, off = [], [], 0
        for na in self.natoms:
            forces.append(f[off:off + 3 * na].reshape(na, 3))
            pos.append(p[off:off + 3 * na].reshape(na, 3))
            off += 3 * na
        return e, forces, pos, st

    def de_generation(self, parents, e_parent, draws, de=None, opts=None, **kw):
        """One differential-evolution generation over the batch (mutation,
        crossover, checks, relax_steps batched CG steps, greedy selection).
        parents: list of (natoms, 3); draws: dict as for de_draws().  Returns
        a dict with trial, attempt_used, e_trial, survivors, e_survivor, take,
        status."""
        o = opts if opts is not None else default_opts(**kw)
        d = de if de is not None else de_opts()
        n = len(self.natoms)
        P = np.ascontiguousarray(np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1)
                                                 for p in parents]))
        ep = _f64(e_parent)
        dr = de_draws(draws)
        trial = np.zeros_like(P)
        surv = np.zeros_like(P)
        used = np.zeros(n, dtype=np.int32)
        et = np.zeros(n)
        es = np.zeros(n)
        take = np.zeros(n, dtype=np.int32)
        st = np.zeros(n, dtype=np.int32)
        rc = self._lib.sgo_batch_de_generation(self._h, ctypes.byref(d), ctypes.byref(o), _dptr(P),
                                               _dptr(ep), dr, _dptr(trial), _iptr(used),
                                               _dptr(et), _dptr(surv), _dptr(es), _iptr(take),
                                               _iptr(st))
        if rc not in (SGO_OK, SGO_ENOTCONV, SGO_ENUMERIC):
            self._check(rc)

        def split(a):
            out, off = [], 0
            for na in self.natoms:
                out.append(a[off:off + 3 * na].reshape(na, 3))
                off += 3 * na
            return out
        return {"trial": split(trial), "attempt_used": used, "e_trial": et,
                "survivors": split(surv), "e_survivor": es, "take": take, "status": st}

    def relax_pcg(self, nsteps, refit=1, opts=None, **kw):
        """nsteps force-fitted PCG relaxation steps of every candidate; returns
        energies (n, nsteps+1), final forces and positions (lists of
        (natoms, 3)), the last force-field fits (n, 3) and status."""
        o = opts if opts is not None else default_opts(**kw)
        n = len(self.natoms)
        e = np.zeros((n, nsteps + 1))
        f = np.zeros(sum(self.natoms) * 3)
        p = np.zeros(sum(self.natoms) * 3)
        prm = np.zeros((n, 3))
        st = np.zeros(n, dtype=np.int32)
        rc = self._lib.sgo_batch_relax_pcg(self._h, int(nsteps), int(refit), ctypes.byref(o),
                                           _dptr(e), _dptr(f), _dptr(p), _dptr(prm), _iptr(st))
        if rc not in (SGO_OK, SGO_ENOTCONV, SGO_ENUMERIC):
            self._check(rc)
        forces, pos, off = [], [], 0
        for na in self.natoms:
            forces.append(f[off:off + 3 * na].reshape(na, 3))
            pos.append(p[off:off + 3 * na].reshape(na, 3))
            off += 3 * na
        return e, forces, pos, prm, st

    def relax_cls(self, nsteps, opts=None, **kw):
        """nsteps curved-line-search relaxation steps of every candidate;
        returns energies (n, nsteps+1), final forces and positions, the last
        force-field fits (n, 3) and status."""
        o = opts if opts is not None else default_opts(**kw)
        n = len(self.natoms)
        e = np.zeros((n, nsteps + 1))
        f = np.zeros(sum(self.natoms) * 3)
        p = np.zeros(sum(self.natoms) * 3)
        prm = np.zeros((n, 3))
        st = np.zeros(n, dtype=np.int32)
        rc = self._lib.sgo_batch_relax_cls(self._h, int(nsteps), ctypes.byref(o), _dptr(e), _dptr(f),
                                           _dptr(p), _dptr(prm), _iptr(st))
        if rc not in (SGO_OK, SGO_ENOTCONV, SGO_ENUMERIC):
            self._check(rc)
        forces, pos, off = [], [], 0
        for na in self.natoms:
            forces.append(f[off:off + 3 * na].reshape(na, 3))
            pos.append(p[off:off + 3 * na].reshape(na, 3))
            off += 3 * na
        return e, forces, pos, prm, st

    def info(self, i):
        inf = sgo_scf_info()
        self._check(self._lib.sgo_batch_info(self._h, int(i), ctypes.byref(inf)))
        return {"iterations": inf.iterations, "converged": bool(inf.converged), "de": inf.de,
                "drho": inf.drho}

    def stress(self):
        """Fixed-basis stress [n, 3, 3] of every candidate after scf."""
        s = np.zeros((len(self.natoms), 3, 3))
        self._check(self._lib.sgo_batch_stress(self._h, _dptr(s)))
        return s


def context_from_system(system, precision=None, device=0):
    if precision is None:
        precision = SGO_FP64 if system.get("precision", "fp64") == "fp64" else SGO_FP32
    return Context(device, precision).load_system(system)
