"""Python binding of the symed C ABI (argument marshalling only).

Every computation runs in the HIP library ``libsymed.so``; this module only
converts arrays and tensors into pointers.  Device vectors are torch tensors
(float64, or complex128 for complex sectors) on the current HIP device; the
stream is torch's current stream unless one is given.

If the library has not been built the import of the library fails loudly:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsymed.so")

ED_OK, ED_EINVAL, ED_ENOTSTABLE, ED_ECHAR, ED_ENOMEM, ED_EDEVICE, ED_EBREAKDOWN = range(7)
STATUS_NAMES = {0: "ED_OK", 1: "ED_EINVAL", 2: "ED_ENOTSTABLE", 3: "ED_ECHAR", 4: "ED_ENOMEM", 5: "ED_EDEVICE",
                6: "ED_EBREAKDOWN"}

EXPORTED = ["ed_last_error", "ed_version", "ed_basis_build", "ed_basis_free", "ed_basis_info", "ed_basis_export",
            "ed_basis_device_reps", "ed_apply_H", "ed_lookup", "ed_lanczos_run", "ed_eigenvalues",
            "ed_tables_inspect", "ed_index_train", "ed_index_info", "ed_mlp_loss_grad",
            "ed_index_predict", "ed_batch_create", "ed_batch_apply", "ed_batch_lanczos", "ed_batch_info",
            "ed_batch_free", "ed_hash_build", "ed_ritz_vector", "ed_lanczos_vector", "ed_expectation", "ed_lanczos_resume",
            "ed_apply_op", "ed_apply_op_noalloc", "ed_tune_decomposition", "ed_basis_build_colors"]


class EdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Model(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("n_bonds", ctypes.c_int32), ("bond_sites", ctypes.c_void_p),
                ("bond_J", ctypes.c_void_p), ("n_tri", ctypes.c_int32), ("tri_sites", ctypes.c_void_p),
                ("tri_Jchi", ctypes.c_void_p)]


class _Group(ctypes.Structure):
    _fields_ = [("n_elem", ctypes.c_int32), ("perm", ctypes.c_void_p), ("flip", ctypes.c_void_p),
                ("chi_re", ctypes.c_void_p), ("chi_im", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("n_sub_rep", ctypes.c_int32), ("n_sub_act", ctypes.c_int32), ("prefix_bits", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("mem_limit_bytes", ctypes.c_int64)]


class BasisInfo(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int64), ("is_complex", ctypes.c_int32), ("n_sites", ctypes.c_int32),
                ("n_elem", ctypes.c_int32), ("n_sub_rep", ctypes.c_int32), ("n_sub_act", ctypes.c_int32),
                ("prefix_bits", ctypes.c_int32), ("n_elements", ctypes.c_int64), ("n_offdiag", ctypes.c_int64),
                ("bytes_device", ctypes.c_int64), ("table_bytes", ctypes.c_int64), ("limits_bytes", ctypes.c_int64),
                ("index_bytes", ctypes.c_int64), ("index_max_err", ctypes.c_int32), ("lds_resident", ctypes.c_int32),
                ("build_seconds", ctypes.c_double), ("limits_mean_window", ctypes.c_double),
                ("limits_max_window", ctypes.c_int64), ("apply_blocks", ctypes.c_int32),
                ("apply_threads", ctypes.c_int32), ("n_colors", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class IndexCfg(ctypes.Structure):
    _fields_ = [("n_features", ctypes.c_int32), ("hidden", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("lr", ctypes.c_float), ("seed", ctypes.c_uint32),
                ("log2_segments", ctypes.c_int32), ("keys_per_cell", ctypes.c_int32),
                ("max_window", ctypes.c_int32), ("routing", ctypes.c_int32)]


# routing of the learned index: what picks the segment
ROUTE_TRAINED, ROUTE_UNTRAINED, ROUTE_NONE = 0, 1, 2


class IndexStats(ctypes.Structure):
    _fields_ = [("max_err", ctypes.c_int32), ("n_segments", ctypes.c_int32), ("final_loss", ctypes.c_float),
                ("mlp_max_err", ctypes.c_float), ("mlp_bytes", ctypes.c_int64), ("table_bytes", ctypes.c_int64),
                ("train_seconds", ctypes.c_double), ("mean_window", ctypes.c_double),
                ("n_features", ctypes.c_int32), ("n_pieces", ctypes.c_int32), ("used_segments", ctypes.c_int64),
                ("feature_offset", ctypes.c_float), ("feature_scale", ctypes.c_float),
                ("n_cells", ctypes.c_int64), ("refined_segments", ctypes.c_int64), ("mean_abs_err", ctypes.c_double),
                ("frac_exact", ctypes.c_double), ("mean_lines", ctypes.c_double), ("lds_bytes", ctypes.c_int64),
                ("routing", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class HashCfg(ctypes.Structure):
    _fields_ = [("load", ctypes.c_double), ("reserved", ctypes.c_int32 * 2)]


class HashStats(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int64), ("bytes", ctypes.c_int64), ("load", ctypes.c_double),
                ("mean_probes", ctypes.c_double), ("max_probes", ctypes.c_int64), ("build_seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BatchCfg(ctypes.Structure):
    _fields_ = [("tile_rows", ctypes.c_int32), ("autotune", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("cache_path", ctypes.c_char_p)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_sectors", ctypes.c_int32), ("tile_rows", ctypes.c_int32), ("n_tiles", ctypes.c_int64),
                ("total_dim", ctypes.c_int64), ("total_elements", ctypes.c_int64), ("apply_blocks", ctypes.c_int32),
                ("n_candidates", ctypes.c_int32), ("tune_rows", ctypes.c_int32 * 8),
                ("tune_blocks", ctypes.c_int32 * 8), ("tune_seconds", ctypes.c_double * 8),
                ("tune_mode", ctypes.c_int32), ("cache_hit", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        n = self.n_candidates
        d["tune_rows"] = list(self.tune_rows)[:n]
        d["tune_blocks"] = list(self.tune_blocks)[:n]
        d["tune_seconds"] = list(self.tune_seconds)[:n]
        return d


class TuneReport(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int32), ("cache_hit", ctypes.c_int32), ("sub_rep", ctypes.c_int32 * 16),
                ("sub_act", ctypes.c_int32 * 16), ("seconds", ctypes.c_double * 16)]

    def as_dict(self):
        n = self.n_candidates
        return {"n_candidates": n, "cache_hit": self.cache_hit,
                "candidates": [(self.sub_rep[k], self.sub_act[k], self.seconds[k]) for k in range(n)]}


_LIB = None


def lib():
    """Load libsymed.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"symed HIP library not built: {LIB_PATH} missing (run __graft_entry__.build())")
        # torch first: its HIP runtime (same soname, libamdhip64.so.7) is then
        # the one the library binds to, so the library and the tensors handed
        # to it share one runtime whichever of the two a program touches first.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.ed_last_error.restype = ctypes.c_char_p
        L.ed_version.restype = ctypes.c_char_p
        L.ed_basis_build.argtypes = [ctypes.POINTER(_Model), ctypes.POINTER(_Group), i32, ctypes.POINTER(_Options),
                                     vp, ctypes.POINTER(vp)]
        L.ed_basis_build_colors.argtypes = [ctypes.POINTER(_Model), ctypes.POINTER(_Group), i32, vp,
                                            ctypes.POINTER(_Options), vp, ctypes.POINTER(vp)]
        L.ed_basis_free.argtypes = [vp]
        L.ed_basis_free.restype = None
        L.ed_basis_info.argtypes = [vp, ctypes.POINTER(BasisInfo)]
        L.ed_basis_export.argtypes = [vp, vp, vp]
        L.ed_basis_device_reps.argtypes = [vp, ctypes.POINTER(vp)]
        L.ed_apply_H.argtypes = [vp, vp, vp, i32, vp]
        L.ed_lookup.argtypes = [vp, vp, i64, vp, i32, vp]
        L.ed_lanczos_run.argtypes = [vp, vp, i32, i32, vp, vp, ctypes.POINTER(i32), vp]
        L.ed_eigenvalues.argtypes = [vp, vp, i32, i32, vp]
        L.ed_tables_inspect.argtypes = [ctypes.POINTER(_Model), ctypes.POINTER(_Group), i32, i32, vp, vp, vp, i64,
                                        ctypes.POINTER(i64), vp]
        L.ed_index_train.argtypes = [vp, ctypes.POINTER(IndexCfg), ctypes.POINTER(IndexStats), vp]
        L.ed_index_info.argtypes = [vp, ctypes.POINTER(IndexStats), vp, i64]
        L.ed_mlp_loss_grad.argtypes = [i32, vp, vp, vp, i64, vp, vp, vp]
        L.ed_index_predict.argtypes = [vp, vp, i64, vp, vp, vp]
        L.ed_lanczos_resume.argtypes = [vp, i32, i32, vp, vp, ctypes.POINTER(i32), vp]
        L.ed_ritz_vector.argtypes = [vp, vp, i32, i32, vp, vp]
        L.ed_lanczos_vector.argtypes = [vp, vp, i32, i32, vp, vp, vp]
        L.ed_expectation.argtypes = [vp, ctypes.POINTER(_Model), vp, i32, vp, vp, vp]
        L.ed_apply_op.argtypes = [vp, ctypes.POINTER(_Model), vp, vp, vp, i32, vp, vp, vp]
        L.ed_apply_op_noalloc.argtypes = [vp, ctypes.POINTER(_Model), vp, vp, vp, i32, vp, vp, vp]
        L.ed_hash_build.argtypes = [vp, ctypes.POINTER(HashCfg), ctypes.POINTER(HashStats), vp]
        L.ed_batch_create.argtypes = [vp, i32, ctypes.POINTER(BatchCfg), vp, ctypes.POINTER(vp)]
        L.ed_batch_apply.argtypes = [vp, vp, vp, i32, vp]
        L.ed_batch_lanczos.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp]
        L.ed_batch_info.argtypes = [vp, ctypes.POINTER(BatchInfo)]
        L.ed_batch_free.argtypes = [vp]
        L.ed_batch_free.restype = None
        L.ed_tune_decomposition.argtypes = [ctypes.POINTER(_Model), ctypes.POINTER(_Group), i32, i32,
                                            ctypes.c_char_p, vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                            ctypes.POINTER(TuneReport)]
        for name in EXPORTED:
            if hasattr(L, name) and name not in ("ed_last_error", "ed_version", "ed_basis_free", "ed_batch_free"):
                getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB


def _check(status):
    if status != ED_OK:
        raise EdError(status, lib().ed_last_error().decode())


def version():
    return lib().ed_version().decode()


def _np_ptr(a):
    return a.ctypes.data if a is not None and a.size else None


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _tensor_ptr(t):
    return t.data_ptr()


class _Arrays:
    """Host copies of a problem description, kept alive across a call."""

    def __init__(self, n_sites, bonds, bond_J, tris, tri_Jchi, perms, flips, chi):
        self.bonds = np.ascontiguousarray(np.asarray(bonds, np.int32).reshape(-1))
        self.bond_J = np.ascontiguousarray(np.asarray(bond_J, np.float64))
        self.tris = np.ascontiguousarray(np.asarray(tris, np.int32).reshape(-1))
        self.tri_J = np.ascontiguousarray(np.asarray(tri_Jchi, np.float64))
        self.perms = np.ascontiguousarray(np.asarray(perms, np.int32).reshape(-1))
        self.flips = np.ascontiguousarray(np.asarray(flips, np.uint8))
        chi = np.asarray(chi)
        self.chi_re = np.ascontiguousarray(chi.real.astype(np.float64))
        self.chi_im = np.ascontiguousarray(np.imag(chi).astype(np.float64))
        self.model = _Model(n_sites, len(self.bond_J), _np_ptr(self.bonds), _np_ptr(self.bond_J), len(self.tri_J),
                            _np_ptr(self.tris), _np_ptr(self.tri_J))
        self.group = _Group(len(self.flips), _np_ptr(self.perms), _np_ptr(self.flips), _np_ptr(self.chi_re),
                            _np_ptr(self.chi_im))


def _arrays_from(inst):
    return _Arrays(inst.n_sites, inst.bonds, inst.bond_J, inst.tris, inst.tri_Jchi, inst.perms, inst.flips, inst.chi)


class Basis:
    """A built sector basis (library-owned device memory)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)
        self._info = None

    @classmethod
    def build(cls, inst, n_sub_rep=0, n_sub_act=0, prefix_bits=0, mem_limit_bytes=0, stream=None):
        """Build the basis of a problem description with attributes n_sites,
        bonds, bond_J, tris, tri_Jchi, perms, flips, chi, n_up; with
        local_dim > 0 (and counts) an SU(local_dim) permutation model in the
        sector of those color counts (ed_basis_build_colors)."""
        arr = _arrays_from(inst)
        opts = _Options(n_sub_rep, n_sub_act, prefix_bits, 0, mem_limit_bytes)
        h = ctypes.c_void_p()
        d = int(getattr(inst, "local_dim", 0) or 0)
        if d:
            counts = np.ascontiguousarray(np.asarray(inst.counts, np.int32))
            _check(lib().ed_basis_build_colors(ctypes.byref(arr.model), ctypes.byref(arr.group), d, _np_ptr(counts),
                                               ctypes.byref(opts), _stream_ptr(stream), ctypes.byref(h)))
        else:
            _check(lib().ed_basis_build(ctypes.byref(arr.model), ctypes.byref(arr.group), int(inst.n_up),
                                        ctypes.byref(opts), _stream_ptr(stream), ctypes.byref(h)))
        return cls(h.value)

    def free(self):
        if self._h:
            lib().ed_basis_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self):
        inf = BasisInfo()
        _check(lib().ed_basis_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    @property
    def dim(self):
        return self.info()["dim"]

    @property
    def is_complex(self):
        return bool(self.info()["is_complex"])

    def export(self):
        d = self.dim
        reps = np.zeros(d, np.uint64)
        stab = np.zeros(d, np.uint32)
        _check(lib().ed_basis_export(self._h, _np_ptr(reps), _np_ptr(stab)))
        return reps, stab

    def device_reps_ptr(self):
        p = ctypes.c_void_p()
        _check(lib().ed_basis_device_reps(self._h, ctypes.byref(p)))
        return p.value

    def apply_H(self, x, y, mode=0, stream=None):
        """y := H x on device tensors (float64 or complex128)."""
        _check(lib().ed_apply_H(self._h, _tensor_ptr(x), _tensor_ptr(y), int(mode), _stream_ptr(stream)))
        return y

    def lookup(self, keys, idx, mode=0, stream=None):
        """idx[k] = position of keys[k] (uint64 stored in an int64 tensor) or -1."""
        _check(lib().ed_lookup(self._h, _tensor_ptr(keys), keys.numel(), _tensor_ptr(idx), int(mode),
                               _stream_ptr(stream)))
        return idx

    def lanczos(self, v0, n_iter, mode=0, stream=None):
        """Run n_iter Lanczos steps from device vector v0; returns (alpha, beta,
        n_done, broken)."""
        a = np.zeros(n_iter)
        b = np.zeros(n_iter)
        nd = ctypes.c_int32(0)
        st = lib().ed_lanczos_run(self._h, _tensor_ptr(v0), int(n_iter), int(mode), _np_ptr(a), _np_ptr(b),
                                  ctypes.byref(nd), _stream_ptr(stream))
        if st not in (ED_OK, ED_EBREAKDOWN):
            _check(st)
        n = nd.value
        return a[:n], b[:n], n, st == ED_EBREAKDOWN

    def lanczos_resume(self, n_more, mode=0, stream=None):
        """n_more further steps of the last lanczos() run; returns (alpha, beta,
        n_done, broken) for the new steps."""
        a = np.zeros(n_more)
        b = np.zeros(n_more)
        nd = ctypes.c_int32(0)
        st = lib().ed_lanczos_resume(self._h, int(n_more), int(mode), _np_ptr(a), _np_ptr(b), ctypes.byref(nd),
                                     _stream_ptr(stream))
        if st not in (ED_OK, ED_EBREAKDOWN):
            _check(st)
        n = nd.value
        return a[:n], b[:n], n, st == ED_EBREAKDOWN

    def train_index(self, n_features=0, hidden=32, steps=0, batch=0, lr=0.0, seed=1, log2_segments=0,
                    keys_per_cell=0, max_window=0, routing=ROUTE_TRAINED, stream=None):
        cfg = IndexCfg(n_features, hidden, steps, batch, lr, seed, log2_segments, keys_per_cell, max_window,
                       routing)
        stats = IndexStats()
        _check(lib().ed_index_train(self._h, ctypes.byref(cfg), ctypes.byref(stats), _stream_ptr(stream)))
        return stats.as_dict()

    def ground_state(self, v0, n_iter, mode=0, k=0, stream=None):
        """Lanczos (n_iter steps from v0), then the k-th Ritz vector rebuilt
        by a second pass; returns (eigenvalue, normalized device vector)."""
        import torch
        a, b, n, broken = self.lanczos(v0, n_iter, mode=mode, stream=stream)
        lam, coef = ritz_vector(a, b, k)
        psi = torch.empty_like(v0)
        _check(lib().ed_lanczos_vector(self._h, _tensor_ptr(v0), n, int(mode), _np_ptr(coef), _tensor_ptr(psi),
                                       _stream_ptr(stream)))
        return lam, psi

    def _op_model(self, bonds, bond_J, tris, tri_Jchi):
        bonds = np.ascontiguousarray(np.zeros((0, 2)) if bonds is None else bonds, np.int32).reshape(-1)
        bond_J = np.ascontiguousarray(np.zeros(0) if bond_J is None else bond_J, np.float64)
        tris = np.ascontiguousarray(np.zeros((0, 3)) if tris is None else tris, np.int32).reshape(-1)
        tri_Jchi = np.ascontiguousarray(np.zeros(0) if tri_Jchi is None else tri_Jchi, np.float64)
        n_sites = self.info()["n_sites"]
        keep = (bonds, bond_J, tris, tri_Jchi)
        return _Model(n_sites, len(bond_J), _np_ptr(bonds), _np_ptr(bond_J), len(tri_Jchi), _np_ptr(tris),
                      _np_ptr(tri_Jchi)), keep

    def expectation(self, psi, bonds=None, bond_J=None, tris=None, tri_Jchi=None, mode=0, stream=None):
        """<psi|O|psi> for O = sum J S_i.S_j (+ sum Jchi S_i.(S_j x S_k)); O must
        be invariant under the basis's group.  Returns a complex number."""
        m, keep = self._op_model(bonds, bond_J, tris, tri_Jchi)
        re = ctypes.c_double(0.0)
        im = ctypes.c_double(0.0)
        _check(lib().ed_expectation(self._h, ctypes.byref(m), _tensor_ptr(psi), int(mode), ctypes.byref(re),
                                    ctypes.byref(im), _stream_ptr(stream)))
        del keep
        return complex(re.value, im.value)

    def apply_op(self, x, y, bonds=None, bond_J=None, tris=None, tri_Jchi=None, z=None, mode=0, stream=None):
        """y := O x for O as in ``expectation`` (device vectors of dim
        entries); with a device vector z also returns <z, y> (complex)."""
        m, keep = self._op_model(bonds, bond_J, tris, tri_Jchi)
        re = ctypes.c_double(0.0)
        im = ctypes.c_double(0.0)
        _check(lib().ed_apply_op(self._h, ctypes.byref(m), _tensor_ptr(x), _tensor_ptr(y),
                                 None if z is None else _tensor_ptr(z), int(mode), ctypes.byref(re), ctypes.byref(im),
                                 _stream_ptr(stream)))
        del keep
        return None if z is None else complex(re.value, im.value)

    def apply_op_noalloc(self, x, y, bonds=None, bond_J=None, tris=None, tri_Jchi=None, z=None, mode=0,
                         stream=None):
        """``apply_op`` through ed_apply_op_noalloc: the operator's tables and
        the dot partials go to the library's static device scratch array."""
        m, keep = self._op_model(bonds, bond_J, tris, tri_Jchi)
        re = ctypes.c_double(0.0)
        im = ctypes.c_double(0.0)
        _check(lib().ed_apply_op_noalloc(self._h, ctypes.byref(m), _tensor_ptr(x), _tensor_ptr(y),
                                         None if z is None else _tensor_ptr(z), int(mode), ctypes.byref(re),
                                         ctypes.byref(im), _stream_ptr(stream)))
        del keep
        return None if z is None else complex(re.value, im.value)

    def build_hash(self, load=0.0, stream=None):
        """Build the hashed staging table (lookup mode 2); returns its stats."""
        cfg = HashCfg(float(load), (ctypes.c_int32 * 2)(0, 0))
        st = HashStats()
        _check(lib().ed_hash_build(self._h, ctypes.byref(cfg), ctypes.byref(st), _stream_ptr(stream)))
        return st.as_dict()

    def index_predict(self, keys, stream=None):
        """(u, y) of the trained network on device keys (int64 tensor holding uint64)."""
        import torch
        u = torch.empty(keys.numel(), dtype=torch.float32, device=keys.device)
        y = torch.empty_like(u)
        _check(lib().ed_index_predict(self._h, _tensor_ptr(keys), keys.numel(), _tensor_ptr(u), _tensor_ptr(y),
                                      _stream_ptr(stream)))
        return u, y

    def index_weights(self):
        """(stats, float32 weights) of the trained learned index."""
        stats = IndexStats()
        buf = np.zeros(1 << 12, np.float32)
        _check(lib().ed_index_info(self._h, ctypes.byref(stats), _np_ptr(buf), buf.size))
        F = stats.n_features
        n = 32 * F + 32 + 32 * 32 + 32 + 32 + 1
        return stats.as_dict(), buf[:n].copy()


class Batch:
    """Several built sectors run together: one persistent launch per H.v and
    one captured HIP graph per Lanczos step.  The sectors must outlive it."""

    def __init__(self, sectors, tile_rows=0, autotune=True, blocks_per_cu=0, cache_path=None, stream=None):
        self.sectors = list(sectors)
        n = len(self.sectors)
        hs = (ctypes.c_void_p * n)(*[s._h.value for s in self.sectors])
        self._cache = None if cache_path is None else str(cache_path).encode()
        cfg = BatchCfg(int(tile_rows), 1 if autotune else 0, int(blocks_per_cu), 0, self._cache)
        h = ctypes.c_void_p()
        _check(lib().ed_batch_create(hs, n, ctypes.byref(cfg), _stream_ptr(stream), ctypes.byref(h)))
        self._h = h

    def free(self):
        if self._h:
            lib().ed_batch_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def info(self):
        inf = BatchInfo()
        _check(lib().ed_batch_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def apply_H(self, xs, ys, mode=0, stream=None):
        """ys[s] := H_s xs[s] for every sector, one launch."""
        n = len(self.sectors)
        px = (ctypes.c_void_p * n)(*[_tensor_ptr(x) for x in xs])
        py = (ctypes.c_void_p * n)(*[_tensor_ptr(y) for y in ys])
        _check(lib().ed_batch_apply(self._h, px, py, int(mode), _stream_ptr(stream)))
        return ys

    def lanczos(self, v0s, n_iter, mode=0, stream=None):
        """n_iter Lanczos steps of every sector; returns a list of
        (alpha, beta, n_done, broken) per sector."""
        n = len(self.sectors)
        pv = (ctypes.c_void_p * n)(*[_tensor_ptr(v) for v in v0s])
        a = np.zeros((n, n_iter))
        b = np.zeros((n, n_iter))
        nd = np.zeros(n, np.int32)
        st = lib().ed_batch_lanczos(self._h, pv, int(n_iter), int(mode), _np_ptr(a), _np_ptr(b), _np_ptr(nd),
                                    _stream_ptr(stream))
        if st not in (ED_OK, ED_EBREAKDOWN):
            _check(st)
        return [(a[s, :nd[s]].copy(), b[s, :nd[s]].copy(), int(nd[s]), int(nd[s]) < n_iter) for s in range(n)]


def mlp_loss_grad(n_features, params, X, t, stream=None):
    """Loss and gradient of the index network on device tensors (float32)."""
    import torch
    n = t.numel()
    grad = torch.zeros(params.numel(), dtype=torch.float32, device=params.device)
    loss = torch.zeros(1, dtype=torch.float32, device=params.device)
    _check(lib().ed_mlp_loss_grad(int(n_features), _tensor_ptr(params), _tensor_ptr(X), _tensor_ptr(t), n,
                                  _tensor_ptr(grad), _tensor_ptr(loss), _stream_ptr(stream)))
    return float(loss.item()), grad


def ritz_vector(alpha, beta, k=0):
    """(k-th lowest eigenvalue, its normalized eigenvector) of the T-matrix."""
    a = np.ascontiguousarray(alpha, np.float64)
    b = np.ascontiguousarray(beta, np.float64)
    coef = np.zeros(len(a))
    lam = ctypes.c_double(0.0)
    _check(lib().ed_ritz_vector(_np_ptr(a), _np_ptr(b) if len(b) else None, len(a), int(k), ctypes.byref(lam),
                                _np_ptr(coef)))
    return lam.value, coef


def tune_decomposition(inst, mode=0, cache_path=None, stream=None):
    """Fastest admissible pair (n_sub_rep, n_sub_act) for a sector by timing
    one H.v per pair in lookup mode `mode` (ed_tune_decomposition); returns
    (n_sub_rep, n_sub_act, report)."""
    arr = _arrays_from(inst)
    r = ctypes.c_int32(0)
    a = ctypes.c_int32(0)
    rep = TuneReport()
    path = None if cache_path is None else str(cache_path).encode()
    _check(lib().ed_tune_decomposition(ctypes.byref(arr.model), ctypes.byref(arr.group), int(inst.n_up), int(mode),
                                       path, _stream_ptr(stream), ctypes.byref(r), ctypes.byref(a),
                                       ctypes.byref(rep)))
    return r.value, a.value, rep.as_dict()


def eigenvalues(alpha, beta, k=1):
    a = np.ascontiguousarray(alpha, np.float64)
    b = np.ascontiguousarray(beta, np.float64)
    out = np.zeros(k)
    _check(lib().ed_eigenvalues(_np_ptr(a), _np_ptr(b) if len(b) else None, len(a), int(k), _np_ptr(out)))
    return out


def tables_inspect(inst, n_sub):
    """Host-only Rep/Sym/SymmetryAction tables of one decomposition."""
    arr = _arrays_from(inst)
    b = inst.n_sites // n_sub
    S = 1 << b
    rep = np.zeros(n_sub * S, np.uint32)
    off = np.zeros(n_sub * S + 1, np.uint32)
    nsym = ctypes.c_int64(0)
    _check(lib().ed_tables_inspect(ctypes.byref(arr.model), ctypes.byref(arr.group), int(inst.n_up), n_sub,
                                   _np_ptr(rep), _np_ptr(off), None, 0, ctypes.byref(nsym), None))
    sym = np.zeros(max(nsym.value, 1), np.uint32)
    act = np.zeros(len(inst.flips) * n_sub * S, np.uint64)
    _check(lib().ed_tables_inspect(ctypes.byref(arr.model), ctypes.byref(arr.group), int(inst.n_up), n_sub,
                                   _np_ptr(rep), _np_ptr(off), _np_ptr(sym), sym.size, ctypes.byref(nsym),
                                   _np_ptr(act)))
    return rep.reshape(n_sub, S), off, sym[: nsym.value], act.reshape(len(inst.flips), n_sub, S)
