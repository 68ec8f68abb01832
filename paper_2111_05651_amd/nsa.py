"""Thin ctypes binding to libnsa (include/nsa.h): argument marshalling only.

Every step of the assembly runs in the library's HIP kernels; PyTorch supplies device memory and
the stream. There is no CPU fallback: if ``libnsa.so`` is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libnsa.so")

NSA_OK, NSA_EINVAL, NSA_ERANGE, NSA_EDEGENERATE, NSA_ENOMEM, NSA_EHIP, NSA_EUNSUPPORTED, NSA_ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7
FP64, MIXED = 0, 1
ATOMIC, COLOUR = 0, 1
KERNEL_AUTO, KERNEL_TILED, KERNEL_DIRECT, KERNEL_GATHER = 0, 1, 2, 3
VEL_AOS, VEL_SOA = 0, 1  # velocity [npoin][ndime] or [ndime][npoin]
GATHER_PLAN = 2
PROBE_READ, PROBE_WRITE, PROBE_COPY = 0, 1, 2
RESIDUAL_PLAN = 3

# every symbol include/nsa.h declares
EXPORTS = ["nsa_status_string", "nsa_last_error", "nsa_version", "nsa_pattern_count", "nsa_pattern_fill",
           "nsa_mesh_create", "nsa_mesh_set_tiling", "nsa_mesh_set_tile_threads", "nsa_mesh_keep_direct", "nsa_mesh_destroy", "nsa_mesh_get_info", "nsa_mesh_get_pattern",
           "nsa_mesh_get_colouring", "nsa_pattern_scalar_csr", "nsa_mesh_get_tiles", "nsa_mesh_get_gather", "nsa_mesh_upload", "nsa_mesh_release_host", "nsa_assemble",
           "nsa_batch_create", "nsa_batch_reserve", "nsa_batch_reset", "nsa_batch_destroy", "nsa_batch_get_info", "nsa_batch_upload", "nsa_batch_set_inputs",
           "nsa_assemble_batched", "nsa_assemble_batched_static", "nsa_fill_uniform", "nsa_bandwidth_probe", "nsa_mesh_get_residual_tiles", "nsa_assemble_residual",
           "nsa_mesh_set_residual_geometry", "nsa_mesh_create_q1", "nsa_mesh_get_q1_tiles"]


class NsaError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class Options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("scatter", C.c_int32), ("accumulate", C.c_int32),
                ("block_threads", C.c_int32), ("kernel", C.c_int32), ("vel_layout", C.c_int32),
                ("err_out", C.c_void_p)]


ERR_CLASSES = ("uu", "up", "pu", "pp", "rhs_u", "rhs_p")  # the classes of nsa_options.err_out
TET4, QUAD4 = 0, 1  # element families (nsa_mesh_info.family)


class MeshInfo(C.Structure):
    _fields_ = [("npoin", C.c_int64), ("nelem", C.c_int64), ("nnzb", C.c_int64), ("ncolours", C.c_int32),
                ("uploaded", C.c_int32), ("ws_bytes", C.c_size_t), ("max_row_blocks", C.c_int64),
                ("ntiles", C.c_int64 * 2), ("tile_runs", C.c_int64 * 2), ("tile_blocks", C.c_int32 * 2),
                ("tile_threads", C.c_int32 * 2), ("tile_max_runs", C.c_int32 * 2),
                ("tile_lds_bytes", C.c_int32 * 2), ("gather_ntiles", C.c_int64), ("gather_records", C.c_int64),
                ("gather_pairs", C.c_int64), ("gather_tile_blocks", C.c_int32), ("gather_threads", C.c_int32),
                ("gather_lds_bytes", C.c_int32 * 2), ("residual_ntiles", C.c_int64),
                ("residual_records", C.c_int64), ("residual_tile_rows", C.c_int32),
                ("residual_lds_bytes", C.c_int32), ("family", C.c_int32), ("pad0", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libnsa.so from the package directory (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2111_05651_amd.build.build_library()")
    lib = C.CDLL(path)
    P, i32, i64, d, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_size_t
    lib.nsa_status_string.argtypes = [i32]
    lib.nsa_status_string.restype = C.c_char_p
    lib.nsa_last_error.argtypes = []
    lib.nsa_last_error.restype = C.c_char_p
    lib.nsa_version.restype = i32
    lib.nsa_pattern_count.argtypes = [i64, i64, P, P, P]
    lib.nsa_pattern_fill.argtypes = [i64, i64, P, P, P, P]
    lib.nsa_mesh_create.argtypes = [i64, i64, P, P, C.POINTER(P)]
    lib.nsa_mesh_set_tiling.argtypes = [P, i32, i32]
    lib.nsa_mesh_set_tile_threads.argtypes = [P, i32]
    lib.nsa_mesh_keep_direct.argtypes = [P, i32]
    lib.nsa_mesh_destroy.argtypes = [P]
    lib.nsa_mesh_get_info.argtypes = [P, C.POINTER(MeshInfo)]
    lib.nsa_mesh_get_pattern.argtypes = [P, P, P, P]
    lib.nsa_mesh_get_colouring.argtypes = [P, P, P]
    lib.nsa_pattern_scalar_csr.argtypes = [P, P, P]
    lib.nsa_mesh_get_tiles.argtypes = [P, i32, P, P, P, P, P, P]
    lib.nsa_mesh_get_gather.argtypes = [P, P, P, P, P, P, P, P, P, P]
    lib.nsa_mesh_upload.argtypes = [P, P, sz, P]
    lib.nsa_mesh_release_host.argtypes = [P]
    lib.nsa_assemble.argtypes = [P, P, d, d, d, C.POINTER(Options), P, P, P]
    lib.nsa_batch_create.argtypes = [i32, P, i32, C.POINTER(P)]
    lib.nsa_batch_reserve.argtypes = [i32, i64, i32, C.POINTER(P)]
    lib.nsa_batch_reset.argtypes = [P, i32, P]
    lib.nsa_batch_destroy.argtypes = [P]
    lib.nsa_batch_get_info.argtypes = [P, P, P, P, P]
    lib.nsa_batch_upload.argtypes = [P, P, sz, P]
    lib.nsa_batch_set_inputs.argtypes = [P, P, P, P, P, P, P, i32, P]
    lib.nsa_assemble_batched.argtypes = [P, C.POINTER(Options), i32, P]
    lib.nsa_assemble_batched_static.argtypes = [i32, P, P, P, P, P, P, P, C.POINTER(Options), P]
    lib.nsa_fill_uniform.argtypes = [P, i64, C.c_uint64, d, d, P]
    lib.nsa_bandwidth_probe.argtypes = [i32, P, P, i64, P]
    lib.nsa_mesh_get_residual_tiles.argtypes = [P, P, P, P, P, P, P]
    lib.nsa_assemble_residual.argtypes = [P, P, d, d, d, C.POINTER(Options), P, P, P, P]
    lib.nsa_mesh_set_residual_geometry.argtypes = [P, i32]
    lib.nsa_mesh_create_q1.argtypes = [i64, i64, P, P, C.POINTER(P)]
    lib.nsa_mesh_get_q1_tiles.argtypes = [P, i32, P, P, P, P, P, P]
    for name in EXPORTS:
        if name not in ("nsa_status_string", "nsa_last_error", "nsa_version"):
            getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(st: int, where: str):
    if st != NSA_OK:
        lib = load()
        raise NsaError(st, where, lib.nsa_last_error().decode() or lib.nsa_status_string(st).decode())


def _ptr(a) -> int:
    """Address of a NumPy array or a torch tensor (CPU or device)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _dev_tensor(t, shape, name: str, device=None):
    """The C entry points take bare pointers, so the binding checks what only it can see: a contiguous
    float64 device tensor of exactly the expected shape (on the mesh's device when one is given)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 device tensor (got {t.dtype}, {t.device}, "
                         f"contiguous={t.is_contiguous()})")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the mesh on {device}")
    return t.data_ptr()


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def pattern(npoin: int, lnods: np.ndarray):
    """Block-CSR pattern (bptr int64, bcol int32, emap int32 [nelem][4][4]) via the library."""
    lib = load()
    ln = np.ascontiguousarray(lnods, dtype=np.int32)
    nelem = ln.shape[0]
    bptr = np.zeros(npoin + 1, dtype=np.int64)
    nnzb = np.zeros(1, dtype=np.int64)
    _check(lib.nsa_pattern_count(npoin, nelem, _ptr(ln), _ptr(bptr), _ptr(nnzb)), "nsa_pattern_count")
    bcol = np.zeros(int(nnzb[0]), dtype=np.int32)
    emap = np.zeros((nelem, 4, 4), dtype=np.int32)
    _check(lib.nsa_pattern_fill(npoin, nelem, _ptr(ln), _ptr(bptr), _ptr(bcol), _ptr(emap)), "nsa_pattern_fill")
    return bptr, bcol, emap


class Mesh:
    """A registered mesh (host handle) and, after upload(), its device workspace (a torch tensor)."""

    def __init__(self, lnods: np.ndarray, coord: np.ndarray, tile_blocks: int | None = None,
                 tile_blocks_colour: int | None = None, keep_direct: bool = True,
                 tile_blocks_gather: int | None = None, tile_rows_residual: int | None = None,
                 tile_threads: int | None = None, residual_geometry: bool = False, family: int = TET4):
        lib = load()
        ln = np.ascontiguousarray(lnods, dtype=np.int32)
        co = np.ascontiguousarray(coord, dtype=np.float64)
        dim = 3 if family == TET4 else 2
        if ln.ndim != 2 or ln.shape[1] != 4 or co.ndim != 2 or co.shape[1] != dim:
            raise ValueError(f"lnods must be [nelem][4] and coord [npoin][{dim}]")
        h = C.c_void_p()
        create = lib.nsa_mesh_create if family == TET4 else lib.nsa_mesh_create_q1
        _check(create(co.shape[0], ln.shape[0], _ptr(ln), _ptr(co), C.byref(h)), "nsa_mesh_create")
        self._h = h
        self.ws = None
        if tile_blocks is not None:
            _check(lib.nsa_mesh_set_tiling(h, ATOMIC, int(tile_blocks)), "nsa_mesh_set_tiling")
        if tile_blocks_colour is not None:
            _check(lib.nsa_mesh_set_tiling(h, COLOUR, int(tile_blocks_colour)), "nsa_mesh_set_tiling")
        if tile_threads is not None:
            _check(lib.nsa_mesh_set_tile_threads(h, int(tile_threads)), "nsa_mesh_set_tile_threads")
        if tile_blocks_gather is not None:
            _check(lib.nsa_mesh_set_tiling(h, GATHER_PLAN, int(tile_blocks_gather)), "nsa_mesh_set_tiling")
        if tile_rows_residual is not None:
            _check(lib.nsa_mesh_set_tiling(h, RESIDUAL_PLAN, int(tile_rows_residual)), "nsa_mesh_set_tiling")
        if not keep_direct:
            _check(lib.nsa_mesh_keep_direct(h, 0), "nsa_mesh_keep_direct")
        if residual_geometry:
            _check(lib.nsa_mesh_set_residual_geometry(h, 1), "nsa_mesh_set_residual_geometry")
        self.info = self._info()

    @classmethod
    def from_inputs(cls, m, tile_blocks: int | None = None, tile_blocks_colour: int | None = None,
                    tile_blocks_gather: int | None = None, keep_direct: bool = True,
                    tile_rows_residual: int | None = None, tile_threads: int | None = None,
                    residual_geometry: bool = False) -> "Mesh":
        return cls(m.lnods, m.coord, tile_blocks, tile_blocks_colour, keep_direct, tile_blocks_gather,
                   tile_rows_residual, tile_threads, residual_geometry)

    @classmethod
    def from_quads(cls, m, tile_blocks: int | None = None, tile_blocks_colour: int | None = None) -> "Mesh":
        """A quadrilateral mesh (the 2-D family; inputs.QuadMesh or any object with lnods and coord [npoin][2])."""
        return cls(m.lnods, m.coord, tile_blocks, tile_blocks_colour, family=QUAD4)

    @property
    def family(self) -> int:
        return self.info.family

    @property
    def ndofn(self) -> int:
        """Dofs per node: 4 (u, v, w, p) for tetrahedra, 3 (u, v, p) for quadrilaterals."""
        return 4 if self.info.family == TET4 else 3

    @property
    def ndime(self) -> int:
        return 3 if self.info.family == TET4 else 2

    def set_tiling(self, tile_blocks: int, scatter: int = ATOMIC):
        _check(load().nsa_mesh_set_tiling(self._h, int(scatter), int(tile_blocks)), "nsa_mesh_set_tiling")
        self.info = self._info()

    def keep_direct(self, keep: bool):
        _check(load().nsa_mesh_keep_direct(self._h, int(bool(keep))), "nsa_mesh_keep_direct")
        self.info = self._info()

    def _info(self) -> MeshInfo:
        info = MeshInfo()
        _check(load().nsa_mesh_get_info(self._h, C.byref(info)), "nsa_mesh_get_info")
        return info

    @property
    def npoin(self):
        return self.info.npoin

    @property
    def nelem(self):
        return self.info.nelem

    @property
    def nnzb(self):
        return self.info.nnzb

    def pattern(self):
        i = self.info
        bptr = np.zeros(i.npoin + 1, dtype=np.int64)
        bcol = np.zeros(i.nnzb, dtype=np.int32)
        emap = np.zeros((i.nelem, 4, 4), dtype=np.int32)
        _check(load().nsa_mesh_get_pattern(self._h, _ptr(bptr), _ptr(bcol), _ptr(emap)), "nsa_mesh_get_pattern")
        return bptr, bcol, emap

    def scalar_csr(self):
        """Scalar CSR view of the block pattern: (row_ptr int64 [4 npoin + 1], col int32 [16 nnzb])."""
        i = self.info
        row_ptr = np.zeros(4 * i.npoin + 1, dtype=np.int64)
        col = np.zeros(16 * i.nnzb, dtype=np.int32)
        _check(load().nsa_pattern_scalar_csr(self._h, _ptr(row_ptr), _ptr(col)), "nsa_pattern_scalar_csr")
        return row_ptr, col

    def colouring(self):
        i = self.info
        cptr = np.zeros(i.ncolours + 1, dtype=np.int32)
        celems = np.zeros(i.nelem, dtype=np.int32)
        _check(load().nsa_mesh_get_colouring(self._h, _ptr(cptr), _ptr(celems)), "nsa_mesh_get_colouring")
        return cptr, celems

    RUN_DTYPE = np.dtype([("row", np.uint16), ("hinge", np.uint16), ("k0", np.uint16), ("len", np.uint16),
                          ("diag", np.uint16), ("jslot", np.uint16), ("last", np.uint16), ("pad", np.uint16),
                          ("knew", np.uint16, (4,)), ("kslot", np.uint16, (4,))])

    def tiles(self, scatter: int = ATOMIC):
        """Row-tile plan of one scatter mode: dict of tile_row, tile_rptr, run_elems (int32 [runs][4]),
        tile_nptr, tile_nodes and runs (structured, RUN_DTYPE)."""
        i = self.info
        nt, nr = i.ntiles[scatter], i.tile_runs[scatter]
        out = dict(tile_row=np.zeros(nt + 1, np.int32), tile_rptr=np.zeros(nt + 1, np.int64),
                   run_elems=np.zeros((nr, 4), np.int32), tile_nptr=np.zeros(nt + 1, np.int64),
                   runs=np.zeros(nr, self.RUN_DTYPE))
        lib = load()
        _check(lib.nsa_mesh_get_tiles(self._h, int(scatter), None, None, None, _ptr(out["tile_nptr"]), None, None),
               "nsa_mesh_get_tiles")
        out["tile_nodes"] = np.zeros(int(out["tile_nptr"][-1]), np.int32)
        _check(lib.nsa_mesh_get_tiles(self._h, int(scatter), _ptr(out["tile_row"]), _ptr(out["tile_rptr"]),
                                      _ptr(out["run_elems"]), None, _ptr(out["tile_nodes"]), _ptr(out["runs"])),
               "nsa_mesh_get_tiles")
        return out

    Q1_REC_DTYPE = np.dtype([("loc", np.uint16, (4,)), ("own", np.uint16), ("pad0", np.uint16),
                             ("slot", np.uint16, (16,)), ("pad1", np.uint16, (2,))])

    def q1_tiles(self, scatter: int = ATOMIC):
        """Row-tile plan of a quadrilateral mesh: dict of tile_row, tile_eptr, elems, recs (Q1_REC_DTYPE),
        tile_nptr and tile_nodes."""
        i = self.info
        nt, nr = i.ntiles[scatter], i.tile_runs[scatter]
        out = dict(tile_row=np.zeros(nt + 1, np.int32), tile_eptr=np.zeros(nt + 1, np.int64),
                   elems=np.zeros(nr, np.int32), recs=np.zeros(nr, self.Q1_REC_DTYPE),
                   tile_nptr=np.zeros(nt + 1, np.int64))
        lib = load()
        _check(lib.nsa_mesh_get_q1_tiles(self._h, int(scatter), None, None, None, None, _ptr(out["tile_nptr"]), None),
               "nsa_mesh_get_q1_tiles")
        out["tile_nodes"] = np.zeros(int(out["tile_nptr"][-1]), np.int32)
        _check(lib.nsa_mesh_get_q1_tiles(self._h, int(scatter), _ptr(out["tile_row"]), _ptr(out["tile_eptr"]),
                                         _ptr(out["elems"]), _ptr(out["recs"]), None, _ptr(out["tile_nodes"])),
               "nsa_mesh_get_q1_tiles")
        return out

    def gather(self):
        """Gather plan: dict of tile_row, tile_nptr, tile_nodes, tile_eptr, elems, local_nodes
        (uint16 [records][4]), tile_pptr, pairs (uint16) and slots (uint32 [nnzb])."""
        i = self.info
        nt, nr, npr = i.gather_ntiles, i.gather_records, i.gather_pairs
        out = dict(tile_row=np.zeros(nt + 1, np.int32), tile_nptr=np.zeros(nt + 1, np.int64),
                   tile_eptr=np.zeros(nt + 1, np.int64), elems=np.zeros(nr, np.int32),
                   local_nodes=np.zeros((nr, 4), np.uint16), tile_pptr=np.zeros(nt + 1, np.int64),
                   pairs=np.zeros(npr, np.uint16), slots=np.zeros(self.nnzb, np.uint32))
        lib = load()
        _check(lib.nsa_mesh_get_gather(self._h, None, _ptr(out["tile_nptr"]), None, None, None, None, None, None,
                                       None), "nsa_mesh_get_gather")
        out["tile_nodes"] = np.zeros(int(out["tile_nptr"][-1]), np.int32)
        _check(lib.nsa_mesh_get_gather(self._h, _ptr(out["tile_row"]), None, _ptr(out["tile_nodes"]),
                                       _ptr(out["tile_eptr"]), _ptr(out["elems"]), _ptr(out["local_nodes"]),
                                       _ptr(out["tile_pptr"]), _ptr(out["pairs"]), _ptr(out["slots"])),
               "nsa_mesh_get_gather")
        return out

    def residual_tiles(self):
        """Residual plan: dict of tile_row, tile_eptr, elems, local_nodes (uint16 [records][4]),
        tile_nptr, tile_nodes."""
        i = self.info
        nt, nr = i.residual_ntiles, i.residual_records
        out = dict(tile_row=np.zeros(nt + 1, np.int32), tile_eptr=np.zeros(nt + 1, np.int64),
                   elems=np.zeros(nr, np.int32), local_nodes=np.zeros((nr, 4), np.uint16),
                   tile_nptr=np.zeros(nt + 1, np.int64))
        lib = load()
        _check(lib.nsa_mesh_get_residual_tiles(self._h, None, None, None, None, _ptr(out["tile_nptr"]), None),
               "nsa_mesh_get_residual_tiles")
        out["tile_nodes"] = np.zeros(int(out["tile_nptr"][-1]), np.int32)
        _check(lib.nsa_mesh_get_residual_tiles(self._h, _ptr(out["tile_row"]), _ptr(out["tile_eptr"]),
                                               _ptr(out["elems"]), _ptr(out["local_nodes"]), None,
                                               _ptr(out["tile_nodes"])), "nsa_mesh_get_residual_tiles")
        return out

    def upload(self, device="cuda", stream=None):
        import torch
        nbytes = int(self.info.ws_bytes)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        _check(load().nsa_mesh_upload(self._h, self.ws.data_ptr(), nbytes, _stream_handle(stream)),
               "nsa_mesh_upload")
        self.info = self._info()
        return self

    def release_host(self):
        _check(load().nsa_mesh_release_host(self._h), "nsa_mesh_release_host")

    def alloc_outputs(self, device="cuda"):
        import torch
        k = self.ndofn
        values = torch.empty((self.nnzb, k, k), dtype=torch.float64, device=device)
        rhs = torch.empty((self.npoin, k), dtype=torch.float64, device=device)
        return values, rhs

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.nsa_mesh_destroy(h)
            self._h = None


def make_options(precision=FP64, scatter=ATOMIC, accumulate=False, block_threads=0, kernel=KERNEL_AUTO,
                 vel_layout=VEL_AOS) -> Options:
    o = Options()
    o.precision, o.scatter, o.accumulate = int(precision), int(scatter), int(accumulate)
    o.block_threads, o.kernel, o.vel_layout = int(block_threads), int(kernel), int(vel_layout)
    return o


def _vel_shape(npoin: int, ndime: int, vel_layout: int):
    return (ndime, npoin) if vel_layout == VEL_SOA else (npoin, ndime)


def assemble(mesh: Mesh, vel, rho: float, mu: float, dt: float, *, precision=FP64, scatter=ATOMIC,
             accumulate=False, block_threads=0, kernel=KERNEL_AUTO, values=None, rhs=None, err_out=None,
             vel_layout=VEL_AOS, stream=None):
    """Launch nsa_assemble on the stream (default: torch's current stream); returns (values, rhs)
    as device tensors [nnzb][4][4] and [npoin][4] (allocated if not given). vel: [npoin][ndime], or
    [ndime][npoin] with vel_layout=VEL_SOA. err_out: optional float64 device tensor of 12 entries for
    the library's error report (see error_report)."""
    if mesh.ws is None:
        raise ValueError("the mesh has not been uploaded (Mesh.upload)")
    dev = mesh.ws.device
    if values is None or rhs is None:
        values, rhs = mesh.alloc_outputs(dev)
    k = mesh.ndofn
    pv = _dev_tensor(vel, _vel_shape(mesh.npoin, mesh.ndime, vel_layout), "vel", dev)
    pval = _dev_tensor(values, (mesh.nnzb, k, k), "values", dev)
    prhs = _dev_tensor(rhs, (mesh.npoin, k), "rhs", dev)
    o = make_options(precision, scatter, accumulate, block_threads, kernel, vel_layout)
    if err_out is not None:
        o.err_out = _dev_tensor(err_out, (12,), "err_out", dev)
    _check(load().nsa_assemble(mesh._h, pv, float(rho), float(mu), float(dt), C.byref(o), pval, prhs,
                               _stream_handle(stream)), "nsa_assemble")
    return values, rhs


def error_report(err_out) -> dict:
    """Relative error per class from an err_out tensor filled by assemble (synchronises): the largest
    difference against FP64 over the sampled elements divided by the largest FP64 magnitude."""
    e = err_out.cpu().tolist()
    return {k: (e[i] / e[6 + i] if e[6 + i] > 0 else 0.0) for i, k in enumerate(ERR_CLASSES)}


def assemble_residual(mesh: Mesh, vel, rho, mu, dt, precision=FP64, accumulate=False, rhsid=None, dt_rho=None,
                      mass_rho=None, vel_layout=VEL_AOS, stream=None):
    """Explicit-residual outputs (rhsid [npoin][3], dt_rho [npoin], mass_rho [npoin]) on the device;
    outputs are allocated when not given."""
    import torch
    if mesh.ws is None:
        raise ValueError("the mesh has not been uploaded (Mesh.upload)")
    dev = mesh.ws.device
    if rhsid is None:
        rhsid = torch.empty((mesh.npoin, 3), dtype=torch.float64, device=dev)
    if dt_rho is None:
        dt_rho = torch.empty(mesh.npoin, dtype=torch.float64, device=dev)
    if mass_rho is None:
        mass_rho = torch.empty(mesh.npoin, dtype=torch.float64, device=dev)
    ptrs = (_dev_tensor(vel, _vel_shape(mesh.npoin, 3, vel_layout), "vel", dev),
            _dev_tensor(rhsid, (mesh.npoin, 3), "rhsid", dev),
            _dev_tensor(dt_rho, (mesh.npoin,), "dt_rho", dev), _dev_tensor(mass_rho, (mesh.npoin,), "mass_rho", dev))
    o = make_options(precision, ATOMIC, accumulate, vel_layout=vel_layout)
    _check(load().nsa_assemble_residual(mesh._h, ptrs[0], float(rho), float(mu), float(dt), C.byref(o), *ptrs[1:],
                                        _stream_handle(stream)), "nsa_assemble_residual")
    return rhsid, dt_rho, mass_rho


def fill_uniform(out, seed: int, lo: float = -1.0, hi: float = 1.0, stream=None):
    """Fill a contiguous float64 device tensor with the library's seeded uniform values."""
    import torch
    if not (isinstance(out, torch.Tensor) and out.dtype == torch.float64 and out.is_contiguous() and out.is_cuda):
        raise ValueError("out must be a contiguous float64 device tensor")
    _check(load().nsa_fill_uniform(out.data_ptr(), out.numel(), int(seed) % (1 << 64), float(lo), float(hi),
                                   _stream_handle(stream)), "nsa_fill_uniform")
    return out


def bandwidth_probe(kind: int, src=None, dst=None, stream=None):
    """One pass of a plain HBM stream (nsa_bandwidth_probe): PROBE_READ of src, PROBE_WRITE of dst or
    PROBE_COPY src -> dst (contiguous float64 device tensors of the same, even size; for a read, dst
    is a one-element device tensor)."""
    import torch
    for t in (src, dst):
        if t is not None and not (isinstance(t, torch.Tensor) and t.dtype == torch.float64 and t.is_contiguous()
                                  and t.is_cuda):
            raise ValueError("probe buffers must be contiguous float64 device tensors")
    n = (src if kind != PROBE_WRITE else dst).numel()
    if kind == PROBE_COPY and dst.numel() < n:
        raise ValueError("dst smaller than src")
    _check(load().nsa_bandwidth_probe(int(kind), _ptr(src), _ptr(dst), n, _stream_handle(stream)),
           "nsa_bandwidth_probe")


def assemble_batched_static(meshes, vels, rho, mu, dt, outputs, precision=MIXED, scatter=ATOMIC, accumulate=False,
                            block_threads=0, vel_layout=VEL_AOS, stream=None):
    """The batched form without a batch handle or workspace (nsa_assemble_batched_static): one launch
    over every tile of the uploaded meshes, the tables in the library's fixed per-GPU device array.
    No device allocation. At most 256 meshes and 2^20 tiles; calls that overlap on one GPU race.
    vels: device tensors [npoin][3] ([3][npoin] with vel_layout=VEL_SOA); rho, mu, dt: sequences;
    outputs: [(values, rhs), ...]."""
    meshes, vels, outputs = list(meshes), list(vels), list(outputs)
    n = len(meshes)
    if not (len(vels) == len(outputs) == len(rho) == len(mu) == len(dt) == n):
        raise ValueError(f"assemble_batched_static: expected {n} velocities, outputs and parameters each")
    P = C.c_void_p
    hs = (P * n)(*[m._h.value for m in meshes])
    if any(m.ws is None for m in meshes):
        raise ValueError("assemble_batched_static: every mesh must be uploaded (Mesh.upload)")
    v = (P * n)(*[_dev_tensor(x, _vel_shape(m.npoin, 3, vel_layout), f"vels[{i}]", m.ws.device)
                  for i, (x, m) in enumerate(zip(vels, meshes))])
    va = (P * n)(*[_dev_tensor(o[0], (m.nnzb, 4, 4), f"outputs[{i}][0]", m.ws.device)
                   for i, (o, m) in enumerate(zip(outputs, meshes))])
    ra = (P * n)(*[_dev_tensor(o[1], (m.npoin, 4), f"outputs[{i}][1]", m.ws.device)
                   for i, (o, m) in enumerate(zip(outputs, meshes))])
    dr = (C.c_double * n)(*[float(x) for x in rho])
    dm = (C.c_double * n)(*[float(x) for x in mu])
    dd = (C.c_double * n)(*[float(x) for x in dt])
    o = make_options(precision, scatter, accumulate=accumulate, block_threads=block_threads, vel_layout=vel_layout)
    _check(load().nsa_assemble_batched_static(n, hs, v, dr, dm, dd, va, ra, C.byref(o), _stream_handle(stream)),
           "nsa_assemble_batched_static")


class Batch:
    """Many uploaded meshes assembled by one launch (nsa_batch_*). Keeps references to
    the meshes, its device workspace and the last inputs so that nothing it points at is freed.

    Batch(meshes, ...) fixes its members; Batch.reserve(max_meshes, max_tiles, ...) makes an empty
    reusable batch whose members are set per launch with reset()."""

    def __init__(self, meshes=None, scatter=ATOMIC, device="cuda", stream=None, *, _capacity=None):
        import torch
        lib = load()
        self.scatter = int(scatter)
        h = C.c_void_p()
        if _capacity is None:
            self.meshes = list(meshes)
            arr = (C.c_void_p * len(self.meshes))(*[m._h.value for m in self.meshes])
            _check(lib.nsa_batch_create(len(self.meshes), arr, self.scatter, C.byref(h)), "nsa_batch_create")
        else:
            self.meshes = []
            _check(lib.nsa_batch_reserve(int(_capacity[0]), int(_capacity[1]), self.scatter, C.byref(h)),
                   "nsa_batch_reserve")
        self._h = h
        self._refresh()
        self.ws = torch.empty(int(self.ws_bytes), dtype=torch.uint8, device=device)
        _check(lib.nsa_batch_upload(h, self.ws.data_ptr(), int(self.ws_bytes), _stream_handle(stream)),
               "nsa_batch_upload")
        self._keep = None

    @classmethod
    def reserve(cls, max_meshes, max_tiles, scatter=ATOMIC, device="cuda", stream=None):
        return cls(None, scatter, device, stream, _capacity=(max_meshes, max_tiles))

    def _refresh(self):
        ws, nt, ne, lds = C.c_size_t(), C.c_int64(), C.c_int64(), C.c_int32()
        _check(load().nsa_batch_get_info(self._h, C.byref(ws), C.byref(nt), C.byref(ne), C.byref(lds)),
               "nsa_batch_get_info")
        self.ws_bytes, self.ntiles, self.nelem, self.lds_bytes = ws.value, nt.value, ne.value, lds.value

    def reset(self, meshes):
        """New members (uploaded meshes; repeats allowed). Call set_inputs before the next launch."""
        meshes = list(meshes)
        arr = (C.c_void_p * len(meshes))(*[m._h.value for m in meshes])
        _check(load().nsa_batch_reset(self._h, len(meshes), arr), "nsa_batch_reset")
        self.meshes = meshes
        self._refresh()

    def alloc_outputs(self, device="cuda"):
        return [m.alloc_outputs(device) for m in self.meshes]

    def set_inputs(self, vels, rho, mu, dt, outputs, accumulate=False, stream=None):
        """vels: device tensors [npoin][3]; rho, mu, dt: sequences; outputs: [(values, rhs), ...]."""
        n = len(self.meshes)
        vels, outputs = list(vels), list(outputs)
        if not (len(vels) == len(outputs) == len(rho) == len(mu) == len(dt) == n):
            raise ValueError(f"set_inputs: expected {n} velocities, outputs and parameters each")
        dev = self.ws.device
        P = C.c_void_p
        v = (P * n)(*[_dev_tensor(x, (m.npoin, 3), f"vels[{i}]", dev) for i, (x, m) in enumerate(zip(vels, self.meshes))])
        va = (P * n)(*[_dev_tensor(o[0], (m.nnzb, 4, 4), f"outputs[{i}][0]", dev)
                       for i, (o, m) in enumerate(zip(outputs, self.meshes))])
        ra = (P * n)(*[_dev_tensor(o[1], (m.npoin, 4), f"outputs[{i}][1]", dev)
                       for i, (o, m) in enumerate(zip(outputs, self.meshes))])
        dr = (C.c_double * n)(*[float(x) for x in rho])
        dm = (C.c_double * n)(*[float(x) for x in mu])
        dd = (C.c_double * n)(*[float(x) for x in dt])
        _check(load().nsa_batch_set_inputs(self._h, v, dr, dm, dd, va, ra, int(bool(accumulate)),
                                           _stream_handle(stream)), "nsa_batch_set_inputs")
        self._keep = (vels, outputs)

    def assemble(self, precision=MIXED, grid_wgs=0, block_threads=0, stream=None):
        o = make_options(precision, self.scatter, block_threads=block_threads)
        _check(load().nsa_assemble_batched(self._h, C.byref(o), int(grid_wgs), _stream_handle(stream)),
               "nsa_assemble_batched")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.nsa_batch_destroy(h)
            self._h = None
