"""MI355X composite spectral direct solver (Gillman & Martinsson, sections 2-5).

Thin Python binding of ``libhps.so``: every function marshals arguments to the
C entry point of the same name (declared in ``include/hps.h``).  All numerical
work runs in the HIP kernels of the library; PyTorch is used only for device
memory and streams.  Arrays may be NumPy arrays (host) or torch tensors; CUDA
(ROCm) tensors are passed as device pointers, on the current stream.
"""
from __future__ import annotations

import ctypes as C
from typing import List, Optional, Sequence

import numpy as np

from ._lib import (HPS_EINVAL, HPS_ENOTCONV, HPS_ESINGULAR, HPS_FP64, HPS_MIXED_BF16X6,
                   HPS_MIXED_SPLIT32, HPS_SURROGATE, BuildOpts, HpsError, OpInfo, Problem, SolveInfo, SolveOpts,
                   check, lib)

__all__ = ["HpsError", "HPS_FP64", "HPS_MIXED_SPLIT32", "HPS_MIXED_BF16X6", "HPS_SURROGATE",
           "HPS_EINVAL",
           "HPS_ESINGULAR", "HPS_ENOTCONV", "Operator", "cheb_nodes", "gauss_nodes_grid",
           "boundary_ids", "leaf_dtn", "build_solution_operator", "build_batch", "solve_batch",
           "leaf_tables", "plan_box", "version", "lib", "batched_solve", "batched_gemm",
           "Surrogate", "hbs_sizes", "hbs_pack", "hbs_apply", "hbs_invert", "hbs_solve",
           "hbs_unpack_inverse", "hbs_compress"]


def version() -> str:
    return lib.hps_version().decode()


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _dev(x) -> bool:
    return _is_torch(x) and x.is_cuda


def _ptr(x):
    """Pointer of a contiguous float64/int32 NumPy array or torch tensor."""
    if _is_torch(x):
        assert x.is_contiguous(), "tensor must be contiguous"
        return C.c_void_p(x.data_ptr())
    assert x.flags["C_CONTIGUOUS"], "array must be C-contiguous"
    return x.ctypes.data_as(C.c_void_p)


def _stream(x=None):
    import torch
    if x is not None and _dev(x):
        return C.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)
    if torch.cuda.is_available():
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(0)


def _f64(x):
    if _is_torch(x):
        import torch
        assert x.dtype == torch.float64, "float64 tensor required"
        return x.contiguous()
    return np.ascontiguousarray(x, dtype=np.float64)


# ---- discretization helpers (host) -----------------------------------------

def cheb_nodes(box, nleaf, p: int) -> np.ndarray:
    nx, ny = nleaf
    xy = np.empty((nx * ny, p * p, 2))
    b = (C.c_double * 4)(*box)
    nl = (C.c_int * 2)(nx, ny)
    check(lib.hps_cheb_nodes(b, nl, p, _ptr(xy)))
    return xy


def gauss_nodes_grid(box, nleaf, q: int) -> np.ndarray:
    b = (C.c_double * 4)(*box)
    nl = (C.c_int * 2)(*nleaf)
    N = C.c_int()
    check(lib.hps_gauss_nodes_grid(b, nl, q, None, C.byref(N)))
    xy = np.empty((N.value, 2))
    check(lib.hps_gauss_nodes_grid(b, nl, q, _ptr(xy), C.byref(N)))
    return xy


def boundary_ids(nleaf, q: int) -> np.ndarray:
    nl = (C.c_int * 2)(*nleaf)
    n = C.c_int()
    check(lib.hps_boundary_ids(nl, q, None, C.byref(n)))
    ids = np.empty(n.value, dtype=np.int32)
    check(lib.hps_boundary_ids(nl, q, _ptr(ids), C.byref(n)))
    return ids


def leaf_tables(p: int, q: int, hx: float, hy: float) -> dict:
    n, m = (p - 2) ** 2, 4 * q
    out = dict(Dx=np.empty((p, p)), Dy=np.empty((p, p)), Dxx=np.empty((p, p)),
               Dyy=np.empty((p, p)), G=np.empty((5, n, m)), P0=np.empty((m, m)),
               P1=np.empty((m, n)), Ji=np.empty(n, dtype=np.int32))
    check(lib.hps_leaf_tables(p, q, hx, hy, *[_ptr(out[k]) for k in
                                              ("Dx", "Dy", "Dxx", "Dyy", "G", "P0", "P1", "Ji")]))
    return out


def plan_box(nleaf, q: int, box: int) -> dict:
    nl = (C.c_int * 2)(*nleaf)
    nb = C.c_int()
    rec = np.empty(8, dtype=np.int32)
    sizes = np.zeros(4, dtype=np.int32)
    check(lib.hps_plan_box(nl, q, box, _ptr(rec), _ptr(sizes), None, None, None, None, None,
                           C.byref(nb)))
    me, m3 = int(sizes[0]), int(sizes[1])
    arrs = dict(pmap=np.empty(me, np.int32), a3=np.empty(m3, np.int32), b3=np.empty(m3, np.int32),
                Ie=np.empty(me, np.int32), Ii=np.empty(m3, np.int32))
    if me:
        check(lib.hps_plan_box(nl, q, box, _ptr(rec), _ptr(sizes), _ptr(arrs["pmap"]),
                               _ptr(arrs["a3"]), _ptr(arrs["b3"]), _ptr(arrs["Ie"]),
                               _ptr(arrs["Ii"]), C.byref(nb)))
    return dict(rec=rec, sizes=sizes, n_boxes=nb.value, **arrs)


# ---- leaf stage ----------------------------------------------------------------

def leaf_dtn(coeffs, hx: float, hy: float, p: int, q: int, out=None):
    """Leaf DtN maps (section 3.2) of a batch of equal leaves; device tensors only."""
    import torch
    coeffs = _f64(coeffs)
    assert _dev(coeffs), "hps_leaf_dtn takes device tensors"
    nl = coeffs.shape[0]
    if out is None:
        out = torch.empty((nl, 4 * q, 4 * q), dtype=torch.float64, device=coeffs.device)
    check(lib.hps_leaf_dtn(_ptr(coeffs), nl, hx, hy, p, q, _ptr(out), _stream(coeffs)))
    return out


# ---- batched dense layer ---------------------------------------------------------

def batched_solve(M, B, X=None):
    """X_i = M_i^-1 B_i (LU with partial pivoting on the device); device tensors."""
    import torch
    M = _f64(M)
    B = _f64(B)
    assert _dev(M) and _dev(B)
    nprob, n, m = B.shape
    if X is None:
        X = torch.empty_like(B)
    check(lib.hps_batched_solve(_ptr(M), _ptr(B), n, m, nprob, _ptr(X), _stream(M)))
    return X


def batched_gemm(A, B, C, alpha: float = 1.0, split32: bool = False, bf16x6: bool = False):
    """C_i += alpha A_i B_i on the device: FP64 MFMA, the split-FP32 form, or BF16 MFMA on
    three-slice splits."""
    A = _f64(A)
    B = _f64(B)
    assert _dev(A) and _dev(B) and _dev(C)
    assert not (split32 and bf16x6)
    nprob, Mr, K = A.shape
    Nc = B.shape[2]
    prec = 1 if split32 else (2 if bf16x6 else 0)
    check(lib.hps_batched_gemm(_ptr(A), _ptr(B), _ptr(C), Mr, Nc, K, nprob, alpha, prec,
                               _stream(A)))
    return C


# ---- HBS matrices (sections 6-7) -------------------------------------------
def hbs_sizes(L: int, m: int, k: int):
    """(doubles in the factor buffer, doubles in the inverse buffer) of an HBS matrix of
    m 2^L rows and rank k (layouts in include/hps.h)."""
    nf, ni = C.c_size_t(), C.c_size_t()
    check(lib.hps_hbs_sizes(L, m, k, C.byref(nf), C.byref(ni)))
    return nf.value, ni.value


def hbs_pack(D, U, Vt, Up, Vtp, B):
    """The factor buffer (a 1-D array or tensor) from its blocks: D [2^L, m, m],
    U [2^L, m, k], Vt [2^L, k, m], Up[l] [2^l, 2k, k] and Vtp[l] [2^l, k, 2k] for
    l = 1 .. L-1 (dicts or lists indexed by l), B[l] [2^l, 2k, 2k] for l = 0 .. L-1."""
    L = int(D.shape[0]).bit_length() - 1
    parts = [D, U, Vt]
    for l in range(L - 1, 0, -1):
        parts += [Up[l], Vtp[l]]
    parts += [B[l] for l in range(L - 1, -1, -1)]
    if _is_torch(D):
        import torch
        return torch.cat([p.reshape(-1) for p in parts]).contiguous()
    return np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1) for p in parts])


def hbs_unpack_inverse(inv, L: int, m: int, k: int):
    """Views of the inverse buffer: dicts E, Fs (F*), G by level (G[0] the root's block)."""
    E, Fs, G = {}, {}, {}
    o = 0
    for l in range(L, 0, -1):
        n = m if l == L else 2 * k
        nn = 1 << l
        E[l] = inv[o:o + nn * n * k].reshape(nn, n, k)
        o += nn * n * k
        Fs[l] = inv[o:o + nn * k * n].reshape(nn, k, n)
        o += nn * k * n
        G[l] = inv[o:o + nn * n * n].reshape(nn, n, n)
        o += nn * n * n
    G[0] = inv[o:o + 4 * k * k].reshape(2 * k, 2 * k)
    return E, Fs, G


def hbs_apply(factors, x, L: int, m: int, k: int, y=None):
    """y = H x for the HBS matrix in ``factors`` (device tensors; x, y [m 2^L, nrhs])."""
    import torch
    assert _dev(factors) and _dev(x)
    x = _f64(x)
    nrhs = x.shape[1] if x.dim() == 2 else 1
    if y is None:
        y = torch.empty_like(x)
    check(lib.hps_hbs_apply(L, m, k, _ptr(factors), _ptr(x), _ptr(y), nrhs, _stream(x)))
    return y


def hbs_compress(H, L: int, k: int, omega, psit, factors=None):
    """Brute-force compression of a dense device matrix (or of an ``Operator``'s root DtN)
    into HBS factors of rank k; omega [M, k] and psit [k, M] are the caller's standard
    normal samples (device tensors)."""
    import torch
    assert _dev(omega) and _dev(psit)
    omega, psit = _f64(omega), _f64(psit)
    if isinstance(H, Operator):
        M = H.n_bdry
        dev = omega.device
    else:
        assert _dev(H)
        H = _f64(H)
        M = H.shape[0]
        dev = H.device
    m = M >> L
    if factors is None:
        factors = torch.empty(hbs_sizes(L, m, k)[0], dtype=torch.float64, device=dev)
    if isinstance(H, Operator):
        check(lib.hps_root_dtn_compress(H._h, L, k, _ptr(omega), _ptr(psit), _ptr(factors),
                                        _stream(omega)))
    else:
        check(lib.hps_hbs_compress(L, m, k, _ptr(H), H.shape[1], _ptr(omega), _ptr(psit),
                                   _ptr(factors), _stream(H)))
    return factors


def hbs_invert(factors, L: int, m: int, k: int, inverse=None):
    """Algorithm 3 on the device: the inverse factors {E, F, G} as one buffer."""
    import torch
    assert _dev(factors)
    if inverse is None:
        inverse = torch.empty(hbs_sizes(L, m, k)[1], dtype=torch.float64, device=factors.device)
    check(lib.hps_hbs_invert(L, m, k, _ptr(factors), _ptr(inverse), _stream(factors)))
    return inverse


def hbs_solve(inverse, x, L: int, m: int, k: int, y=None):
    """Algorithm 4 on the device: y = H^-1 x from the buffer of ``hbs_invert``."""
    import torch
    assert _dev(inverse) and _dev(x)
    x = _f64(x)
    nrhs = x.shape[1] if x.dim() == 2 else 1
    if y is None:
        y = torch.empty_like(x)
    check(lib.hps_hbs_solve(L, m, k, _ptr(inverse), _ptr(x), _ptr(y), nrhs, _stream(x)))
    return y


def tune_set(knob: str, value: int) -> None:
    """Forces a kernel variant ("leaf_variant", "gemm_variant", "gj_variant"); -1 clears."""
    check(lib.hps_tune_set(knob.encode(), int(value)))


def bgj_fallbacks() -> int:
    """Merge levels (all builds of this process) whose blocked Gauss-Jordan fell back to
    partial pivoting."""
    n = C.c_longlong()
    check(lib.hps_bgj_fallbacks(C.byref(n)))
    return n.value


def autotune(shapes, stream=None) -> float:
    """Times every kernel variant for the builds of the given problem shapes
    (dicts with nleaf, p, q and optionally box) and keeps the fastest per shape
    bucket in this process's tuning table.  Returns the seconds spent."""
    arr = (Problem * len(shapes))()
    for i, sh in enumerate(shapes):
        arr[i].coeffs = None
        box = sh.get("box", (0.0, 1.0, 0.0, 1.0))
        for k in range(4):
            arr[i].box[k] = float(box[k])
        arr[i].nleaf[0], arr[i].nleaf[1] = int(sh["nleaf"][0]), int(sh["nleaf"][1])
        arr[i].p, arr[i].q = int(sh["p"]), int(sh["q"])
    sec = C.c_double()
    check(lib.hps_autotune(arr, len(shapes), _stream(stream), C.byref(sec)))
    return sec.value


def tune_save(path) -> None:
    check(lib.hps_tune_save(str(path).encode()))


def tune_load(path) -> None:
    check(lib.hps_tune_load(str(path).encode()))


def tune_reset() -> None:
    check(lib.hps_tune_reset())


# ---- learned leaf surrogate -------------------------------------------------------

class Surrogate:
    """Owner of an ``hps_surrogate`` (MLP leaf-DtN surrogate in device memory)."""

    def __init__(self, handle):
        self._h = handle
        dims = np.zeros(7, dtype=np.int32)
        sc = C.c_double()
        check(lib.hps_surrogate_info(self._h, _ptr(dims), C.byref(sc)))
        self.p, self.q, self.hidden, self.rank, self.D, self.O, self.step = (int(x) for x in dims)
        self.m = 4 * self.q

    @classmethod
    def create(cls, p, q, hx, hy, hidden=256, rank=16, seed=0):
        h = C.c_void_p()
        check(lib.hps_surrogate_create(p, q, hx, hy, hidden, rank, seed, _stream(), C.byref(h)))
        return cls(h)

    @classmethod
    def load(cls, path):
        h = C.c_void_p()
        check(lib.hps_surrogate_load(str(path).encode(), _stream(), C.byref(h)))
        return cls(h)

    @property
    def handle(self):
        return self._h

    @property
    def out_scale(self) -> float:
        sc = C.c_double()
        check(lib.hps_surrogate_info(self._h, None, C.byref(sc)))
        return sc.value

    def __del__(self):
        if getattr(self, "_h", None):
            lib.hps_surrogate_destroy(self._h)
            self._h = None

    def train(self, coeffs, T, epochs=10, batch=256, lr=1e-3, seed=0):
        coeffs, T = _f64(coeffs), _f64(T)
        assert _dev(coeffs) and _dev(T)
        hist = np.zeros(epochs)
        L = C.c_double()
        check(lib.hps_surrogate_train(self._h, _ptr(coeffs), _ptr(T), coeffs.shape[0], epochs,
                                      batch, lr, seed, _stream(coeffs), C.byref(L), _ptr(hist)))
        return hist

    def grad(self, coeffs, T):
        coeffs, T = _f64(coeffs), _f64(T)
        n = coeffs.shape[0]
        sizes = [self.hidden * self.D, self.hidden, self.hidden * self.hidden, self.hidden,
                 self.O * self.hidden, self.O]
        g = np.zeros(sum(sizes), dtype=np.float32)
        L = C.c_double()
        check(lib.hps_surrogate_grad(self._h, _ptr(coeffs), _ptr(T), n, _ptr(g), C.byref(L),
                                     _stream(coeffs)))
        out, o = {}, 0
        for name, s_ in zip(("W1", "b1", "W2", "b2", "W3", "b3"), sizes):
            out[name] = g[o:o + s_].astype(np.float64)
            o += s_
        return L.value, out

    def predict(self, coeffs, out=None):
        import torch
        coeffs = _f64(coeffs)
        n = coeffs.shape[0]
        if out is None:
            out = torch.empty((n, self.m, self.m), dtype=torch.float64, device=coeffs.device)
        check(lib.hps_surrogate_predict(self._h, _ptr(coeffs), n, _ptr(out), _stream(coeffs)))
        return out

    def state(self) -> dict:
        """Shape, normalisation, scale, training ranges and FP32 weights."""
        n = C.c_size_t()
        check(lib.hps_surrogate_get_state(self._h, None, C.byref(n)))
        buf = np.zeros(n.value, dtype=np.uint8)
        check(lib.hps_surrogate_get_state(self._h, _ptr(buf), C.byref(n)))
        meta = buf[:14 * 8].view(np.float64)
        f = buf[14 * 8:].view(np.float32)
        D, H, O = self.D, self.hidden, self.O
        st = dict(out_scale=float(meta[6]), step=int(meta[7]), lo=meta[8:11].copy(),
                  hi=meta[11:14].copy())
        o = 0
        for name, s_ in (("mu", D), ("sigma", D), ("W1", H * D), ("b1", H), ("W2", H * H),
                         ("b2", H), ("W3", O * H), ("b3", O)):
            st[name] = f[o:o + s_].copy()
            o += s_
        st["W1"] = st["W1"].reshape(H, D)
        st["W2"] = st["W2"].reshape(H, H)
        st["W3"] = st["W3"].reshape(O, H)
        return st

    def save(self, path):
        check(lib.hps_surrogate_save(self._h, str(path).encode()))


# ---- launch timing -----------------------------------------------------------------

PROF_CLASSES = {"leaf_assemble": 0, "lu_panel": 1, "swap_trsm": 2, "lu_update": 3,
                "back_subst": 4, "gemm": 5, "gemm_split32": 6, "merge_gather": 7,
                "downward": 8, "residual": 9, "upward": 10, "leaf_lu": 11, "mlp_train": 12,
                "mlp_infer": 13, "postprocess": 14, "gemm_bf16x6": 15,
                "body_flux": 16, "leaf_gemm": 17, "merge_s": 18, "bgj_diag": 19,
                "bgj_rows": 20, "bgj_update": 21, "merge_small": 22, "hbs": 23}


def mem_trim() -> int:
    """Frees the parked operators (destroyed operators kept for the next build of their
    shape) and the device blocks the library keeps cached for reuse; returns the bytes freed."""
    f = C.c_size_t()
    check(lib.hps_mem_trim(C.byref(f)))
    return f.value


def mem_stats() -> dict:
    """Bytes of device memory the library holds cached (free) and in use."""
    a, b = C.c_size_t(), C.c_size_t()
    check(lib.hps_mem_stats(C.byref(a), C.byref(b)))
    return dict(cached=a.value, in_use=b.value)


def prof_enable(classes) -> None:
    mask = 0
    for c in classes:
        mask |= 1 << (PROF_CLASSES[c] if isinstance(c, str) else int(c))
    check(lib.hps_prof_enable(mask))


def prof_reset() -> None:
    check(lib.hps_prof_reset())


def prof_query(cls) -> dict:
    ms, n, fl, by = C.c_double(), C.c_longlong(), C.c_double(), C.c_double()
    c = PROF_CLASSES[cls] if isinstance(cls, str) else int(cls)
    check(lib.hps_prof_query(c, C.byref(ms), C.byref(n), C.byref(fl), C.byref(by)))
    return dict(ms=ms.value, launches=n.value, flops=fl.value, bytes=by.value)


# ---- operator --------------------------------------------------------------------

class Operator:
    """Owner of an ``hps_op`` (solution operators in device memory)."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle
        info = OpInfo()
        check(lib.hps_op_query(self._h, C.byref(info)))
        self.nx, self.ny, self.p, self.q = info.nx, info.ny, info.p, info.q
        self.N, self.n_bdry = info.N, info.n_bdry
        self.n_boxes, self.n_levels = info.n_boxes, info.n_levels
        self.mode = info.mode
        self.box = tuple(info.box)
        self.bytes_S, self.bytes_total, self.flops_build = info.bytes_S, info.bytes_total, info.flops_build
        self.n_fallback_leaves = info.n_fallback_leaves
        self.judge_worst = info.judge_worst
        self.n_judged = info.n_judged

    def __del__(self):
        try:
            self.destroy()
        except (AttributeError, TypeError):
            pass  # interpreter shutdown: the library binding may already be gone

    def destroy(self):
        if getattr(self, "_h", None):
            lib.hps_destroy(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    @property
    def n_tot(self) -> int:
        """Total discretization points: Chebyshev grid points plus Gauss nodes (Table 1's N_tot)."""
        return (self.nx * (self.p - 1) + 1) * (self.ny * (self.p - 1) + 1) + self.N

    def gauss_nodes(self) -> np.ndarray:
        xy = np.empty((self.N, 2))
        N = C.c_int()
        check(lib.hps_gauss_nodes(self._h, _ptr(xy), C.byref(N)))
        return xy

    def boundary_nodes(self) -> np.ndarray:
        xy = np.empty((self.n_bdry, 2))
        n = C.c_int()
        check(lib.hps_boundary_nodes(self._h, _ptr(xy), C.byref(n)))
        return xy

    def solve(self, f, u=None, refine: bool = False, tol: float = 1e-12, max_iter: int = 10,
              info: Optional[dict] = None):
        """Algorithm 2: f [nrhs, n_bdry] -> u [nrhs, N]."""
        f = _f64(f)
        if f.ndim == 1:
            f = f.reshape(1, -1)
        nrhs = f.shape[0]
        dev = _dev(f)
        if u is None:
            if dev:
                import torch
                u = torch.empty((nrhs, self.N), dtype=torch.float64, device=f.device)
            else:
                u = np.empty((nrhs, self.N))
        so = SolveOpts(_stream(f) if dev else None, int(dev), int(refine), tol, max_iter)
        si = SolveInfo()
        check(lib.hps_solve(self._h, _ptr(f), nrhs, _ptr(u), C.byref(so), C.byref(si)))
        if info is not None:
            info.update(iters=si.iters, last_update_rel=si.last_update_rel,
                        first_update_rel=si.first_update_rel,
                        n_fallback_leaves=si.n_fallback_leaves)
        return u

    def root_dtn_apply(self, f, v=None):
        f = _f64(f)
        if f.ndim == 1:
            f = f.reshape(1, -1)
        dev = _dev(f)
        if v is None:
            if dev:
                import torch
                v = torch.empty_like(f)
            else:
                v = np.empty_like(f)
        so = SolveOpts(_stream(f) if dev else None, int(dev), 0, 0.0, 0)
        check(lib.hps_root_dtn_apply(self._h, _ptr(f), f.shape[0], _ptr(v), C.byref(so)))
        return v

    def postprocess(self, u, uc=None):
        """Section 5.3: u [nrhs, N] at the Gauss nodes -> uc [nrhs, nx*ny, p*p] on every
        leaf's Chebyshev grid (operator built with keep_leaf_solution=True)."""
        u = _f64(u)
        if u.ndim == 1:
            u = u.reshape(1, -1)
        dev = _dev(u)
        shape = (u.shape[0], self.nx * self.ny, self.p * self.p)
        if uc is None:
            if dev:
                import torch
                uc = torch.empty(shape, dtype=torch.float64, device=u.device)
            else:
                uc = np.empty(shape)
        so = SolveOpts(_stream(u) if dev else None, int(dev), 0, 0.0, 0)
        check(lib.hps_postprocess(self._h, _ptr(u), u.shape[0], _ptr(uc), C.byref(so)))
        return uc

    def solve_body(self, f, g, grid: bool = False):
        """A u = g, u = f on the boundary: f [nrhs, n_bdry], g [nrhs, nx*ny, p*p] at the
        Chebyshev nodes.  Returns u [nrhs, N], and with grid=True also the solution on
        every leaf grid [nrhs, nx*ny, p*p] (operator built with keep_factors, and
        keep_leaf_solution for the grid)."""
        f = _f64(f)
        g = _f64(g)
        if f.ndim == 1:
            f = f.reshape(1, -1)
        nrhs = f.shape[0]
        shape = (nrhs, self.nx * self.ny, self.p * self.p)
        assert tuple(g.shape) == shape, "g must be [nrhs, nx*ny, p*p]"
        dev = _dev(f)
        assert _dev(g) == dev
        if dev:
            import torch
            u = torch.empty((nrhs, self.N), dtype=torch.float64, device=f.device)
            uc = torch.empty(shape, dtype=torch.float64, device=f.device) if grid else None
        else:
            u = np.empty((nrhs, self.N))
            uc = np.empty(shape) if grid else None
        so = SolveOpts(_stream(f) if dev else None, int(dev), 0, 0.0, 0)
        check(lib.hps_solve_body(self._h, _ptr(f), _ptr(g), nrhs, _ptr(u),
                                 _ptr(uc) if grid else None, C.byref(so)))
        return (u, uc) if grid else u

    def interface_residual(self, u, r=None):
        import torch
        u = _f64(u)
        assert _dev(u)
        if r is None:
            r = torch.empty_like(u)
        check(lib.hps_interface_residual(self._h, _ptr(u), u.shape[0], _ptr(r), _stream(u)))
        return r

    def interface_residual_noalloc(self, u, r):
        """hps_interface_residual_noalloc: the residual into a caller-given r, with no
        allocation in the library (its scratch is a fixed per-device array)."""
        u, r = _f64(u), _f64(r)
        assert _dev(u) and _dev(r) and r.shape == u.shape
        check(lib.hps_interface_residual_noalloc(self._h, _ptr(u), u.shape[0], _ptr(r),
                                                 _stream(u)))
        return r

    def solve_with_sources(self, f, s, u=None):
        import torch
        f = _f64(f)
        s = _f64(s)
        assert _dev(f) and _dev(s)
        if u is None:
            u = torch.empty((f.shape[0], self.N), dtype=torch.float64, device=f.device)
        check(lib.hps_solve_with_sources(self._h, _ptr(f), _ptr(s), f.shape[0], _ptr(u),
                                         _stream(f)))
        return u

    def box_record(self, b: int) -> np.ndarray:
        rec = np.empty(8, dtype=np.int32)
        check(lib.hps_box(self._h, b, _ptr(rec)))
        return rec

    def export_S(self, b: int) -> np.ndarray:
        r, c = C.c_int(), C.c_int()
        check(lib.hps_export_S(self._h, b, None, C.byref(r), C.byref(c)))
        S = np.empty((r.value, c.value))
        check(lib.hps_export_S(self._h, b, _ptr(S), C.byref(r), C.byref(c)))
        return S

    def level_conditions(self) -> np.ndarray:
        """Per tree depth: the largest max|M| / min |pivot| of its merge systems M."""
        n = C.c_int()
        check(lib.hps_level_conditions(self._h, None, C.byref(n)))
        out = np.zeros(n.value)
        check(lib.hps_level_conditions(self._h, _ptr(out), C.byref(n)))
        return out

    def export_root_dtn(self) -> np.ndarray:
        T = np.empty((self.n_bdry, self.n_bdry))
        check(lib.hps_export_root_dtn(self._h, _ptr(T)))
        return T

    def export_leaf_dtn(self, leaf: int) -> np.ndarray:
        m = 4 * self.q
        T = np.empty((m, m))
        check(lib.hps_export_leaf_dtn(self._h, leaf, _ptr(T)))
        return T


def _build_opts(mode, stream, device_ptrs, keep_factors, root_dtn, surrogate=None,
                judge_samples=64, judge_tol=1e-6, keep_leaf_solution=False,
                keep_body_operator=False, pivot_tol=0.0):
    return BuildOpts(mode, stream, int(device_ptrs), 1, int(keep_factors), int(root_dtn),
                     float(pivot_tol),
                     surrogate.handle if surrogate is not None else None, int(judge_samples),
                     float(judge_tol), int(keep_leaf_solution), int(keep_body_operator))


def build_solution_operator(coeffs, box, nleaf, p: int, q: int, mode: int = HPS_FP64,
                            keep_factors: bool = False, root_dtn: bool = True, surrogate=None,
                            judge_samples: int = 64, judge_tol: float = 1e-6,
                            keep_leaf_solution: bool = False,
                            keep_body_operator: bool = False,
                            pivot_tol: float = 0.0) -> Operator:
    """Algorithm 1.  coeffs [nx*ny, 6, p*p] (c11, c12, c22, c1, c2, c at Chebyshev nodes).
    keep_leaf_solution keeps every leaf's interior solution operator for postprocess();
    keep_body_operator keeps P1 A_ii^-1 per leaf for fast solve_body(); pivot_tol > 0
    rejects near-singular leaf and merge systems (HPS_ESINGULAR)."""
    coeffs = _f64(coeffs)
    dev = _dev(coeffs)
    if surrogate is not None:
        mode = HPS_SURROGATE
    bo = _build_opts(mode, _stream(coeffs) if dev else None, dev, keep_factors, root_dtn,
                     surrogate, judge_samples, judge_tol, keep_leaf_solution,
                     keep_body_operator, pivot_tol)
    h = C.c_void_p()
    check(lib.hps_build_solution_operator(_ptr(coeffs), (C.c_double * 4)(*box),
                                          (C.c_int * 2)(*nleaf), p, q, C.byref(bo), C.byref(h)))
    return Operator(h)


def build_batch(problems: Sequence[dict], mode: int = HPS_FP64, keep_factors: bool = False,
                root_dtn: bool = True, keep_leaf_solution: bool = False,
                keep_body_operator: bool = False, pivot_tol: float = 0.0) -> List[Operator]:
    """Heterogeneous batch; problems are dicts with coeffs (device), box, nleaf, p, q."""
    arr = (Problem * len(problems))()
    keep = []
    for i, pr in enumerate(problems):
        c = _f64(pr["coeffs"])
        assert _dev(c), "hps_build_batch takes device coefficient tensors"
        keep.append(c)
        arr[i].coeffs = c.data_ptr()
        arr[i].box = (C.c_double * 4)(*pr["box"])
        arr[i].nleaf = (C.c_int * 2)(*pr["nleaf"])
        arr[i].p = pr["p"]
        arr[i].q = pr["q"]
    bo = _build_opts(mode, _stream(keep[0]), 1, keep_factors, root_dtn,
                     keep_leaf_solution=keep_leaf_solution,
                     keep_body_operator=keep_body_operator, pivot_tol=pivot_tol)
    hs = (C.c_void_p * len(problems))()
    check(lib.hps_build_batch(arr, len(problems), C.byref(bo), hs))
    return [Operator(C.c_void_p(h)) for h in hs]


def solve_batch(ops: Sequence[Operator], fs, us=None):
    """Solves every problem of a batch (device tensors)."""
    import torch
    n = len(ops)
    fs = [_f64(f) for f in fs]
    if us is None:
        us = [torch.empty((f.shape[0], op.N), dtype=torch.float64, device=f.device)
              for op, f in zip(ops, fs)]
    hs = (C.c_void_p * n)(*[op.handle.value if isinstance(op.handle, C.c_void_p) else op.handle
                            for op in ops])
    fp = (C.c_void_p * n)(*[f.data_ptr() for f in fs])
    up = (C.c_void_p * n)(*[u.data_ptr() for u in us])
    nr = (C.c_int * n)(*[f.shape[0] for f in fs])
    so = SolveOpts(_stream(fs[0]), 1, 0, 0.0, 0)
    check(lib.hps_solve_batch(hs, n, fp, nr, up, C.byref(so)))
    return us
