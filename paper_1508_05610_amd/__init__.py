"""lf2 for MI355X: LATfield2's 3-D FFT, spectral Poisson solve and power
spectrum (arXiv:1508.05610) as hand-written HIP kernels behind a C ABI.

PyTorch supplies device memory and streams only; every step of a transform
runs in the library's kernels.  ``Plan`` is the torch-facing helper over the
C calls in ``_lib`` (which keep the C names).

Layouts (N0 fastest, paper section 3.4; components innermost, 3.5):
  real field     torch.float32 of shape (N2+2h, N1+2h, N0+2h[, ncomp])
  complex field  torch.complex64 of the same shape
  half spectrum  torch.complex64 of shape (N2, N1, N0//2+1[, ncomp])
  full spectrum  torch.complex64 of shape (N2, N1, N0[, ncomp])
"""
from __future__ import annotations

from . import _lib
from ._lib import (LF2_BACKWARD, LF2_BATCH_GROUPED, LF2_BATCH_ONE_QUEUE, LF2_BATCH_PK,
                   LF2_BATCH_POISSON, LF2_C2C, LF2_FORWARD,
                   LF2_PK_OF_PHI, LF2_POISSON_DISCRETE_K2, LF2_R2C, LF2Error, lf2_batch_destroy,
                   lf2_batch_error, lf2_batch_execute, lf2_batch_info, lf2_batch_plan,
                   lf2_fft_execute, lf2_fft_kspace, lf2_fft_plan, lf2_plan_destroy,
                   lf2_plan_set_workspace, lf2_plan_workspace_bytes, lf2_poisson_solve,
                   lf2_power_spectrum, lf2_version)
from ._lib import (LF2_ERR_BUDGET, LF2_ERR_BUSY, LF2_ERR_DEVICE, LF2_ERR_INVALID_ARG,  # noqa: F401
                   LF2_ERR_NOT_READY, LF2_ERR_UNSUPPORTED, LF2_OK)

__all__ = ["Plan", "Batch", "LF2Error", "LF2_R2C", "LF2_C2C", "LF2_FORWARD", "LF2_BACKWARD",
           "LF2_POISSON_DISCRETE_K2", "LF2_PK_OF_PHI", "LF2_BATCH_POISSON", "LF2_BATCH_PK", "LF2_BATCH_GROUPED",
           "LF2_BATCH_ONE_QUEUE",
           "lf2_fft_plan", "lf2_fft_execute", "lf2_fft_kspace", "lf2_poisson_solve",
           "lf2_power_spectrum", "lf2_plan_destroy", "lf2_plan_workspace_bytes",
           "lf2_plan_set_workspace", "lf2_batch_plan", "lf2_batch_execute", "lf2_batch_error",
           "lf2_batch_info", "lf2_batch_destroy", "lf2_version", "load", "Server",
           "latency_percentiles", "update_halo", "gradient"]


def load():
    """Load liblf2.so (raises ImportError if it was not built)."""
    return _lib.load()


def _stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t, what, dtype, shape):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t.data_ptr()


class Plan:
    """A PlanFFT (paper section 3.6) on an N0 x N1 x N2 lattice with halo h."""

    def __init__(self, sizes, kind=LF2_R2C, ncomp=1, halo=0, autotune=False, in_place=False,
                 paper_layout=False):
        self.sizes = tuple(int(s) for s in sizes)
        self.kind = kind
        self.ncomp = int(ncomp)
        self.halo = int(halo)
        self.in_place = bool(in_place)
        self.paper_layout = bool(paper_layout)
        flags = ((_lib.LF2_PLAN_AUTOTUNE if autotune else 0) |
                 (_lib.LF2_IN_PLACE if in_place else 0) |
                 (_lib.LF2_KLAYOUT_PAPER if paper_layout else 0))
        self.handle = lf2_fft_plan(self.sizes, self.halo, self.ncomp, kind, flags)
        self.ksize, self.kstride = lf2_fft_kspace(self.handle)

    def tuning(self, axis):
        """(variant, chunk, us_default, us_tuned): the strided pass along axis 1 or 2, the
        x pass's stage exchange (axis 0: 0 LDS, 1 ds_bpermute, 2 DPP), or the fused
        Poisson pass (axis 3: 0 LDS stages, 1 register tile)."""
        return _lib.lf2_plan_get_tuning(self.handle, axis)

    def set_tuning(self, axis, variant, chunk=16):
        _lib.lf2_plan_set_tuning(self.handle, axis, variant, chunk)

    def schedule(self, axis):
        """(radices, runtime) of the passes along axis (0 = x, 1 = y, 2 = z)."""
        return _lib.lf2_plan_get_schedule(self.handle, axis)

    def set_schedule(self, axis, radices):
        _lib.lf2_plan_set_schedule(self.handle, axis, radices)

    def close(self):
        if self.handle:
            lf2_plan_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # shapes ---------------------------------------------------------------
    def _comp(self):
        return (self.ncomp,) if self.ncomp > 1 else ()

    @property
    def x_shape(self):
        """Real-space array shape; in-place r2c rows are padded to 2 (N0/2 + 1)."""
        n0, n1, n2 = self.sizes
        h = self.halo
        if self.in_place and self.kind == LF2_R2C:
            return (n2, n1, 2 * (n0 // 2 + 1)) + self._comp()
        return (n2 + 2 * h, n1 + 2 * h, n0 + 2 * h) + self._comp()

    @property
    def k_shape(self):
        """Spectrum array shape: natural (N2, N1, Nk) or, with paper_layout,
        the paper's order: r2c (N1, N2, Nh), c2c (N1, N0, N2)."""
        if self.paper_layout and self.kind == LF2_R2C:
            return (self.ksize[1], self.ksize[2], self.ksize[0]) + self._comp()
        if self.paper_layout:
            return (self.ksize[1], self.ksize[0], self.ksize[2]) + self._comp()
        return (self.ksize[2], self.ksize[1], self.ksize[0]) + self._comp()

    # transforms -------------------------------------------------------------
    def forward(self, x, out=None, stream=None):
        import torch
        xdt = torch.float32 if self.kind == LF2_R2C else torch.complex64
        xp = _ptr(x, "x", xdt, self.x_shape)
        if out is None:
            out = torch.empty(self.k_shape, dtype=torch.complex64, device=x.device)
        op = _ptr(out, "out", torch.complex64, self.k_shape)
        lf2_fft_execute(self.handle, LF2_FORWARD, xp, op, _stream_handle(stream))
        return out

    def forward_(self, x, stream=None):
        """In-place forward (plan made with in_place=True): x is overwritten by
        its spectrum; returns the spectrum as a complex64 view of x's memory."""
        import torch
        if not self.in_place:
            raise ValueError("plan was not made with in_place=True")
        xdt = torch.float32 if self.kind == LF2_R2C else torch.complex64
        xp = _ptr(x, "x", xdt, self.x_shape)
        lf2_fft_execute(self.handle, LF2_FORWARD, xp, xp, _stream_handle(stream))
        if self.kind == LF2_R2C:  # each padded real row holds one spectrum row
            return x.reshape(x.shape[0], x.shape[1], -1).view(torch.complex64).reshape(self.k_shape)
        return x.reshape(self.k_shape)

    def backward_(self, k, stream=None):
        """In-place backward: k is overwritten by the real (or complex) field;
        returns it as a view of k's memory with x_shape."""
        import torch
        if not self.in_place:
            raise ValueError("plan was not made with in_place=True")
        kp = _ptr(k, "k", torch.complex64, self.k_shape)
        lf2_fft_execute(self.handle, LF2_BACKWARD, kp, kp, _stream_handle(stream))
        if self.kind == LF2_R2C:
            return k.reshape(k.shape[0], k.shape[1], -1).view(torch.float32).reshape(self.x_shape)
        return k.reshape(self.x_shape)

    def backward(self, k, out=None, stream=None):
        import torch
        kp = _ptr(k, "k", torch.complex64, self.k_shape)
        xdt = torch.float32 if self.kind == LF2_R2C else torch.complex64
        if out is None:
            out = torch.zeros(self.x_shape, dtype=xdt, device=k.device)
        op = _ptr(out, "out", xdt, self.x_shape)
        lf2_fft_execute(self.handle, LF2_BACKWARD, kp, op, _stream_handle(stream))
        return out

    def poisson(self, rho, phi=None, dx=1.0, flags=0, nbins=0, parseval=False, stream=None):
        """Solve laplacian(phi) = rho; returns phi or (phi, pk, kmean, count[, parseval])."""
        import torch
        rp = _ptr(rho, "rho", torch.float32, self.x_shape)
        if phi is None:
            phi = torch.zeros(self.x_shape, dtype=torch.float32, device=rho.device)
        pp = _ptr(phi, "phi", torch.float32, self.x_shape)
        dev = rho.device
        pk = kmean = count = pv = None
        if nbins > 0:
            pk = torch.empty(nbins, dtype=torch.float64, device=dev)
            kmean = torch.empty(nbins, dtype=torch.float64, device=dev)
            count = torch.empty(nbins, dtype=torch.float64, device=dev)
        if parseval:
            pv = torch.empty(2, dtype=torch.float64, device=dev)
        ptr = lambda t: t.data_ptr() if t is not None else 0  # noqa: E731
        lf2_poisson_solve(self.handle, rp, pp, dx, flags, nbins, ptr(pk), ptr(kmean), ptr(count),
                          ptr(pv), _stream_handle(stream))
        if nbins == 0 and not parseval:
            return phi
        res = (phi, pk, kmean, count)
        return res + (pv,) if parseval else res

    def power_spectrum_into(self, field, nbins, pk, kmean, count, dx=1.0, field_is_kspace=False,
                            stream=None):
        """Like power_spectrum, into caller-owned float64 device tensors."""
        import torch
        if field_is_kspace:
            fp = _ptr(field, "field", torch.complex64, self.k_shape)
        else:
            xdt = torch.float32 if self.kind == LF2_R2C else torch.complex64
            fp = _ptr(field, "field", xdt, self.x_shape)
        lf2_power_spectrum(self.handle, fp, int(bool(field_is_kspace)), nbins, dx,
                           pk.data_ptr() if pk is not None else 0,
                           kmean.data_ptr() if kmean is not None else 0,
                           count.data_ptr() if count is not None else 0, _stream_handle(stream))

    def power_spectrum(self, field, nbins, dx=1.0, field_is_kspace=False, stream=None):
        """Returns (pk, kmean, count) as float64 device tensors."""
        import torch
        if field_is_kspace:
            fp = _ptr(field, "field", torch.complex64, self.k_shape)
        else:
            xdt = torch.float32 if self.kind == LF2_R2C else torch.complex64
            fp = _ptr(field, "field", xdt, self.x_shape)
        dev = field.device
        pk = torch.empty(nbins, dtype=torch.float64, device=dev)
        kmean = torch.empty(nbins, dtype=torch.float64, device=dev)
        count = torch.empty(nbins, dtype=torch.float64, device=dev)
        lf2_power_spectrum(self.handle, fp, int(bool(field_is_kspace)), nbins, dx, pk.data_ptr(),
                           kmean.data_ptr(), count.data_ptr(), _stream_handle(stream))
        return pk, kmean, count


class Batch:
    """Batched Poisson solves (optionally with fused power spectra) on many
    lattices: one persistent launch replayed from a hipGraph, or with
    grouped=True one launch per (pass, line length) group (see lf2_batch_plan
    in include/lf2.h)."""

    def __init__(self, sizes_list, nbins=0, dx=1.0, poisson_flags=0, grouped=False,
                 one_queue=False):
        self.sizes = [tuple(int(v) for v in s) for s in sizes_list]
        self.nbins = int(nbins)
        ops = LF2_BATCH_POISSON | (LF2_BATCH_PK if nbins > 0 else 0)
        if grouped:
            ops |= LF2_BATCH_GROUPED
        if one_queue:
            ops |= LF2_BATCH_ONE_QUEUE
        self.handle = lf2_batch_plan(self.sizes, ops, nbins, dx, poisson_flags)
        self.nitems, self.launches, self.workspace_bytes = lf2_batch_info(self.handle)
        self.queues, self.per_xcd = _lib.lf2_batch_queues(self.handle)

    def close(self):
        if self.handle:
            lf2_batch_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, rhos, phis, pks=None, kmeans=None, counts=None, stream=None):
        """rhos, phis: lists of float32 device tensors (N2, N1, N0) per field;
        pks/kmeans/counts: optional lists of float64 device tensors (nbins)."""
        import torch
        n = len(self.sizes)
        assert len(rhos) == n and len(phis) == n
        for s, r, p in zip(self.sizes, rhos, phis):
            shape = (s[2], s[1], s[0])
            _ptr(r, "rho", torch.float32, shape)
            _ptr(p, "phi", torch.float32, shape)
        ptrs = lambda ts: None if ts is None else [t.data_ptr() if t is not None else 0 for t in ts]  # noqa: E731
        lf2_batch_execute(self.handle, ptrs(rhos), ptrs(phis), ptrs(pks), ptrs(kmeans),
                          ptrs(counts), _stream_handle(stream))

    def error(self) -> int:
        return lf2_batch_error(self.handle)


class Server:
    """Continuous-batching request loop for Poisson solves with power spectra
    (lf2_server_* in include/lf2.h).  Tensors of a request are held until its
    result has been polled.  Inputs must be ready on the device when submitted:
    the server's streams do not wait for torch's stream."""

    def __init__(self, budget_bytes, max_slots=16, nstreams=4, max_queue=4096, fake=False,
                 delay_us=0, fail_ticket=0):
        if fake:
            self.handle = _lib.lf2_server_create_fake(budget_bytes, max_slots, max_queue,
                                                      delay_us, fail_ticket)
        else:
            self.handle = _lib.lf2_server_create(budget_bytes, max_slots, nstreams, max_queue)
        self._held = {}

    def prepare(self, sizes_list, nbins=0, dx=1.0, flags=0):
        _lib.lf2_server_prepare(self.handle, [tuple(s) for s in sizes_list], nbins, dx, flags)

    def submit_raw(self, sizes, rho_ptr, phi_ptr, dx=1.0, flags=0, nbins=0, pk_ptr=0,
                   kmean_ptr=0, count_ptr=0, t_arrival=0.0, hold=None):
        """(status, ticket); status LF2_ERR_BUSY / LF2_ERR_BUDGET are rejections."""
        req = _lib.make_request(sizes, rho_ptr, phi_ptr, dx, flags, nbins, pk_ptr, kmean_ptr,
                                count_ptr, t_arrival)
        st, ticket = _lib.lf2_server_submit_status(self.handle, req)
        if st == LF2_OK and hold is not None:
            self._held[ticket] = hold
        return st, ticket

    def submit(self, rho, phi, dx=1.0, flags=0, nbins=0, pk=None, kmean=None, count=None,
               t_arrival=0.0):
        import torch
        n2, n1, n0 = rho.shape
        _ptr(rho, "rho", torch.float32, (n2, n1, n0))
        _ptr(phi, "phi", torch.float32, (n2, n1, n0))
        bins = []
        for t, nm in ((pk, "pk"), (kmean, "kmean"), (count, "count")):
            bins.append(0 if t is None else _ptr(t, nm, torch.float64, (nbins,)))
        return self.submit_raw((n0, n1, n2), rho.data_ptr(), phi.data_ptr(), dx, flags, nbins,
                               *bins, t_arrival=t_arrival, hold=(rho, phi, pk, kmean, count))

    def poll(self, ticket, wait=True):
        """None while running (wait=False), else (status, t_arrival, t_admit, t_done)."""
        r = _lib.lf2_server_poll(self.handle, ticket, wait)
        if r is not None:
            self._held.pop(ticket, None)
        return r

    def footprint(self, sizes, nbins=0) -> int:
        return _lib.lf2_server_footprint(_lib.make_request(sizes, 0, 0, 1.0, 0, nbins))

    def stats(self) -> dict:
        return _lib.lf2_server_get_stats(self.handle)

    def close(self):
        if self.handle:
            _lib.lf2_server_destroy(self.handle)
            self.handle = 0
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def latency_percentiles(values, qs=(50, 99)):
    """Nearest-rank percentiles: the q-th is the ceil(q n / 100)-th smallest
    value (1-based), so it is always one of the observed latencies."""
    import math
    v = sorted(float(x) for x in values)
    if not v:
        raise ValueError("no latencies")
    out = []
    for q in qs:
        if not 0 < q <= 100:
            raise ValueError("percentile must be in (0, 100]")
        out.append(v[max(1, math.ceil(q * len(v) / 100.0)) - 1])
    return tuple(out)


def update_halo(field, sizes, halo, stream=None):
    """Periodic halo update of a (N2+2h, N1+2h, N0+2h[, ncomp]) float32 or
    complex64 tensor in place (lf2_update_halo)."""
    import torch
    n0, n1, n2 = (int(v) for v in sizes)
    h = int(halo)
    if not isinstance(field, torch.Tensor) or not field.is_cuda or not field.is_contiguous():
        raise TypeError("field must be a contiguous CUDA (HIP) tensor")
    if tuple(field.shape[:3]) != (n2 + 2 * h, n1 + 2 * h, n0 + 2 * h):
        raise ValueError("field shape does not match the lattice")
    if field.dtype not in (torch.float32, torch.complex64):
        raise TypeError("field must be float32 or complex64")
    ncomp = int(field[0, 0, 0].numel())
    eb = 4 if field.dtype == torch.float32 else 8
    _lib.lf2_update_halo((n0, n1, n2), h, ncomp, eb, field.data_ptr(), _stream_handle(stream))
    return field


def gradient(field, sizes, halo, dx=1.0, out=None, stream=None):
    """First-order forward derivative of every component (lf2_gradient): a
    (N2+2h, N1+2h, N0+2h, 3 ncomp) float32 tensor whose interior is written."""
    import torch
    n0, n1, n2 = (int(v) for v in sizes)
    h = int(halo)
    if field.dtype != torch.float32 or not field.is_cuda or not field.is_contiguous():
        raise TypeError("field must be a contiguous float32 CUDA (HIP) tensor")
    if tuple(field.shape[:3]) != (n2 + 2 * h, n1 + 2 * h, n0 + 2 * h):
        raise ValueError("field shape does not match the lattice")
    ncomp = int(field[0, 0, 0].numel())
    shape = (n2 + 2 * h, n1 + 2 * h, n0 + 2 * h, 3 * ncomp)
    if out is None:
        out = torch.zeros(shape, dtype=torch.float32, device=field.device)
    _ptr(out, "out", torch.float32, shape)
    _lib.lf2_gradient((n0, n1, n2), h, ncomp, field.data_ptr(), out.data_ptr(), dx,
                      _stream_handle(stream))
    return out
