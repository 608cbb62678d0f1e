"""cqc: cut-circuit reconstruction on AMD MI355X.

Thin Python binding of libcqc.so (include/cqc.h).  PyTorch provides device
memory and the current stream; every step of the reconstruction runs in the
library's HIP kernels.  There is no CPU fallback: if the library or a GPU is
missing, calls raise.

    cut = CutMap(n, f, edges=[(up, down), ...], out_qubits=[...])
    p, mass = reconstruct_fd(entries, cut, precision="fp32")
    bins, records = reconstruct_dd(entries, cut, n_active, n_recursions)
    p = ReconstructFD.apply(cut, "fp32", *entries)      # differentiable
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import CqcError, PREC

__all__ = ["CutMap", "reconstruct_fd", "reconstruct_dd", "reconstruct_backward", "FDCall", "Batch", "BatchBackward", "build_entries", "chi2", "xent_grad", "shard",
           "ReconstructFD", "BackwardCall", "cost", "autotune", "tune_reset", "trace", "CqcError", "selftest_mfma", "library_path"]

_DT = {torch.float32: _lib.F32, torch.float64: _lib.F64}


def library_path():
    return _lib.LIB_PATH


class CutMap:
    """Cut description: n output qubits, f[c] output qubits per subcircuit,
    edges[e] = (upstream, downstream) subcircuit of cut e, out_qubits =
    concatenated local-bit -> global-qubit map (local bit 0 most significant)."""

    def __init__(self, n, f, edges, out_qubits):
        self.n = int(n)
        self.f = [int(v) for v in f]
        self.edges = [(int(u), int(d)) for (u, d) in edges]
        self.out_qubits = [int(q) for q in out_qubits]
        I32 = ctypes.c_int32
        self._f = (I32 * max(1, len(self.f)))(*self.f)
        self._up = (I32 * max(1, len(self.edges)))(*[u for u, _ in self.edges])
        self._down = (I32 * max(1, len(self.edges)))(*[d for _, d in self.edges])
        self._oq = (I32 * max(1, len(self.out_qubits)))(*self.out_qubits)
        self.c = _lib.CqcCut(self.n, len(self.f), len(self.edges), self._f, self._up, self._down, self._oq)

    @classmethod
    def from_workload(cls, cm):
        """From a workloads.CutMap (f, edge_up, edge_down, out_qubit)."""
        return cls(cm.n, cm.f, list(zip(cm.edge_up, cm.edge_down)), cm.out_qubit)

    @property
    def n_sub(self):
        return len(self.f)

    @property
    def n_cuts(self):
        return len(self.edges)

    def k(self, c):
        return sum(1 for (u, d) in self.edges if u == c or d == c)

    def entry_shape(self, c):
        return (4 ** self.k(c), 2 ** self.f[c])


def _stream_ptr(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_entries(entries, cut, dtype=None):
    if len(entries) != cut.n_sub:
        raise ValueError(f"expected {cut.n_sub} entry tensors, got {len(entries)}")
    dt = dtype or entries[0].dtype
    for c, E in enumerate(entries):
        if not E.is_cuda:
            raise ValueError("entry tensors must be on the GPU")
        if E.dtype != dt:
            raise ValueError("all entry tensors must share one dtype")
        if tuple(E.shape) != cut.entry_shape(c) or not E.is_contiguous():
            raise ValueError(f"entries[{c}] must be contiguous with shape {cut.entry_shape(c)}")
    if dt not in _DT:
        raise ValueError("entries must be float32 or float64")
    return dt


def _workspace(nbytes, device):
    """A fresh workspace for one enqueued call.  Torch's caching allocator
    orders its reuse on the current stream, which is the stream the call runs
    on, so concurrent calls on different streams never share one."""
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class FDCall:
    """A prepared FD reconstruction: validated shapes, workspace and output
    buffers allocated once; run() enqueues the whole hot path on the current
    stream with one library call."""

    def __init__(self, entries_list, cuts, precision="fp32", out_dtype=None, outs=None,
                 with_mass=True, workspace=None, noalloc=False):
        if isinstance(cuts, CutMap):
            cuts, entries_list = [cuts], [entries_list]
        self.cuts = list(cuts)
        self.entries_list = [list(e) for e in entries_list]
        in_dt = _check_entries(self.entries_list[0], self.cuts[0])
        for e, c in zip(self.entries_list, self.cuts):
            _check_entries(e, c, in_dt)
        self.in_dtype = in_dt
        self.out_dtype = out_dtype or in_dt
        self.prec = PREC[precision]
        dev = self.entries_list[0][0].device
        self.device = dev
        n_inst = len(self.cuts)
        self.outs = list(outs) if outs is not None else [
            torch.empty(2 ** c.n, dtype=self.out_dtype, device=dev) for c in self.cuts]
        self.mass = torch.zeros(n_inst, dtype=torch.float64, device=dev) if with_mass else None
        Arr = _lib.CqcInstance * n_inst
        self._insts = Arr()
        self._keep = []
        for i, (c, ents) in enumerate(zip(self.cuts, self.entries_list)):
            ptrs = (ctypes.c_void_p * len(ents))(*[E.data_ptr() for E in ents])
            self._keep.append(ptrs)
            self._insts[i] = _lib.CqcInstance(
                c.c, ptrs, self.outs[i].data_ptr() if self.outs[i] is not None else None,
                (self.mass.data_ptr() + 8 * i) if with_mass else None)
        self.n_inst = n_inst
        self._in_t, self._out_t = _DT[self.in_dtype], _DT[self.out_dtype]
        nb = ctypes.c_size_t(0)
        _lib.check(_lib.lib().cqc_fd_workspace_size(self._insts, n_inst, self._in_t, self._out_t,
                                                    self.prec, ctypes.byref(nb)))
        self.ws_bytes = int(nb.value)
        self.noalloc = bool(noalloc)
        if self.noalloc:
            # run() uses the library's fixed workspace array (cqc_reconstruct_fd_noalloc)
            if self.ws_bytes > _lib.NOALLOC_WORKSPACE_BYTES:
                raise ValueError(f"needs {self.ws_bytes} bytes of workspace; the static workspace "
                                 f"holds {_lib.NOALLOC_WORKSPACE_BYTES}")
            self.ws = None
        else:
            self.ws = workspace if workspace is not None else torch.empty(
                max(self.ws_bytes, 256), dtype=torch.uint8, device=dev)
        self._fn = _lib.lib().cqc_reconstruct_fd

    def set_outputs(self, outs):
        for i, o in enumerate(outs):
            self.outs[i] = o
            self._insts[i].out = o.data_ptr()

    def run(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        if self.noalloc:
            _lib.check(_lib.lib().cqc_reconstruct_fd_noalloc(self._insts, self.n_inst, self._in_t,
                                                             self._out_t, self.prec, s))
            return
        _lib.check(self._fn(self._insts, self.n_inst, self._in_t, self._out_t, self.prec,
                            self.ws.data_ptr(), self.ws_bytes, s))


class Batch(FDCall):
    """A prepared batch of instances (cqc_batch_create): the descriptor tables
    are uploaded once; run() enqueues a fixed handful of kernel launches and is
    safe to capture into a CUDA/HIP graph.  Outputs and masses are bound at
    construction.

    With targets (one per instance, the output dtype and size) the batch is
    the cross-entropy form (cqc_batch_create_xent): every run also writes
    dL/dp = -t/p (0 where p <= 1e-30) into self.grads (the given grads, else
    new tensors) from inside the kernels that compute p, and, with with_loss,
    L_i = -sum t log max(p, 1e-30) into self.losses[i] (FP64) in place of the
    mass.  keep_outputs=False writes no p at all (self.outs[i] is None)."""

    def __init__(self, entries_list, cuts, precision="fp32", outs=None, with_mass=True, targets=None,
                 grads=None, with_loss=False, keep_outputs=True):
        if targets is None and (grads is not None or with_loss or not keep_outputs):
            raise ValueError("grads, with_loss and keep_outputs=False need targets")
        if targets is not None:
            if with_loss:
                with_mass = False
            if not keep_outputs:
                if outs is not None:
                    raise ValueError("keep_outputs=False takes no outs")
                outs = [None] * len(cuts)
        super().__init__(entries_list, cuts, precision, None, outs, with_mass)
        if self.n_inst < 2:
            raise ValueError("a batch needs at least two instances")
        h = ctypes.c_void_p(0)
        s = torch.cuda.current_stream(self.device).cuda_stream
        self.targets = self.grads = self.losses = None
        if targets is None:
            _lib.check(_lib.lib().cqc_batch_create(self._insts, self.n_inst, self._in_t, self._out_t, self.prec,
                                                   self.ws.data_ptr(), self.ws_bytes, s, ctypes.byref(h)))
        else:
            targets = list(targets)
            if len(targets) != self.n_inst:
                raise ValueError("one target per instance")
            if grads is None:
                grads = [torch.empty(2 ** c.n, dtype=self.out_dtype, device=self.device) for c in self.cuts]
            grads = list(grads)
            if len(grads) != self.n_inst:
                raise ValueError("one gradient buffer per instance")
            for c, t, g in zip(self.cuts, targets, grads):
                for x, what in ((t, "target"), (g, "gradient")):
                    if (x.shape != (2 ** c.n,) or x.dtype != self.out_dtype or x.device != self.device
                            or not x.is_contiguous()):
                        raise ValueError(f"each {what} must be a contiguous [2^n] tensor of the output "
                                         "dtype on the batch's device")
            self.targets, self.grads = targets, grads
            self.losses = torch.zeros(self.n_inst, dtype=torch.float64, device=self.device) if with_loss else None
            n = self.n_inst
            self._tp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in targets])
            self._gp = (ctypes.c_void_p * n)(*[g.data_ptr() for g in grads])
            self._lp = (ctypes.c_void_p * n)(*[self.losses.data_ptr() + 8 * i for i in range(n)]) \
                if with_loss else None
            _lib.check(_lib.lib().cqc_batch_create_xent(self._insts, n, self._in_t, self._out_t, self.prec,
                                                        self._tp, self._gp, self._lp, self.ws.data_ptr(),
                                                        self.ws_bytes, s, ctypes.byref(h)))
        self._h = h

    def set_outputs(self, outs):
        raise RuntimeError("outputs of a prepared batch are fixed; create a new Batch")

    def run(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(_lib.lib().cqc_batch_run(self._h, s))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.lib().cqc_batch_destroy(h)
            self._h = None


class BatchBackward:
    """Adjoint of a prepared Batch (cqc_batch_backward_create): dL/dE for every
    instance from dL/dp, using the forward tensors the batch's last run left
    in its workspace.  grads_out[i] (dL/dp, the batch's output dtype) and the
    entry gradients are bound at construction; run() enqueues a fixed handful
    of kernel launches (graph-capturable) and must follow batch.run() on the
    same stream."""

    def __init__(self, batch, grads_out):
        if len(grads_out) != batch.n_inst:
            raise ValueError("one dL/dp per instance")
        for g, c in zip(grads_out, batch.cuts):
            if (g.shape != (2 ** c.n,) or g.dtype != batch.out_dtype or g.device != batch.device
                    or not g.is_contiguous()):
                raise ValueError("each dL/dp must match its instance's output (shape, dtype, device, contiguous)")
        self.batch = batch
        self.grads_out = list(grads_out)
        self.grads = [[torch.empty_like(E) for E in e] for e in batch.entries_list]
        n = batch.n_inst
        self._gout = (ctypes.c_void_p * n)(*[g.data_ptr() for g in self.grads_out])
        rows = []
        for gl in self.grads:
            r = (ctypes.c_void_p * len(gl))(*[g.data_ptr() for g in gl])
            rows.append(r)
        self._rows = rows
        self._gents = (ctypes.POINTER(ctypes.c_void_p) * n)(
            *[ctypes.cast(r, ctypes.POINTER(ctypes.c_void_p)) for r in rows])
        nb = ctypes.c_size_t(0)
        _lib.check(_lib.lib().cqc_batch_backward_workspace_size(batch._h, ctypes.byref(nb)))
        self.ws_bytes = int(nb.value)
        self.ws = torch.zeros(max(self.ws_bytes, 256), dtype=torch.uint8, device=batch.device)
        h = ctypes.c_void_p(0)
        s = torch.cuda.current_stream(batch.device).cuda_stream
        _lib.check(_lib.lib().cqc_batch_backward_create(batch._h, self._gout, self._gents, self.ws.data_ptr(),
                                                        self.ws_bytes, s, ctypes.byref(h)))
        self._h = h

    def run(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream(self.batch.device).cuda_stream
        _lib.check(_lib.lib().cqc_batch_backward_run(self._h, s))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.lib().cqc_batch_backward_destroy(h)
            self._h = None


def build_entries(jobs, out_dtype=None, outs=None, form="pauli"):
    """Entry tensors from stacked variant distributions, on the device
    (cqc_build_entries).  jobs: list of (variants, cut_kind) with variants a
    contiguous device tensor [4^k_in][3^k_out][2^f][2^k_out] and cut_kind the
    incident cuts in ascending cut id (0 incoming, 1 outgoing); form "pauli"
    (Eq. 1, labels I X Y Z) or "eigen" (Eq. 2, labels A1..A4).  Returns one
    [4^k][2^f] tensor per job (the given outs, if any, are filled instead),
    enqueued on the current stream."""
    jobs = list(jobs)
    if not jobs:
        raise ValueError("no jobs")
    forms = {"pauli": 0, "eigen": 1}
    if form not in forms:
        raise ValueError("form must be 'pauli' or 'eigen'")
    in_dt = jobs[0][0].dtype
    out_dt = out_dtype or in_dt
    if in_dt not in _DT or out_dt not in _DT:
        raise ValueError("variants and entries must be float32 or float64")
    arr = (_lib.CqcEntryJob * len(jobs))()
    result, keep = [], []
    for j, (V, kinds) in enumerate(jobs):
        kinds = [int(k) for k in kinds]
        k_in, k_out = kinds.count(0), kinds.count(1)
        if V.dtype != in_dt or not V.is_cuda or not V.is_contiguous() or V.dim() != 4:
            raise ValueError("variants must be contiguous 4-d device tensors of one dtype")
        if V.shape[0] != 4 ** k_in or V.shape[1] != 3 ** k_out or V.shape[3] != 2 ** k_out:
            raise ValueError(f"variants shape {tuple(V.shape)} does not match cut_kind {kinds}")
        nf = V.shape[2]
        f = nf.bit_length() - 1
        if nf != 1 << f:
            raise ValueError("the output axis must have 2^f entries")
        if outs is not None:
            E = outs[j]
            if E.shape != (4 ** len(kinds), nf) or E.dtype != out_dt or not E.is_contiguous():
                raise ValueError("outs must match the entry shapes and dtype")
        else:
            E = torch.empty((4 ** len(kinds), nf), dtype=out_dt, device=V.device)
        ck = (ctypes.c_int32 * max(1, len(kinds)))(*kinds)
        keep.append(ck)
        arr[j] = _lib.CqcEntryJob(f, len(kinds), ck, V.data_ptr(), E.data_ptr(), forms[form])
        result.append(E)
    s = torch.cuda.current_stream(jobs[0][0].device).cuda_stream
    _lib.check(_lib.lib().cqc_build_entries(arr, len(jobs), _DT[in_dt], _DT[out_dt], s))
    return result


def chi2(a, b):
    """Eq. 16 chi-square distance of two device vectors (cqc_chi2) -> 0-d FP64
    device tensor, enqueued on the current stream."""
    if a.shape != b.shape or a.dim() != 1 or not a.is_cuda or not b.is_cuda:
        raise ValueError("a and b must be 1-d device tensors of one length")
    if a.dtype not in _DT or b.dtype not in _DT or not a.is_contiguous() or not b.is_contiguous():
        raise ValueError("a and b must be contiguous float32 or float64")
    out = torch.empty((), dtype=torch.float64, device=a.device)
    ws = _workspace(8192, a.device)
    s = torch.cuda.current_stream(a.device).cuda_stream
    _lib.check(_lib.lib().cqc_chi2(a.data_ptr(), _DT[a.dtype], b.data_ptr(), _DT[b.dtype], a.numel(),
                                    out.data_ptr(), ws.data_ptr(), ws.numel(), s))
    return out


def shard(entries, cut, n_shards, index):
    """One GPU's share of an FD reconstruction over n_shards GPUs: the outputs
    whose top log2(n_shards) global bits equal `index`.  Those bits must be the
    leading local bits of one subcircuit (its columns are then sliced); the
    shard is an ordinary instance -> (entries', cut') whose 2^(n-b) outputs
    are p[index * 2^(n-b) : (index + 1) * 2^(n-b)] of the full reconstruction.
    Host-side slicing only; every GPU runs the same kernels on its shard."""
    b = int(n_shards).bit_length() - 1
    if n_shards < 1 or (1 << b) != n_shards or not 0 <= index < n_shards:
        raise ValueError("n_shards must be a power of two and 0 <= index < n_shards")
    if b == 0:
        return list(entries), cut
    off, owner = 0, None
    for c, fc in enumerate(cut.f):
        local = cut.out_qubits[off:off + fc]
        if local[:b] == list(range(b)) and fc >= b:
            owner = (c, off)
        off += fc
    if owner is None:
        raise ValueError("the top output bits are not the leading local bits of one subcircuit")
    c, off = owner
    fc = cut.f[c]
    w = 1 << (fc - b)
    new_entries = list(entries)
    new_entries[c] = entries[c][:, index * w:(index + 1) * w].contiguous()
    f = list(cut.f)
    f[c] = fc - b
    oq = [q - b for q in cut.out_qubits[:off]] + [q - b for q in cut.out_qubits[off + b:]]
    return new_entries, CutMap(cut.n - b, f, cut.edges, oq)


def xent_grad(p, t, grad=None, with_loss=False):
    """Cross-entropy gradient dL/dp = -t/p where p > 1e-30, else 0, in one pass
    (cqc_xent_grad), enqueued on the current stream -> grad (or (grad, loss)
    with with_loss: loss = -sum t log max(p, 1e-30) as a 0-d FP64 tensor).
    p, t, grad: contiguous 1-d device tensors of one float dtype; a flat buffer
    of many instances' outputs is one call."""
    if p.shape != t.shape or p.dim() != 1 or not p.is_cuda or not t.is_cuda or p.dtype != t.dtype:
        raise ValueError("p and t must be 1-d device tensors of one shape and dtype")
    if p.dtype not in _DT or not p.is_contiguous() or not t.is_contiguous():
        raise ValueError("p and t must be contiguous float32 or float64")
    if grad is None:
        grad = torch.empty_like(p)
    elif grad.shape != p.shape or grad.dtype != p.dtype or not grad.is_contiguous() or not grad.is_cuda:
        raise ValueError("grad must be a contiguous device tensor like p")
    loss = torch.empty((), dtype=torch.float64, device=p.device) if with_loss else None
    ws = _workspace(8192, p.device) if with_loss else None
    s = torch.cuda.current_stream(p.device).cuda_stream
    _lib.check(_lib.lib().cqc_xent_grad(p.data_ptr(), t.data_ptr(), _DT[p.dtype], p.numel(), grad.data_ptr(),
                                         loss.data_ptr() if with_loss else None,
                                         ws.data_ptr() if with_loss else None, ws.numel() if with_loss else 0, s))
    return (grad, loss) if with_loss else grad


def reconstruct_fd(entries, cut, precision="fp32", out_dtype=None, with_mass=True):
    """Full-definition reconstruction of one instance -> (p[2^n], mass or None)."""
    call = FDCall(entries, cut, precision, out_dtype, with_mass=with_mass)
    call.run()
    return call.outs[0], (call.mass[0] if with_mass else None)


DD_STRATEGIES = {"heaviest": 0, "dfs": 1, "bfs": 2}


def reconstruct_dd(entries, cut, n_active, n_recursions, first_active=None, precision="fp32",
                   strategy="heaviest", bins_per_round=1, bins_dtype=torch.float64):
    """Dynamic definition (Algorithm 1) -> (bins [R_done, 2^a], records list).

    strategy: "heaviest" (Algorithm 1), "dfs" or "bfs" (Section 4.3);
    bins_per_round: bins expanded per host round trip; bins_dtype: float64, or
    float32 for half the memory (masses and the selection stay FP64)."""
    if strategy not in DD_STRATEGIES:
        raise ValueError(f"unknown strategy {strategy!r}")
    if bins_dtype not in (torch.float64, torch.float32):
        raise ValueError("bins_dtype must be float64 or float32")
    in_dt = _check_entries(entries, cut)
    dev = entries[0].device
    ptrs = (ctypes.c_void_p * len(entries))(*[E.data_ptr() for E in entries])
    inst = _lib.CqcInstance(cut.c, ptrs, None, None)
    fa = None
    if first_active is not None:
        fa = (ctypes.c_int32 * len(first_active))(*[int(q) for q in first_active])
    params = _lib.CqcDDParams(int(n_active), int(n_recursions), fa, DD_STRATEGIES[strategy], int(bins_per_round),
                              1 if bins_dtype == torch.float32 else 0)
    L = _lib.lib()
    nb = ctypes.c_size_t(0)
    _lib.check(L.cqc_dd_workspace_size(ctypes.byref(inst), _DT[in_dt], PREC[precision],
                                       ctypes.byref(params), ctypes.byref(nb)))
    ws = _workspace(int(nb.value), dev)
    a = min(int(n_active), cut.n)
    bins = torch.empty((int(n_recursions), 2 ** a), dtype=bins_dtype, device=dev)   # rows past n_done unused
    recs = (_lib.CqcDDRecord * int(n_recursions))()
    done = ctypes.c_int32(0)
    _lib.check(L.cqc_reconstruct_dd(ctypes.byref(inst), _DT[in_dt], PREC[precision],
                                    ctypes.byref(params), bins.data_ptr(), recs,
                                    ctypes.byref(done), ws.data_ptr(), int(nb.value),
                                    _stream_ptr(dev)))
    return bins[:done.value], _decode_records(recs, done.value, cut.n)


def _decode_records(recs, n, n_cut_qubits):
    out = []
    for r in range(n):
        rec = recs[r]
        role = [int(rec.role[q]) for q in range(n_cut_qubits)]
        parent = (int(rec.parent_rec), int(rec.parent_bin))
        out.append(dict(parent=parent, n_active=int(rec.n_active), mass=float(rec.mass), role=role,
                        active=[q for q in range(n_cut_qubits) if role[q] == -2],
                        depth=0 if parent[0] < 0 else out[parent[0]]["depth"] + 1))
    return out


class DDQuery:
    """A prepared device-resident dynamic-definition query
    (cqc_dd_query_create): the bins, records and recursion count live in
    device memory and run() enqueues the whole search with no host round
    trip, so it can be captured in a CUDA/HIP graph.  Same search and results
    as reconstruct_dd with one bin per round.  result() reads the records
    back (one copy) -> (bins [R_done, 2^a], records list)."""

    def __init__(self, entries, cut, n_active, n_recursions, first_active=None, precision="fp32",
                 strategy="heaviest", bins_dtype=torch.float64):
        if strategy not in DD_STRATEGIES:
            raise ValueError(f"unknown strategy {strategy!r}")
        if bins_dtype not in (torch.float64, torch.float32):
            raise ValueError("bins_dtype must be float64 or float32")
        in_dt = _check_entries(entries, cut)
        dev = entries[0].device
        self.entries, self.cut, self.device = list(entries), cut, dev
        self._ptrs = (ctypes.c_void_p * len(entries))(*[E.data_ptr() for E in entries])
        self._inst = _lib.CqcInstance(cut.c, self._ptrs, None, None)
        self._fa = None
        if first_active is not None:
            self._fa = (ctypes.c_int32 * len(first_active))(*[int(q) for q in first_active])
        self._params = _lib.CqcDDParams(int(n_active), int(n_recursions), self._fa, DD_STRATEGIES[strategy], 1,
                                        1 if bins_dtype == torch.float32 else 0)
        L = _lib.lib()
        nb = ctypes.c_size_t(0)
        _lib.check(L.cqc_dd_query_workspace_size(ctypes.byref(self._inst), _DT[in_dt], PREC[precision],
                                                 ctypes.byref(self._params), ctypes.byref(nb)))
        self.ws = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=dev)
        a = min(int(n_active), cut.n)
        self.R = int(n_recursions)
        self.bins = torch.empty((self.R, 2 ** a), dtype=bins_dtype, device=dev)
        self.records = torch.zeros(self.R * ctypes.sizeof(_lib.CqcDDRecord), dtype=torch.uint8, device=dev)
        self.n_done = torch.zeros(1, dtype=torch.int32, device=dev)
        h = ctypes.c_void_p(0)
        _lib.check(L.cqc_dd_query_create(ctypes.byref(self._inst), _DT[in_dt], PREC[precision],
                                         ctypes.byref(self._params), self.bins.data_ptr(), self.records.data_ptr(),
                                         self.n_done.data_ptr(), self.ws.data_ptr(), self.ws.numel(),
                                         _stream_ptr(dev), ctypes.byref(h)))
        self._h = h

    def run(self, stream=None):
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(_lib.lib().cqc_dd_query_run(self._h, s))

    def run_range(self, first, count, stream=None):
        """Recursions [first, first + count): first = 0 starts a search, a
        later first resumes the one this query holds."""
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _lib.check(_lib.lib().cqc_dd_query_run_range(self._h, int(first), int(count), s))

    def result(self):
        done = int(self.n_done.cpu()[0])
        raw = self.records.cpu().numpy().tobytes()
        recs = (_lib.CqcDDRecord * self.R).from_buffer_copy(raw)
        return self.bins[:done], _decode_records(recs, done, self.cut.n)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _lib.lib().cqc_dd_query_destroy(h)
            self._h = None


def reconstruct_backward(entries, cut, grad_out, precision="fp32"):
    """dL/dE_c for every subcircuit given dL/dp (same dtype as the entries)."""
    in_dt = _check_entries(entries, cut)
    dev = entries[0].device
    if grad_out.dtype != in_dt or not grad_out.is_contiguous() or grad_out.numel() != 2 ** cut.n:
        raise ValueError("grad_out must be a contiguous [2^n] tensor of the entry dtype")
    grads = [torch.empty_like(E) for E in entries]
    ptrs = (ctypes.c_void_p * len(entries))(*[E.data_ptr() for E in entries])
    inst = _lib.CqcInstance(cut.c, ptrs, None, None)
    gptr = (ctypes.c_void_p * 1)(grad_out.data_ptr())
    gents = (ctypes.c_void_p * len(grads))(*[g.data_ptr() for g in grads])
    gents_pp = (ctypes.POINTER(ctypes.c_void_p) * 1)(gents)
    L = _lib.lib()
    nb = ctypes.c_size_t(0)
    _lib.check(L.cqc_backward_workspace_size(ctypes.byref(inst), 1, _DT[in_dt], PREC[precision],
                                             ctypes.byref(nb)))
    ws = _workspace(int(nb.value), dev)
    _lib.check(L.cqc_reconstruct_backward(ctypes.byref(inst), 1, _DT[in_dt], PREC[precision],
                                          gptr, gents_pp, ws.data_ptr(), int(nb.value),
                                          _stream_ptr(dev)))
    return grads


class BackwardCall:
    """A prepared adjoint call over many instances: dL/dE_c of every instance
    for the given dL/dp buffers.  Workspace and gradient buffers are allocated
    once; run() enqueues kernels only (graph-capturable)."""

    def __init__(self, entries_list, cuts, grad_outs, precision="fp32"):
        if isinstance(cuts, CutMap):
            cuts, entries_list, grad_outs = [cuts], [entries_list], [grad_outs]
        self.cuts = list(cuts)
        self.entries_list = [list(e) for e in entries_list]
        in_dt = _check_entries(self.entries_list[0], self.cuts[0])
        for e, c, g in zip(self.entries_list, self.cuts, grad_outs):
            _check_entries(e, c, in_dt)
            if g.dtype != in_dt or not g.is_contiguous() or g.numel() != 2 ** c.n:
                raise ValueError("grad_out must be a contiguous [2^n] tensor of the entry dtype")
        self.grad_outs = list(grad_outs)
        self.prec = PREC[precision]
        self.in_t = _DT[in_dt]
        dev = self.entries_list[0][0].device
        self.device = dev
        n = len(self.cuts)
        self.grads = [[torch.empty_like(E) for E in e] for e in self.entries_list]
        self._insts = (_lib.CqcInstance * n)()
        self._keep = []
        for i, (c, ents) in enumerate(zip(self.cuts, self.entries_list)):
            ptrs = (ctypes.c_void_p * len(ents))(*[E.data_ptr() for E in ents])
            self._keep.append(ptrs)
            self._insts[i] = _lib.CqcInstance(c.c, ptrs, None, None)
        self._gout = (ctypes.c_void_p * n)(*[g.data_ptr() for g in self.grad_outs])
        rows = []
        for gl in self.grads:
            r = (ctypes.c_void_p * len(gl))(*[g.data_ptr() for g in gl])
            self._keep.append(r)
            rows.append(ctypes.cast(r, ctypes.POINTER(ctypes.c_void_p)))
        self._gents = (ctypes.POINTER(ctypes.c_void_p) * n)(*rows)
        nb = ctypes.c_size_t(0)
        _lib.check(_lib.lib().cqc_backward_workspace_size(self._insts, n, self.in_t, self.prec,
                                                           ctypes.byref(nb)))
        self.ws_bytes = int(nb.value)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=dev)   # owned

    def run(self):
        _lib.check(_lib.lib().cqc_reconstruct_backward(self._insts, len(self.cuts), self.in_t, self.prec,
                                                        self._gout, self._gents, self.ws.data_ptr(),
                                                        self.ws_bytes, _stream_ptr(self.device)))
        return self.grads


class ReconstructFD(torch.autograd.Function):
    """p = FD(entries); backward runs the library's adjoint kernels.  The
    adjoint has no split-BF16 form: a BF16X6 or BF16X3 forward is differentiated
    in FP32."""

    @staticmethod
    def forward(ctx, cut, precision, *entries):
        p, _ = reconstruct_fd(list(entries), cut, precision, with_mass=False)
        ctx.cut, ctx.precision = cut, precision
        ctx.save_for_backward(*entries)
        return p

    @staticmethod
    def backward(ctx, grad_p):
        entries = ctx.saved_tensors
        g = grad_p.contiguous().to(entries[0].dtype)
        prec = "fp32" if ctx.precision in ("bf16x6", "bf16x3") else ctx.precision
        grads = reconstruct_backward(list(entries), ctx.cut, g, prec)
        return (None, None) + tuple(grads)


def autotune(call):
    """Time every tile shape / XCD mapping for the steps of a prepared FDCall
    (outputs are clobbered) and keep the fastest for their shape classes."""
    s = torch.cuda.current_stream(call.device).cuda_stream
    _lib.check(_lib.lib().cqc_autotune(call._insts, call.n_inst, call._in_t, call._out_t, call.prec,
                                       call.ws.data_ptr(), call.ws_bytes, s))


def tune_reset():
    """Clear the process-wide tile cache (cqc_tune_reset); the next plan reloads
    the file named by CQC_TUNE_CACHE, if set."""
    _lib.check(_lib.lib().cqc_tune_reset())


def cost(cut):
    """(Eq. 14 multiplications with greedy order, multiply-adds of the library's plan)."""
    a, b = ctypes.c_double(0), ctypes.c_double(0)
    _lib.check(_lib.lib().cqc_cost(ctypes.byref(cut.c), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


class trace:
    """Context manager: per-kernel event timing of every library launch."""

    def __enter__(self):
        _lib.lib().cqc_trace_enable(1)
        return self

    def __exit__(self, *exc):
        _lib.lib().cqc_trace_enable(0)
        self.result = read_trace()
        return False


def read_trace(max_kernels=64):
    L = _lib.lib()
    names = ctypes.create_string_buffer(8192)
    counts = (ctypes.c_int32 * max_kernels)()
    ms = (ctypes.c_double * max_kernels)()
    nk = ctypes.c_int32(0)
    _lib.check(L.cqc_trace_read(names, 8192, counts, ms, max_kernels, ctypes.byref(nk)))
    nl = names.value.decode().split("\n") if nk.value else []
    return {nl[i]: (int(counts[i]), float(ms[i])) for i in range(nk.value)}


def selftest_mfma(device="cuda"):
    """Run the MFMA lane-layout probe -> (D_f32[16,16], D_f64[16,16], D_bf16[16,16])."""
    buf = torch.zeros(256 * 4 + 256 * 8 + 256 * 4, dtype=torch.uint8, device=device)
    _lib.check(_lib.lib().cqc_selftest_mfma(buf.data_ptr(), _stream_ptr()))
    torch.cuda.synchronize()
    f = buf[:1024].view(torch.float32).reshape(16, 16).cpu()
    d = buf[1024:3072].view(torch.float64).reshape(16, 16).cpu()
    b = buf[3072:].view(torch.float32).reshape(16, 16).cpu()
    return f, d, b
