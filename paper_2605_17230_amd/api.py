"""PyTorch-facing calls of the C ABI.  Torch provides device memory and the
stream; all arithmetic runs in libtnmld.so on the GPU."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import PRECISIONS, Segment, lib
from ._lib import check as check_rc

_workspaces: dict = {}
_retired: list = []  # buffers a captured graph may still write: never freed


def _stream_ptr(stream, device) -> int:
    if stream is None:
        return torch.cuda.current_stream(device).cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _torch_stream(stream, device):
    if stream is None:
        return torch.cuda.current_stream(device)
    if isinstance(stream, torch.cuda.Stream):
        return stream
    return torch.cuda.ExternalStream(int(stream), device=device)


def workspace(nbytes: int, device, stream=None) -> torch.Tensor:
    """Scratch buffer of one (device, stream), grown on demand and reused by
    later calls on that stream (calls on one stream are ordered, so they never
    overlap in it).  A buffer that was used while the stream was being
    captured into a graph stays allocated when it is outgrown: the graph keeps
    its address."""
    dev = torch.device(device)
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    key = (idx, _stream_ptr(stream, dev))
    ent = _workspaces.get(key)
    capturing = torch.cuda.is_current_stream_capturing()
    if ent is None or ent[0].numel() < nbytes:
        if ent is not None and ent[1]:
            _retired.append(ent[0])
        buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=dev)
        ent = [buf, False]
        _workspaces[key] = ent
    ent[1] = ent[1] or capturing
    return ent[0]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _need_cuda(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA (HIP) tensor" % name)


def check_input_values(syndromes, rates, model_index=None, meas_rates=None):
    """Value checks of one segment's inputs (any device; one host read-back):
    syndrome bytes in {0, 1}, model indices in [0, M), rates in [0, 1] with no
    NaN and p_X + p_Y + p_Z <= 1 + 1e-12 per qubit, measurement flip rates (if
    given) in [0, 1].  Raises ValueError.  The kernels repeat these checks per
    syndrome (tn_workspace_status)."""
    r = rates if rates.dim() == 3 else rates.unsqueeze(0)
    flags = [(syndromes > 1).any()]
    ok01 = (r >= 0) & (r <= 1)  # False for NaN
    flags.append(~ok01.all())
    flags.append((r.sum(-1) > 1.0 + 1e-12).any())
    if model_index is not None and model_index.numel() > 0:
        flags.append((model_index < 0).any() | (model_index >= r.shape[0]).any())
    else:
        flags.append(torch.zeros((), dtype=torch.bool, device=r.device))
    if meas_rates is not None:
        flags.append(~((meas_rates >= 0) & (meas_rates <= 1)).all())
    else:
        flags.append(torch.zeros((), dtype=torch.bool, device=r.device))
    bad = torch.stack([f.to(torch.bool).reshape(()) for f in flags]).tolist()
    what = ["a syndrome byte above 1", "a rate outside [0, 1] or NaN", "p_X + p_Y + p_Z above 1",
            "a model index outside [0, %d)" % r.shape[0], "a measurement flip rate outside [0, 1] or NaN"]
    msg = [w for w, b in zip(what, bad) if b]
    if msg:
        raise ValueError("invalid decoder inputs: " + ", ".join(msg))


@dataclass
class SegmentInput:
    """One homogeneous group: distance d, bond cap chi, precision, noise models."""
    d: int
    chi: int
    syndromes: torch.Tensor            # uint8 [B, d*d-1] on the GPU
    rates: torch.Tensor                # float64 [M, d*d, 3] (or [d*d, 3]) on the GPU
    model_index: torch.Tensor | None = None  # int32 [B] or None
    precision: str = "fp32"
    rounds: int = 1                    # T >= 2: repeated noisy rounds, syndromes [B, T, d*d-1], last round perfect
    meas_rates: torch.Tensor | None = None  # float64 [M, d*d-1] (or [d*d-1]): check flip rates of rounds 1..T-1


@dataclass
class SegmentOutput:
    logz: torch.Tensor   # float64 [B, 4]
    logp: torch.Tensor   # float64 [B]
    cls: torch.Tensor    # uint8 [B]


def _prepare(segs, check=True):
    if not 1 <= len(segs) <= _lib.TN_MAX_SEGMENTS:
        raise ValueError("between 1 and 16 segments per call")
    arr = (Segment * len(segs))()
    outs, keep = [], []
    for i, s in enumerate(segs):
        _need_cuda(s.syndromes, "syndromes")
        _need_cuda(s.rates, "rates")
        n, m = s.d * s.d, s.d * s.d - 1
        T = int(s.rounds) if s.rounds else 1
        if not 1 <= T <= _lib.TN_MAX_ROUNDS:
            raise ValueError("rounds must be in [1, %d]" % _lib.TN_MAX_ROUNDS)
        syn = s.syndromes.to(torch.uint8).contiguous()
        if T > 1 and syn.dim() == 3:
            if syn.shape[1:] != (T, m):
                raise ValueError("syndromes must be [B, T, d*d-1]")
            syn = syn.reshape(syn.shape[0], T * m)
        if syn.dim() != 2 or syn.shape[1] != m * T:
            raise ValueError("syndromes must be [B, d*d-1]" if T == 1 else "syndromes must be [B, T, d*d-1]")
        rates = s.rates.to(torch.float64).contiguous()
        if rates.dim() == 2:
            rates = rates.unsqueeze(0)
        if rates.shape[1:] != (n, 3):
            raise ValueError("rates must be [M, d*d, 3]")
        mi = None
        if s.model_index is not None:
            _need_cuda(s.model_index, "model_index")
            mi = s.model_index.to(torch.int32).contiguous()
            if mi.shape != (syn.shape[0],):
                raise ValueError("model_index must be [B]")
        meas = None
        if T > 1:
            if s.meas_rates is None:
                raise ValueError("repeated rounds need meas_rates")
            _need_cuda(s.meas_rates, "meas_rates")
            meas = s.meas_rates.to(torch.float64).contiguous()
            if meas.dim() == 1:
                meas = meas.unsqueeze(0)
            if meas.shape != (rates.shape[0], m):
                raise ValueError("meas_rates must be [M, d*d-1]")
        if check:
            check_input_values(syn, rates, mi, meas)
        b = syn.shape[0]
        dev = syn.device
        o = SegmentOutput(torch.empty((b, 4), dtype=torch.float64, device=dev),
                          torch.empty(b, dtype=torch.float64, device=dev),
                          torch.empty(b, dtype=torch.uint8, device=dev))
        arr[i] = Segment(s.d, s.chi, PRECISIONS[s.precision], rates.shape[0], rates.data_ptr(),
                         mi.data_ptr() if mi is not None else None, syn.data_ptr(), b,
                         o.logz.data_ptr(), o.logp.data_ptr(), o.cls.data_ptr(),
                         T, 0, meas.data_ptr() if meas is not None else None)
        outs.append(o)
        keep += [t for t in (syn, rates, mi, meas) if t is not None]
    return arr, outs, keep


def _launch_stream(stream, dev, keep, outs):
    """Raw stream pointer of the launch; when it is not the current stream,
    the temporaries and outputs (allocated on the current stream) are marked
    as used by it, so the caching allocator does not hand their memory out
    while the kernels may still read or write it."""
    cur = torch.cuda.current_stream(dev)
    ptr = _stream_ptr(stream, dev)
    if ptr != cur.cuda_stream:
        ts = _torch_stream(stream, dev)
        for t in keep:
            t.record_stream(ts)
        for o in outs:
            for t in (o.logz, o.logp, o.cls):
                t.record_stream(ts)
    return ptr


class UnresolvedCosetsWarning(RuntimeWarning):
    """Some cosets of strictly positive noise models came out with Z <= 0 in
    a reduced-precision form and were reported as -inf (below the form's
    resolution at their syndrome; log P(s) and the class are unaffected)."""


def _check_status(ws, st_ptr):
    """Read the call's status word (synchronises the stream): raises TNError
    for TN_EINVAL (invalid input values) and TN_ENUMERIC (a syndrome's log P(s)
    was lost); warns with the count of unresolved cosets.  Returns that count."""
    cnt = ctypes.c_int64(0)
    check_rc(lib().tn_workspace_status(ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(st_ptr),
                                       ctypes.byref(cnt)))
    if cnt.value:
        import warnings
        warnings.warn("%d coset(s) below the resolution of the precision form were reported as log Z = -inf"
                      % cnt.value, UnresolvedCosetsWarning, stacklevel=3)
    return int(cnt.value)


def decode_segments(segs, tie_tol: float = 1e-9, stream=None, workspace_buf=None, check: bool = True):
    """Decode several segments in one persistent launch per precision.

    stream: torch.cuda.Stream or raw hipStream_t (default: the current
    stream).  workspace_buf: caller-owned uint8 device tensor of at least
    workspace_bytes(segs) bytes (default: a buffer kept per device and
    stream).  check: True validates the input values on the host before the
    launch and reads the call's status word after it (TN_EINVAL, TN_ENUMERIC;
    both synchronise), "device" only reads the status word, False neither;
    both are skipped while the stream is being captured into a graph."""
    capturing = torch.cuda.is_current_stream_capturing()
    do_check = bool(check) and not capturing
    arr, outs, keep = _prepare(segs, do_check and check != "device")
    L = lib()
    nbytes = L.tn_workspace_size(arr, len(segs), 0)
    if nbytes == 0:
        check_rc(_lib.TN_EINVAL if not L.tn_last_error() else -1)
    dev = segs[0].syndromes.device
    ws = _pick_workspace(workspace_buf, nbytes, dev, stream)
    st = _launch_stream(stream, dev, keep, outs)
    check_rc(L.tn_decode_batch(arr, len(segs), float(tie_tol), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                               ctypes.c_void_p(st)))
    if do_check:
        _check_status(ws, st)
    del keep
    return outs


def _pick_workspace(buf, nbytes, dev, stream):
    if buf is None:
        return workspace(nbytes, dev, stream)
    if buf.dtype != torch.uint8 or not buf.is_cuda or buf.numel() < nbytes:
        raise ValueError("workspace_buf must be a uint8 device tensor of at least %d bytes" % nbytes)
    return buf


def workspace_bytes(segs, with_backward=False):
    """Bytes of device workspace a call on these segments needs."""
    arr, _, _ = _prepare(segs, check=False)
    n = lib().tn_workspace_size(arr, len(segs), 1 if with_backward else 0)
    if n == 0:
        check_rc(_lib.TN_EINVAL)
    return int(n)


def decode(syndromes, rates, d, chi, precision="fp32", model_index=None, tie_tol=1e-9):
    """(logz [B,4], logp [B], class [B]) for one homogeneous batch."""
    o = decode_segments([SegmentInput(d, chi, syndromes, rates, model_index, precision)], tie_tol)[0]
    return o.logz, o.logp, o.cls


def decode_rounds(syndromes, rates, meas_rates, d, chi, precision="fp32", model_index=None, tie_tol=1e-9):
    """Repeated noisy rounds: syndromes [B, T, d*d-1] (rounds 1..T-1 with check
    flips at meas_rates [M, d*d-1], round T perfect), rates [M, d*d, 3].
    Returns (logz [B,4], logp [B], class [B]) of the accumulated error."""
    T = int(syndromes.shape[1])
    o = decode_segments([SegmentInput(d, chi, syndromes, rates, model_index, precision, T, meas_rates)], tie_tol)[0]
    return o.logz, o.logp, o.cls


def coset_loglik(syndromes, rates, d, chi, precision="fp32", model_index=None, check=True):
    """log Z_l(s) [B,4] and log P(s) [B]."""
    do_check = check and not torch.cuda.is_current_stream_capturing()
    arr, outs, keep = _prepare([SegmentInput(d, chi, syndromes, rates, model_index, precision)], do_check)
    L = lib()
    nbytes = L.tn_workspace_size(arr, 1, 0)
    if nbytes == 0:
        check_rc(_lib.TN_EINVAL)
    ws = workspace(nbytes, syndromes.device)
    st = torch.cuda.current_stream(syndromes.device).cuda_stream
    check_rc(L.tn_coset_loglik(arr, 1, ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(st)))
    if do_check:
        _check_status(ws, st)
    del keep
    return outs[0].logz, outs[0].logp


def coset_loglik_backward(segs, grad_logp, stream=None, outputs=None, workspace_buf=None, check=True):
    """d (sum_b grad_logp[b] log P(s_b)) / d ln rates for each segment.

    grad_logp: list of float64 [B] device tensors, one per segment.  outputs:
    the SegmentOutput list of an earlier decode of exactly these inputs, whose
    log Z / log P(s) are then reused instead of recomputed.  Returns
    (outputs, grads) with grads[i] float64 [M, d*d, 3] (a fresh zeroed tensor
    that the library accumulates into).  stream, workspace_buf, check: as for
    decode_segments."""
    if any((s.rounds or 1) > 1 for s in segs):
        raise ValueError("the gradient takes segments of one syndrome round")
    do_check = bool(check) and not torch.cuda.is_current_stream_capturing()
    arr, outs, keep = _prepare(segs, do_check and check != "device")
    forward_done = 0
    if outputs is not None:
        if len(outputs) != len(segs):
            raise ValueError("one output per segment")
        for i, o in enumerate(outputs):
            if o.logz.shape != outs[i].logz.shape or o.logp.shape != outs[i].logp.shape:
                raise ValueError("outputs do not match the segments")
            arr[i].out_logz = o.logz.data_ptr()
            arr[i].out_logp = o.logp.data_ptr()
            arr[i].out_class = o.cls.data_ptr()
        outs = list(outputs)
        forward_done = 1
    L = lib()
    nbytes = L.tn_workspace_size(arr, len(segs), 1)
    if nbytes == 0:
        check_rc(_lib.TN_EINVAL if not L.tn_last_error() else -1)
    dev = segs[0].syndromes.device
    ws = _pick_workspace(workspace_buf, nbytes, dev, stream)
    gp = [g.to(device=dev, dtype=torch.float64).contiguous() for g in grad_logp]
    grads = []
    for s, g in zip(segs, gp):
        m = s.rates.shape[0] if s.rates.dim() == 3 else 1
        if g.shape != (s.syndromes.shape[0],):
            raise ValueError("grad_logp[i] must be [B]")
        grads.append(torch.zeros((m, s.d * s.d, 3), dtype=torch.float64, device=dev))
    gp_arr = (ctypes.c_void_p * len(segs))(*[g.data_ptr() for g in gp])
    gr_arr = (ctypes.c_void_p * len(segs))(*[g.data_ptr() for g in grads])
    st = _launch_stream(stream, dev, keep + gp + grads, outs)
    check_rc(L.tn_coset_loglik_backward(arr, len(segs), gp_arr, gr_arr, forward_done, ctypes.c_void_p(ws.data_ptr()),
                                        ws.numel(), ctypes.c_void_p(st)))
    if do_check:
        _check_status(ws, st)
    del keep
    return outs, grads


def states_bytes(segs):
    """Device bytes of the top-sweep states that coset_loglik_save keeps for
    coset_loglik_backward_saved (the MPS before every row of every coset, the
    rows common to the cosets once per syndrome)."""
    arr, _, _ = _prepare(segs, check=False)
    return int(lib().tn_states_size(arr, len(segs)))


def coset_loglik_save(segs, stream=None, workspace_buf=None, check: bool = True, states=None):
    """First call of the two-call gradient: log Z / log P(s) of every segment
    (as coset_loglik) and the top sweep's states, kept in a device buffer for
    coset_loglik_backward_saved, which then runs only the bottom sweeps.
    Returns (outputs, states).  states: optional caller-owned uint8 device
    tensor of at least states_bytes(segs) bytes."""
    capturing = torch.cuda.is_current_stream_capturing()
    do_check = bool(check) and not capturing
    arr, outs, keep = _prepare(segs, do_check and check != "device")
    L = lib()
    nbytes = L.tn_workspace_size(arr, len(segs), 1)
    sbytes = L.tn_states_size(arr, len(segs))
    if nbytes == 0 or sbytes == 0:
        check_rc(_lib.TN_EINVAL if not L.tn_last_error() else -1)
    dev = segs[0].syndromes.device
    ws = _pick_workspace(workspace_buf, nbytes, dev, stream)
    if states is None:
        states = torch.empty(sbytes, dtype=torch.uint8, device=dev)
    elif states.dtype != torch.uint8 or not states.is_cuda or states.numel() < sbytes:
        raise ValueError("states must be a uint8 device tensor of at least %d bytes" % sbytes)
    st = _launch_stream(stream, dev, keep + [states], outs)
    check_rc(L.tn_coset_loglik_save(arr, len(segs), ctypes.c_void_p(states.data_ptr()), states.numel(),
                                    ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(st)))
    if do_check:
        _check_status(ws, st)
    del keep
    return outs, states


def coset_loglik_backward_saved(segs, grad_logp, outputs, states, stream=None, workspace_buf=None, check=True):
    """Second call of the two-call gradient: d (sum_b grad_logp[b] log P(s_b))
    / d ln rates from the outputs and states of coset_loglik_save on exactly
    these inputs (the bottom sweeps and row environments only).  Returns grads
    as coset_loglik_backward."""
    if any((s.rounds or 1) > 1 for s in segs):
        raise ValueError("the gradient takes segments of one syndrome round")
    arr, outs, keep = _prepare(segs, False)
    if len(outputs) != len(segs):
        raise ValueError("one output per segment")
    for i, o in enumerate(outputs):
        if o.logz.shape != outs[i].logz.shape or o.logp.shape != outs[i].logp.shape:
            raise ValueError("outputs do not match the segments")
        arr[i].out_logz = o.logz.data_ptr()
        arr[i].out_logp = o.logp.data_ptr()
        arr[i].out_class = o.cls.data_ptr()
    L = lib()
    nbytes = L.tn_workspace_size(arr, len(segs), 1)
    if nbytes == 0:
        check_rc(_lib.TN_EINVAL if not L.tn_last_error() else -1)
    dev = segs[0].syndromes.device
    ws = _pick_workspace(workspace_buf, nbytes, dev, stream)
    gp = [g.to(device=dev, dtype=torch.float64).contiguous() for g in grad_logp]
    grads = []
    for s, g in zip(segs, gp):
        m = s.rates.shape[0] if s.rates.dim() == 3 else 1
        if g.shape != (s.syndromes.shape[0],):
            raise ValueError("grad_logp[i] must be [B]")
        grads.append(torch.zeros((m, s.d * s.d, 3), dtype=torch.float64, device=dev))
    gp_arr = (ctypes.c_void_p * len(segs))(*[g.data_ptr() for g in gp])
    gr_arr = (ctypes.c_void_p * len(segs))(*[g.data_ptr() for g in grads])
    st = _launch_stream(stream, dev, keep + gp + grads + [states], list(outputs))
    check_rc(L.tn_coset_loglik_backward_saved(arr, len(segs), gp_arr, gr_arr, ctypes.c_void_p(states.data_ptr()),
                                              states.numel(), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                              ctypes.c_void_p(st)))
    do_check = bool(check) and not torch.cuda.is_current_stream_capturing()
    if do_check:
        _check_status(ws, st)
    del keep
    return grads


# Largest top-sweep state buffer the autograd binding keeps between its
# forward and backward; above it the backward recomputes the top sweep.
STATES_LIMIT_BYTES = 32 << 30


class _LogPosterior(torch.autograd.Function):
    """log P(s_b) as a function of theta = ln rates; the backward is the
    library's adjoint contraction.  The forward keeps the top sweep's states
    (when they fit STATES_LIMIT_BYTES), so the backward runs only the bottom
    sweeps."""

    @staticmethod
    def forward(ctx, log_rates, syndromes, model_index, d, chi, precision, keep_states):
        rates = log_rates.detach().exp()
        seg = SegmentInput(d, chi, syndromes, rates, model_index, precision)
        ctx.states = None
        if keep_states and states_bytes([seg]) <= STATES_LIMIT_BYTES:
            outs, ctx.states = coset_loglik_save([seg])
            o = outs[0]
        else:
            o = decode_segments([seg])[0]
        ctx.seg = seg
        ctx.out = o
        ctx.rates_dim = log_rates.dim()
        ctx.mark_non_differentiable(o.logz)
        return o.logp, o.logz

    @staticmethod
    def backward(ctx, g_logp, g_logz):
        if g_logz is not None and bool((g_logz != 0).any()):
            raise NotImplementedError("only log P(s) is differentiable")
        if ctx.states is not None:
            grads = coset_loglik_backward_saved([ctx.seg], [g_logp], [ctx.out], ctx.states)
            ctx.states = None
        else:
            _, grads = coset_loglik_backward([ctx.seg], [g_logp], outputs=[ctx.out])
        g = grads[0] if ctx.rates_dim == 3 else grads[0][0]
        return g, None, None, None, None, None, None


def log_posterior(log_rates, syndromes, d, chi, precision="fp32", model_index=None):
    """(log P(s) [B], log Z [B, 4]) with autograd through log_rates
    ([d*d, 3] or [M, d*d, 3] float64 = ln p_{q,X|Y|Z}).  The forward keeps the
    top sweep's states for the backward only when a gradient can follow."""
    keep = torch.is_grad_enabled() and log_rates.requires_grad
    return _LogPosterior.apply(log_rates, syndromes, model_index, d, chi, precision, keep)


def _bitflip_rates(rates, n):
    r = rates.to(torch.float64)
    if r.dim() == 1:  # p_X per qubit
        r = torch.stack([r, torch.zeros_like(r), torch.zeros_like(r)], -1)
    if r.dim() == 2:
        r = r.unsqueeze(0)
    if r.shape[1:] != (n, 3):
        raise ValueError("bit-flip rates must be [d*d] (p_X), [d*d, 3] or [M, d*d, 3]")
    return r.contiguous()


def decode_bitflip_segments(segs, tie_tol: float = 1e-9, stream=None, workspace_buf=None, check: bool = True):
    """Exact decoding under bit-flip noise by the planar (Kac-Ward) solver.

    segs: SegmentInput list (chi and precision are ignored; the solver runs in
    FP64); rates may be p_X per qubit [d*d].  Returns SegmentOutput per
    segment: log Z (Y and Z cosets -inf), log P(s), class.  check: as for
    decode_segments (the host check also requires p_Y = p_Z = 0)."""
    capturing = torch.cuda.is_current_stream_capturing()
    do_check = bool(check) and not capturing
    conv = []
    for s in segs:
        _need_cuda(s.rates, "rates")
        r = _bitflip_rates(s.rates, s.d * s.d)
        if do_check and check != "device" and bool((r[..., 1:] != 0).any()):
            raise ValueError("the planar solver needs bit-flip noise: p_Y = p_Z = 0")
        conv.append(SegmentInput(s.d, 0, s.syndromes, r, s.model_index, "fp64"))
    arr, outs, keep = _prepare(conv, do_check and check != "device")
    L = lib()
    nbytes = L.tn_bitflip_workspace_size(arr, len(conv))
    if nbytes == 0:
        check_rc(_lib.TN_EINVAL)
    dev = conv[0].syndromes.device
    ws = _pick_workspace(workspace_buf, nbytes, dev, stream)
    st = _launch_stream(stream, dev, keep, outs)
    check_rc(L.tn_bitflip_decode(arr, len(conv), float(tie_tol), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                 ctypes.c_void_p(st)))
    if do_check:
        _check_status(ws, st)
    del keep
    return outs


def decode_bitflip(syndromes, rates, d, model_index=None, tie_tol=1e-9):
    """(logz [B,4], logp [B], class [B]) under bit-flip noise, exactly."""
    o = decode_bitflip_segments([SegmentInput(d, 0, syndromes, rates, model_index, "fp64")], tie_tol)[0]
    return o.logz, o.logp, o.cls


def bitflip_plan_info(d):
    info = (ctypes.c_double * 5)()
    check_rc(lib().tn_bitflip_plan_info(d, info))
    return dict(order=int(info[0]), nnz=int(info[1]), lu_flops=info[2], scratch_bytes=info[3], log_pref=info[4])


def plan_info(d, chi, precision="fp32", rounds=1):
    info = (ctypes.c_double * 8)()
    check_rc(lib().tn_plan_info_rounds(d, chi, PRECISIONS[precision], int(rounds), info))
    out = dict(flops=info[0], scratch_bytes=info[1], lds_bytes=info[2], sites=int(info[3]),
               rows=int(info[4]), group=int(info[5]), wg_per_cu=int(info[6]), flops_syndrome=info[7])
    if rounds <= 1:  # GEMM-class and adjoint counts of the one-round plan
        gemm = (ctypes.c_double * 2)()
        check_rc(lib().tn_plan_gemm_flops(d, chi, PRECISIONS[precision], gemm))
        out.update(gemm_flops=gemm[0], gemm_flops_syndrome=gemm[1])
        adj = (ctypes.c_double * 3)()
        check_rc(lib().tn_plan_adjoint_flops(d, chi, PRECISIONS[precision], adj))
        out.update(bottom_sweep_flops=adj[0], environment_flops=adj[1], adjoint_flops_syndrome=adj[2])
    return out


def set_tuning(d, chi, precision, group=0, wg_per_cu=0, threads=0):
    """Launch shape for (d, chi, precision): columns per site, work-groups per
    CU, work-group size (512 or 256; 0 automatic); zeros restore the default."""
    check_rc(lib().tn_set_tuning_ex(d, chi, PRECISIONS[precision], group, wg_per_cu, threads))


def launch_shape(d, chi, precision):
    """(group, wg_per_cu, threads) a one-segment call of this bucket uses now."""
    out = (ctypes.c_int32 * 3)()
    check_rc(lib().tn_get_launch(d, chi, PRECISIONS[precision], out))
    return int(out[0]), int(out[1]), int(out[2])


def launch_plan(segs):
    """The persistent forward launches decode_segments(segs) makes, in order:
    dicts of precision, threads, wg_per_cu and the number of segments each
    carries."""
    arr, _, _ = _prepare(segs, check=False)
    cap = 3 * len(PRECISIONS)
    out = (ctypes.c_int32 * (4 * cap))()
    count = ctypes.c_int32(0)
    check_rc(lib().tn_get_launches(arr, len(segs), out, cap, ctypes.byref(count)))
    names = {v: k for k, v in PRECISIONS.items()}
    return [dict(precision=names[out[4 * i]], threads=int(out[4 * i + 1]), wg_per_cu=int(out[4 * i + 2]),
                 segments=int(out[4 * i + 3])) for i in range(min(count.value, cap))]


def code_stabilizers(d):
    import numpy as np
    m = d * d - 1
    t = np.zeros(m, np.int32)
    s = np.zeros((m, 4), np.int32)
    rc = lib().tn_code_stabilizers(d, t.ctypes.data_as(ctypes.c_void_p), s.ctypes.data_as(ctypes.c_void_p))
    if rc < 0:
        check_rc(rc)
    return t, s
