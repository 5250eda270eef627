"""Bilevel tuning of the regularization parameter over a batch of problems.

Each problem p has its own lambda_p, optimized on a validation loss with an independent
noise draw b_val (Sec. 2 eq. (tiksol) for x(lambda); the adjoint for dL/dlambda):

    L_p(lambda_p) = 1/2 ||T_p x_p(lambda_p) - b_val,p||^2,
    dL/dx = T^H (T x - b_val) = T^H (b - b_val) - lambda^2 x      (normal equations of x),
    dL/dlambda = -2 lambda Re<w, x>,  w = (T^H T + lambda^2 I)^{-1} dL/dx   (backward solve),

with Adam on log lambda.  One step = the batched forward solve, the upstream gradient, the
batched backward solve and the Adam update; the two solves are prepared batches
(tikh_prepare_batched / tikh_prepare_backward_batched), so the whole step is captured into
one graph and replayed.  The constant T^H (b - b_val), T^H b and T^H b_val are formed once
with the library's FFT (circulant embedding of T).  The elementwise work of a step (the
upstream gradient, the Adam update, the loss) is PyTorch on the device.
"""

import torch

from . import _lib


def _circulant_spectra(ms, ns, col, row):
    """Per problem: (N, spectrum of the circulant C_N whose top-left m x n block is T),
    with the library's FFT (sign -1) and its own extension size N."""
    out = []
    co = ro = 0
    for m, n in zip(ms, ns):
        N = _lib.plan_info(m, n)[0]
        c = torch.zeros((1, 1, N), dtype=torch.complex128, device=col.device)
        c[0, 0, :m] = col[co:co + m].to(torch.complex128)
        if n > 1:
            # C[N - s, 0] = a_{-s}, s = 1..n-1
            c[0, 0, N - n + 1:] = torch.flip(row[ro + 1:ro + n], dims=[0]).to(torch.complex128)
        _lib.fft_batched(c, -1)
        out.append((N, c[0, 0]))
        co += m
        ro += n
    return out


def _circ_apply(spectra, lin, lout, v, adjoint):
    res = []
    vo = 0
    for (N, chat), a, c in zip(spectra, lin, lout):
        buf = torch.zeros((1, 1, N), dtype=torch.complex128, device=v.device)
        buf[0, 0, :a] = v[vo:vo + a].to(torch.complex128)
        _lib.fft_batched(buf, -1)
        buf[0, 0] *= torch.conj(chat) if adjoint else chat
        _lib.fft_batched(buf, +1)
        r = buf[0, 0, :c] / N
        res.append(r if v.is_complex() else r.real.contiguous())
        vo += a
    return torch.cat(res)


def adjoint_apply(spectra, ms, ns, v):
    """T_p^H v_p for every problem (v packed [sum m]); returns the packed [sum n] result."""
    return _circ_apply(spectra, ms, ns, v, True)


def apply(spectra, ms, ns, x):
    """T_p x_p for every problem (x packed [sum n]); returns the packed [sum m] result."""
    return _circ_apply(spectra, ns, ms, x, False)


class BilevelTuner:
    """Adam on log lambda for a batch of real problems (one right-hand side each).

    ms, ns: host sizes; col, row, b, b_val: packed float64 device tensors (col/b/b_val
    [sum m], row [sum n]); lam0: initial lambdas [nprob] (device).  capture() records one
    step into a graph; step() replays it (or runs it eagerly before capture)."""

    def __init__(self, ms, ns, col, row, b, b_val, lam0, lr=0.1, betas=(0.9, 0.999), eps=1e-8, **options):
        """options: library options (set_options keywords) in force while the two batches are
        prepared; they apply to every run of them.  By default merge_tol = 4: extended sizes
        within a factor 5 share one plan, so a batch spanning 2^12..2^16 runs as two chunks
        (measured on 256 problems: 4.7 s per step against 9.2 s with the library's default
        of 0.25, whose dozen chunks of ~20 small groups are bound by launch overhead), and
        refine = 2: a prepared batch takes a fixed number of refinement steps (no adaptive
        ones), and with one step a few solves of the 256-problem workload end above the
        refinement's failure estimate (info bit 16) once lambda has fallen below 4e-3 (from
        step 10 of 20); with two none do (7.2 s per step)."""
        options.setdefault("merge_tol", 4.0)
        options.setdefault("refine", 2)
        dev = col.device
        self.ms, self.ns = list(ms), list(ns)
        self.nprob = len(ms)
        self.lr, self.b1, self.b2, self.eps = float(lr), float(betas[0]), float(betas[1]), float(eps)
        self.loglam = torch.log(lam0.to(torch.float64)).contiguous()
        self.lam = torch.exp(self.loglam)
        self._spectra = spectra = _circulant_spectra(self.ms, self.ns, col, row)
        self._bval = b_val
        self.d = adjoint_apply(spectra, self.ms, self.ns, b - b_val)           # T^H (b - b_val)
        self.y_b = adjoint_apply(spectra, self.ms, self.ns, b)                 # T^H b
        self.y_val = adjoint_apply(spectra, self.ms, self.ns, b_val)           # T^H b_val
        self.bval_sq = torch.stack([torch.dot(b_val[o:o + m], b_val[o:o + m])
                                    for o, m in zip(_offsets(self.ms), self.ms)])
        self.idx = torch.cat([torch.full((n,), p, dtype=torch.int64, device=dev) for p, n in enumerate(self.ns)])
        keep = _lib.get_options()
        _lib.set_options(**options)
        try:
            self.fwd = _lib.prepare_batched(self.ms, self.ns, col, row, self.lam, 1, b)
            self.gx = torch.empty_like(self.fwd.x)
            self._upstream()
            self.bwd = _lib.prepare_backward_batched(self.ms, self.ns, col, row, self.lam, 1, b, self.fwd.x,
                                                     self.gx)
        finally:
            _lib.set_options(**keep)
        self.m = torch.zeros(self.nprob, dtype=torch.float64, device=dev)
        self.v = torch.zeros_like(self.m)
        self.t = torch.zeros((), dtype=torch.float64, device=dev)
        self.grad = torch.zeros_like(self.m)      # dL/dlog(lambda) of the last step
        # L at the lambdas the last step started from, by the normal-equation identity below
        # (no products with T inside the step; the cancellation in it leaves a relative error
        # of about ||x - x*|| ||b||^2 / (||x|| L), i.e. 1e-5 at a solve error of 1e-12 and
        # L / ||b||^2 = 1e-7: a running estimate; validation_loss() gives L to rounding)
        self.loss = torch.zeros_like(self.m)
        self.graph = None

    def _upstream(self):
        lx = self.lam.index_select(0, self.idx)
        torch.sub(self.d, lx * lx * self.fwd.x, out=self.gx)

    def _ops(self):
        self.fwd.run()
        self._upstream()
        x = self.fwd.x
        # L = 1/2 (<x, T^H b - lambda^2 x> - 2 <x, T^H b_val> + ||b_val||^2)
        lx = self.lam.index_select(0, self.idx)
        term = x * (self.y_b - lx * lx * x - 2.0 * self.y_val)
        self.loss.zero_()
        self.loss.index_add_(0, self.idx, term)
        self.loss.add_(self.bval_sq).mul_(0.5)
        self.bwd.run()
        torch.mul(self.lam, self.bwd.g_lam, out=self.grad)
        self.t.add_(1.0)
        self.m.mul_(self.b1).add_(self.grad, alpha=1.0 - self.b1)
        self.v.mul_(self.b2).addcmul_(self.grad, self.grad, value=1.0 - self.b2)
        mhat = self.m / (1.0 - torch.pow(self.b1, self.t))
        vhat = self.v / (1.0 - torch.pow(self.b2, self.t))
        self.loglam.sub_(self.lr * mhat / (torch.sqrt(vhat) + self.eps))
        torch.exp(self.loglam, out=self.lam)

    def validation_loss(self):
        """L_p = 1/2 ||T_p x_p - b_val,p||^2 at the current forward solutions x (outside any
        graph: products with T by the library's FFT)."""
        r = apply(self._spectra, self.ms, self.ns, self.fwd.x) - self._bval
        out = torch.zeros(self.nprob, dtype=torch.float64, device=r.device)
        idx = torch.cat([torch.full((m,), p, dtype=torch.int64, device=r.device) for p, m in enumerate(self.ms)])
        out.index_add_(0, idx, r * r)
        return 0.5 * out

    def state(self):
        return [t.clone() for t in (self.loglam, self.lam, self.m, self.v, self.t)]

    def set_state(self, s):
        for dst, src in zip((self.loglam, self.lam, self.m, self.v, self.t), s):
            dst.copy_(src)

    def capture(self):
        """One eager step on a side stream (loads every kernel), the state restored, then the
        step recorded into a graph."""
        s0 = self.state()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self._ops()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        # the eager step's results, for comparison with the first replay
        self.eager_step = (self.loglam.clone(), self.grad.clone(), self.loss.clone())
        self.set_state(s0)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._ops()
        torch.cuda.synchronize()

    def step(self):
        if self.graph is not None:
            self.graph.replay()
        else:
            self._ops()

    def info(self):
        return self.fwd.info, self.bwd.info

    def free(self):
        self.graph = None
        self.bwd.free()
        self.fwd.free()


def _offsets(sizes):
    out, o = [], 0
    for s in sizes:
        out.append(o)
        o += s
    return out
