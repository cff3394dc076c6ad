"""The learned correction of the sampled preconditioner.

The sampled plan (``MixedPlan(sample_rows=...)``) factors a row sample of A in
FP32 and uses that R~ to precondition the FP64 correction; the result is the
R of A whatever R~ is, as long as A R~^-1 is well conditioned.  This module
trains a small MLP that maps features of a sampled R~ (its log-diagonal
profile and first superdiagonal, ``tsqr_surrogate_features``) to a row
scaling of it (``tsqr_surrogate_apply``), fitted to the diagonal of the R of
all of A (``tsqr_surrogate_targets``).  Every arithmetic step runs in the
library's kernels: the layers are ``tsqr_gemm_bf16`` (BF16 matrix cores, FP32
accumulation), then ``tsqr_mlp_bias_act``; the backward pass uses the same
GEMM with transposed operands, ``tsqr_mlp_relu_grad`` and ``tsqr_mlp_colsum``;
the loss is ``tsqr_mlp_mse`` and the update ``tsqr_mlp_adam``.  This module
only allocates device tensors and sequences the calls.
"""
import ctypes

from . import tsqr


def _p(t):
    return t.data_ptr()


class Mlp:
    """F -> H -> H -> O with ReLU after the two hidden layers; parameters and
    activations are FP32 device tensors, stored column-major (a batch of B
    rows is a B x width matrix with leading dimension B).  He-initialized
    hidden layers; with ``zero_output`` the output layer starts at zero, so
    the untrained network outputs the zero correction."""

    def __init__(self, F, O, H=256, seed=0, device=None, h=None, zero_output=True):
        import torch
        self.torch = torch
        self.dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.h = h or tsqr.handle(self.dev.index or 0)
        self.F, self.H, self.O = int(F), int(H), int(O)
        g = torch.Generator(device="cpu")
        g.manual_seed(int(seed))
        shapes = [(self.F, self.H), (self.H,), (self.H, self.H), (self.H,), (self.H, self.O), (self.O,)]
        self.params = []
        for k, shp in enumerate(shapes):
            if len(shp) == 2 and (k < 4 or not zero_output):     # He initialization, column-major storage: W[i + j ld]
                w = torch.randn(shp[1], shp[0], generator=g) * (2.0 / shp[0]) ** 0.5
                self.params.append(w.reshape(-1).to(self.dev))
            else:
                # biases, and the output layer, start at zero: the untrained
                # network is the zero correction (the un-learned R~)
                self.params.append(torch.zeros(shp[0] * (shp[1] if len(shp) == 2 else 1), device=self.dev))
        self.grads = [torch.zeros_like(p) for p in self.params]
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.loss = torch.zeros(1, device=self.dev)
        self.t = 0
        self._acts = None

    def _stream(self):
        return tsqr._stream_ptr(self.torch, self.dev)

    def _gemm(self, ta, tb, M, N, K, A, lda, B, ldb, C, ldc, beta=0.0):
        st = tsqr.lib().tsqr_gemm_bf16(self.h, int(ta), int(tb), M, N, K, 1.0, _p(A), lda, _p(B), ldb, float(beta),
                                       _p(C), ldc, self._stream())
        tsqr._check("tsqr_gemm_bf16", st, self.h)

    def _bias_act(self, Z, rows, cols, bias, relu):
        st = tsqr.lib().tsqr_mlp_bias_act(self.h, _p(Z), rows, cols, rows, _p(bias), int(relu), self._stream())
        tsqr._check("tsqr_mlp_bias_act", st, self.h)

    def forward(self, X, B):
        """Y (B x O) for the input X (B x F, column-major, ld B)."""
        torch = self.torch
        W1, b1, W2, b2, W3, b3 = self.params
        Z1 = torch.empty(B * self.H, device=self.dev)
        Z2 = torch.empty(B * self.H, device=self.dev)
        Y = torch.empty(B * self.O, device=self.dev)
        self._gemm(0, 0, B, self.H, self.F, X, B, W1, self.F, Z1, B)
        self._bias_act(Z1, B, self.H, b1, True)
        self._gemm(0, 0, B, self.H, self.H, Z1, B, W2, self.H, Z2, B)
        self._bias_act(Z2, B, self.H, b2, True)
        self._gemm(0, 0, B, self.O, self.H, Z2, B, W3, self.H, Y, B)
        self._bias_act(Y, B, self.O, b3, False)
        self._acts = (X, Z1, Z2, B)
        return Y

    def backward(self, dY):
        """Parameter gradients (into self.grads) for the output gradient dY
        (B x O) of the last forward call; returns nothing."""
        torch = self.torch
        X, Z1, Z2, B = self._acts
        W1, b1, W2, b2, W3, b3 = self.params
        gW1, gb1, gW2, gb2, gW3, gb3 = self.grads
        lib, s = tsqr.lib(), self._stream()
        # layer 3: dW3 = Z2^T dY, db3 = colsum(dY), dZ2 = dY W3^T
        self._gemm(1, 0, self.H, self.O, B, Z2, B, dY, B, gW3, self.H)
        tsqr._check("tsqr_mlp_colsum", lib.tsqr_mlp_colsum(self.h, _p(dY), B, self.O, B, _p(gb3), s), self.h)
        dZ2 = torch.empty(B * self.H, device=self.dev)
        self._gemm(0, 1, B, self.H, self.O, dY, B, W3, self.H, dZ2, B)
        tsqr._check("tsqr_mlp_relu_grad", lib.tsqr_mlp_relu_grad(self.h, _p(dZ2), _p(Z2), B, self.H, B, s), self.h)
        # layer 2
        self._gemm(1, 0, self.H, self.H, B, Z1, B, dZ2, B, gW2, self.H)
        tsqr._check("tsqr_mlp_colsum", lib.tsqr_mlp_colsum(self.h, _p(dZ2), B, self.H, B, _p(gb2), s), self.h)
        dZ1 = torch.empty(B * self.H, device=self.dev)
        self._gemm(0, 1, B, self.H, self.H, dZ2, B, W2, self.H, dZ1, B)
        tsqr._check("tsqr_mlp_relu_grad", lib.tsqr_mlp_relu_grad(self.h, _p(dZ1), _p(Z1), B, self.H, B, s), self.h)
        # layer 1
        self._gemm(1, 0, self.F, self.H, B, X, B, dZ1, B, gW1, self.F)
        tsqr._check("tsqr_mlp_colsum", lib.tsqr_mlp_colsum(self.h, _p(dZ1), B, self.H, B, _p(gb1), s), self.h)

    def mse(self, Y, T, B):
        """dY and the device loss for targets T (B x O)."""
        dY = self.torch.empty(B * self.O, device=self.dev)
        st = tsqr.lib().tsqr_mlp_mse(self.h, _p(Y), _p(T), _p(dY), B, self.O, B, _p(self.loss), self._stream())
        tsqr._check("tsqr_mlp_mse", st, self.h)
        return dY

    def step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        for p, g, m, v in zip(self.params, self.grads, self.m, self.v):
            st = tsqr.lib().tsqr_mlp_adam(self.h, _p(p), _p(g), _p(m), _p(v), p.numel(), lr, b1, b2, eps, self.t,
                                          self._stream())
            tsqr._check("tsqr_mlp_adam", st, self.h)

    def train_step(self, X, T, B, lr=1e-3):
        """One Adam step on the batch (X, T); returns the device loss tensor."""
        Y = self.forward(X, B)
        dY = self.mse(Y, T, B)
        self.backward(dY)
        self.step(lr)
        return self.loss


def features(Rt, batch, n, h=None):
    """X (batch x (2n - 1), column-major) of a (batch, n, n) float32 R~ tensor."""
    import torch
    h = h or tsqr.handle(Rt.device.index or 0)
    X = torch.empty(batch * (2 * n - 1), dtype=torch.float32, device=Rt.device)
    st = tsqr.lib().tsqr_surrogate_features(h, _p(Rt), batch, n, _p(X), tsqr._stream_ptr(torch, Rt.device))
    tsqr._check("tsqr_surrogate_features", st, h)
    return X


def targets(R, Rt, batch, n, h=None):
    """T (batch x n, column-major): log(|R(i,i)|/|R~(i,i)|) centered, R a
    (batch, n, n) float64 tensor of the FP64 R factors (column-major [b])."""
    import torch
    h = h or tsqr.handle(Rt.device.index or 0)
    T = torch.empty(batch * n, dtype=torch.float32, device=Rt.device)
    st = tsqr.lib().tsqr_surrogate_targets(h, _p(R), n, _p(Rt), batch, n, _p(T), tsqr._stream_ptr(torch, Rt.device))
    tsqr._check("tsqr_surrogate_targets", st, h)
    return T


def apply(Rt, Y, batch, n, h=None):
    """R~ with row i of instance b scaled by exp(Y(b, i))."""
    import torch
    h = h or tsqr.handle(Rt.device.index or 0)
    out = torch.empty_like(Rt)
    st = tsqr.lib().tsqr_surrogate_apply(h, _p(Rt), _p(Y), batch, n, _p(out), tsqr._stream_ptr(torch, Rt.device))
    tsqr._check("tsqr_surrogate_apply", st, h)
    return out


class Dataset:
    """Features X (F x N) and targets T (n x N) of N training instances, each
    column one instance (the column-major batch x width layout of the
    kernels, transposed), gathered from sampled plans run on generated
    batches."""

    def __init__(self, X, T):
        self.X, self.T = X, T

    @property
    def count(self):
        return self.X.shape[1]

    def minibatch(self, idx):
        """(X, T) of the instances idx, each column-major with ld len(idx)."""
        return self.X[:, idx].contiguous().reshape(-1), self.T[:, idx].contiguous().reshape(-1)


def gather(plan, batches, log10_kappa_max=8.0, seed=0):
    """Run the sampled ``plan`` (a tsqr.MixedPlan over batch x m x n) on
    ``batches`` generated batches (inputs.conditioned_batch_device, seeds
    seed, seed + 1, ...) and keep the features of each R~ and the targets
    from the R of A.  Returns a Dataset."""
    import torch
    from . import inputs
    b, m, n = plan.batch, plan.m, plan.n
    R = torch.empty((b, n, n), dtype=torch.float64, device=plan.dev)
    flags = torch.zeros(b, dtype=torch.int32, device=plan.dev)
    Xs, Ts = [], []
    for k in range(batches):
        A, _ = inputs.conditioned_batch_device(torch, b, m, n, log10_kappa_max, seed + k, plan.dev)
        plan.launch(A, R, flags)
        Rt = plan.rtilde()
        Xs.append(features(Rt, b, n, plan.h).reshape(2 * n - 1, b))
        Ts.append(targets(R, Rt, b, n, plan.h).reshape(n, b))
        del A
    return Dataset(torch.cat(Xs, 1), torch.cat(Ts, 1))


def train(model, data, steps, minibatch=256, lr=1e-3, seed=0, log_every=0):
    """Adam on random minibatches of ``data``; returns the host list of the
    losses at steps 0, log_every, 2 log_every, ... (one synchronization each)
    and the last one."""
    import torch
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    losses = []
    perm, pos = torch.randperm(data.count, generator=g), 0
    for t in range(steps):
        if pos + minibatch > data.count:
            perm, pos = torch.randperm(data.count, generator=g), 0
        idx = perm[pos:pos + minibatch].to(data.X.device)
        pos += minibatch
        X, T = data.minibatch(idx)
        loss = model.train_step(X, T, minibatch, lr)
        if (log_every and t % log_every == 0) or t == steps - 1:
            losses.append(float(loss.item()))
    return losses


def predict_mse(model, data):
    """(mean squared error of the model, of the zero prediction, i.e. of the
    un-learned R~) on all of ``data``, computed by the library's kernels."""
    import torch
    B = data.count
    X = data.X.contiguous().reshape(-1)
    T = data.T.contiguous().reshape(-1)
    Y = model.forward(X, B)
    model.mse(Y, T, B)
    mse_model = float(model.loss.item())
    model.mse(torch.zeros_like(T), T, B)
    mse_zero = float(model.loss.item())
    return mse_model, mse_zero


def learned_launch(model, plan, A, R, flags):
    """The learned preconditioner on the stream: R~ of the sample (the plan's
    FP32 stage), its features, the network, the corrected R~' and the FP64
    correction with R~'.  Returns R~' (device)."""
    b, n = plan.batch, plan.n
    plan.launch_first_stage(A)
    Rt = plan.rtilde()
    Y = model.forward(features(Rt, b, n, plan.h), b)
    Rp = apply(Rt, Y, b, n, plan.h)
    plan.launch_rtilde(A, Rp, R, flags)
    return Rp
