"""Learned refinement predictor: reference side (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Not a method of the paper: a small network decides, for the pairs that enlargement rule (b)
of Sec. 4.2 (eq. HartenLossOfRegularity) would refine, whether the refinement is needed;
rule (a) is untouched. The paper's heuristic stays the judge: after a step, any declined
pair whose new detail still reaches the rule-(b) threshold is a miss; the step is then
redone from t^n with those pairs refined (eq. DetailRatio is the reason the post-step
detail of the pair predicts its children's details). "Parity unpinned" by the paper: this
module is pinned by the closed-form and finite-difference checks of ``tests/``.

Network: 32 inputs (31 used) -> 64 (ReLU) -> 64 (ReLU) -> 1 logit; parameters in one flat
vector, order W1[64][32], b1[64], W2[64][64], b2[64], w3[64], b3.

Features of a candidate pair (l, p) (split cell p of level l, detail (l+1, 2p)): for the five
split cells p-2..p+2 of level l (wrapped or clamped like every stencil) and every population
h, d / (|d| + eps_{l+1}) with d the detail of that cell (0 when the cell is not split), in
order [delta][h]; then (l + 1) / J; zeros up to 32.

Two forward passes:
* ``forward64`` mirrors the training kernels: inputs, weights and the first hidden layer
  rounded to bfloat16 as the matrix-core products take them, everything else in float64;
* ``logits32`` is the in-step decision: bfloat16 weights, float32 inputs, sums taken
  sequentially in float32 (no fused multiply-add), ReLU, decision logit >= 0.
"""

import numpy as np

from . import mr

NIN, H = 32, 64
SIZES = [("W1", (H, NIN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)
MAX_ATTEMPTS = 8  # redos of one step before the plain rule (b) is restored


def unpack(theta):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n]).reshape(shape)
        o += n
    return out


def bf16_round(x):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).reshape(a.shape)


def bf16_bits(x):
    a = bf16_round(x)
    return (a.view(np.uint32) >> 16).astype(np.uint16)


def forward64(theta, X, quantize=True):
    """Logits (float64) for features X (n, 32), bf16 rounding where the kernels round
    (``quantize=False``: plain float64 network, for finite-difference checks)."""
    if quantize:
        P = unpack(np.asarray(theta, dtype=np.float32))
        q = lambda a: bf16_round(a).astype(np.float64)  # noqa: E731
    else:
        P = unpack(np.asarray(theta, dtype=np.float64))
        q = lambda a: np.asarray(a, dtype=np.float64)  # noqa: E731
    Xq = q(X)
    W1 = q(P["W1"])
    W2 = q(P["W2"])
    w3 = q(P["w3"])
    z1 = Xq @ W1.T + P["b1"].astype(np.float64)
    h1 = np.maximum(z1, 0.0)
    h1q = q(h1.astype(np.float32)) if quantize else h1
    z2 = h1q @ W2.T + P["b2"].astype(np.float64)
    h2 = np.maximum(z2, 0.0)
    out = h2 @ w3 + float(P["b3"][0])
    return out, dict(Xq=Xq, W1=W1, W2=W2, w3=w3, z1=z1, h1q=h1q, z2=z2, h2=h2)


def loss_and_grad64(theta, X, y, pos_weight, quantize=True):
    """Mean weighted binary cross-entropy on the logits and its gradient (float64), with the
    gradient of every parameter taken through the bf16-rounded forward values."""
    out, c = forward64(theta, X, quantize)
    y = np.asarray(y, dtype=np.float64)
    n = out.shape[0]
    sig = 1.0 / (1.0 + np.exp(-out))
    log_s = -np.logaddexp(0.0, -out)
    log_1ms = -np.logaddexp(0.0, out)
    loss = float(np.mean(-(pos_weight * y * log_s + (1 - y) * log_1ms)))
    dout = (sig * (pos_weight * y + 1.0 - y) - pos_weight * y) / n
    g = {}
    g["w3"] = c["h2"].T @ dout
    g["b3"] = np.array([dout.sum()])
    dz2 = np.outer(dout, c["w3"]) * (c["z2"] > 0)
    g["W2"] = dz2.T @ c["h1q"]
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ c["W2"]
    dz1 = dh1 * (c["z1"] > 0)
    g["W1"] = dz1.T @ c["Xq"]
    g["b1"] = dz1.sum(0)
    flat = np.concatenate([g[name].ravel() for name, _ in SIZES])
    return loss, flat


def logits32(wbf, X):
    """In-step decision logits: ``wbf`` the parameters as bf16 values (float32 array), X the
    float32 features; sums in float32, inputs 0..NIN-2, hidden units in order."""
    P = unpack(np.asarray(wbf, dtype=np.float32))
    X = np.asarray(X, dtype=np.float32)
    n = X.shape[0]
    h1 = np.empty((n, H), dtype=np.float32)
    for j in range(H):
        acc = np.full(n, P["b1"][j], dtype=np.float32)
        for i in range(NIN - 1):
            acc = (acc + np.float32(P["W1"][j, i]) * X[:, i]).astype(np.float32)
        h1[:, j] = np.maximum(acc, np.float32(0.0))
    h2 = np.empty((n, H), dtype=np.float32)
    for j in range(H):
        acc = np.full(n, P["b2"][j], dtype=np.float32)
        for i in range(H):
            acc = (acc + np.float32(P["W2"][j, i]) * h1[:, i]).astype(np.float32)
        h2[:, j] = np.maximum(acc, np.float32(0.0))
    acc = np.full(n, P["b3"][0], dtype=np.float32)
    for j in range(H):
        acc = (acc + np.float32(P["w3"][j]) * h2[:, j]).astype(np.float32)
    return acc


def pair_details(state, l, p):
    """Signed details d^h of the split cells p (level l) of ``state``, shape (q, len(p))."""
    return mr.details_even(state.F[l + 1], state.F[l], np.asarray(p), state.gamma, state.bc)


def features(state, l, p):
    """Feature rows (len(p), 32) of candidate pairs p at level l (see the module doc)."""
    p = np.asarray(p)
    q = state.sch.q
    n = 1 << l
    eps_l1 = float(np.ldexp(state.eps, l + 1 - state.jmax))
    X = np.zeros((p.size, NIN), dtype=np.float32)
    for di, dl in enumerate(range(-2, 3)):
        c = mr.bc_index(p + dl, n, state.bc)
        sp = state.split[l][c]
        d = np.zeros((q, p.size))
        if sp.any():
            d[:, sp] = pair_details(state, l, c[sp])
        f = d / (np.abs(d) + eps_l1)
        for h in range(q):
            X[:, di * q + h] = f[h].astype(np.float32)
    X[:, 5 * q] = np.float32((l + 1) / state.jmax)
    return X


class LearnedRefinement:
    """Drives an ``AdaptiveMRLBM`` with the predictor in place of rule (b).

    mode "learned": rule (b) pairs with D < gate * threshold go through the network; pairs
    it declines are judged after the step and the step is redone with the misses refined.
    mode "record": plain rule (b); after each step the rule-(b) pairs are returned as
    training samples, labelled 1 when the judge would call a decline a miss (the pair's new
    detail still reaches the rule-(b) threshold).
    """

    def __init__(self, state, wbf=None, gate=8.0, mode="learned"):
        self.s = state
        self.wbf = None if wbf is None else np.asarray(wbf, dtype=np.float32)
        self.gate = float(gate)
        self.mode = mode
        self.misses = 0
        self.redos = 0
        self.samples_X, self.samples_y = [], []

    def _snapshot(self):
        s = self.s
        return ({l: v.copy() for l, v in s.F.items()}, {l: v.copy() for l, v in s.split.items()})

    def _restore(self, snap):
        F, split = snap
        self.s.F = {l: v.copy() for l, v in F.items()}
        self.s.split = {l: v.copy() for l, v in split.items()}

    def _decide(self, keep, D, forced):
        s, J = self.s, self.s.jmax
        plain = s.rule_b(keep, D)
        use, declined = {}, {}
        for l in range(s.jmin, J):
            use[l] = plain[l].copy()
            declined[l] = np.zeros_like(plain[l])
            if self.mode != "learned" or not plain[l].any():
                continue
            thrb = float(np.ldexp(s.eps, s.mu_bar + 1 + (l + 1) - J))
            cand = plain[l] & (D[l] < self.gate * thrb) & ~forced[l]
            p = np.nonzero(cand)[0]
            if p.size:
                acc = logits32(self.wbf, features(s, l, p)) >= 0
                use[l][p[~acc]] = False
                declined[l][p[~acc]] = True
        return plain, use, declined

    def step(self, nsteps=1):
        s = self.s
        J = s.jmax
        for _ in range(int(nsteps)):
            forced = {l: np.zeros(2 ** l, dtype=bool) for l in range(s.jmin, J)}
            snap = self._snapshot()
            attempt = 0
            while True:
                s.project_up()
                D = s.details()
                s.last_D = D
                keep = s.threshold(D)
                plain, use, declined = self._decide(keep, D, forced)
                old_state = self._snapshot() if self.mode == "record" else None
                new = s.grade(s.enlarge(keep, D, rule_b=use))
                s.transfer(new)
                s.collide_leaves()
                s.project_up()
                s.stream()
                s.project_up()
                D2 = s.details()
                if self.mode == "record":
                    self._record(old_state, plain, D2)
                    break
                miss_any = False
                for l in range(s.jmin, J):
                    if not declined[l].any():
                        continue
                    thrb = float(np.ldexp(s.eps, s.mu_bar + 1 + (l + 1) - J))
                    miss = declined[l] & (D2[l] >= thrb)
                    if miss.any():
                        forced[l] |= miss
                        self.misses += int(miss.sum())
                        miss_any = True
                if not miss_any:
                    break
                self.redos += 1
                attempt += 1
                if attempt >= MAX_ATTEMPTS:
                    # every rule-(b) pair forced: the plain rule, which has nothing to miss
                    forced = {l: np.ones(2 ** l, dtype=bool) for l in range(s.jmin, J)}
                self._restore(snap)
            nl = s.n_leaves()
            s.leaf_history.append(nl)
            s.leaf_updates += nl
            s.steps += 1
        return self

    def _record(self, old_state, plain, D2):
        s, J = self.s, self.s.jmax
        cur = self._snapshot()
        self._restore(old_state)
        feats = {}
        for l in range(s.jmin, J):
            p = np.nonzero(plain[l])[0]
            if p.size:
                feats[l] = (p, features(s, l, p))
        self._restore(cur)
        for l, (p, X) in feats.items():
            thrb = float(np.ldexp(s.eps, s.mu_bar + 1 + (l + 1) - J))
            y = (D2[l][p] >= thrb).astype(np.float32)
            self.samples_X.append(X)
            self.samples_y.append(y)
