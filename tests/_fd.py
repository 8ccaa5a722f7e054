"""FP64 helpers for the finite-difference checks of the residual adjoint
(Sec. 3.6, detached target): everything here is host numpy on the oracle's
encodings and the FP32 masters, never on GPU results.

What separates a difference quotient from the derivative. With the target
frozen, the loss is sum_b |L(x_b) - T_b|^2 / (3B). The decoder is linear
layers with ReLU, so along a direction that moves only feature-table entries
(h is linear in the tables) or only one layer's weights, every
pre-activation is affine in the step until a ReLU changes branch; L is then
affine and the loss quadratic, and the central difference equals the
derivative at the midpoint of the two evaluation points. So the quotient
differs from the derivative at theta by exactly
 - kappa: for the queries whose ReLU pattern changes inside the step (found
   from the linearised pre-activations), their exact FP64 quotient minus
   their derivative;
 - the midpoint shift of an asymmetric FP32 step, 2 gamma ((up + dn)/2 - v0)
   with gamma the curvature of the other queries' terms;
which are computed here in FP64 and removed from the GPU's quotient, and
 - nu: the rounding noise of the FP32 radiance in the two loss evaluations,
   which bounds what is left. Each rounding in a query's FP32 evaluation is
   modelled as independent with standard deviation sqrt(n) u S (u = 2^-24,
   n the length of the dot product, S the sum of absolute values of its
   terms), carried to the outputs by the decoder's Jacobian; nu is six
   standard deviations of the difference of the two evaluations over the
   queries the step moves, divided by the step.
"""
import numpy as np

import oracle

U32 = 2.0 ** -24


def forward64(H, W, b):
    """Decoder forward in FP64: hidden pre-activations zs and the output."""
    zs, a = [], H
    for i in range(len(W) - 1):
        z = a @ np.asarray(W[i], np.float64).T + np.asarray(b[i], np.float64)
        zs.append(z)
        a = np.maximum(z, 0.0)
    return zs, a @ np.asarray(W[-1], np.float64).T + np.asarray(b[-1], np.float64)


def output_sigma(H, Habs, zs, W, b, chunk=32768):
    """Per query and output channel, the standard deviation of the FP32
    evaluation error under the model above: 4-term gathers (sum of |w T|
    = Habs), then one dot product per neuron of every layer."""
    Ws = [np.asarray(w, np.float64) for w in W]
    bs = [np.abs(np.asarray(x, np.float64)) for x in b]
    n_out = Ws[-1].shape[0]
    out = np.zeros((H.shape[0], n_out))
    for c0 in range(0, H.shape[0], chunk):
        sl = slice(c0, c0 + chunk)
        acts = [H[sl]] + [np.maximum(z[sl], 0.0) for z in zs]
        var = np.zeros((acts[0].shape[0], n_out))
        # output layer: its own dot products
        S = np.abs(acts[-1]) @ np.abs(Ws[-1]).T + bs[-1]
        var += Ws[-1].shape[1] * S ** 2
        J = np.broadcast_to(Ws[-1][None, :, :], (acts[0].shape[0],) + Ws[-1].shape)  # dL/da_last [n, out, H]
        for i in range(len(Ws) - 2, -1, -1):
            Jz = J * (zs[i][sl] > 0.0)[:, None, :]  # dL/dz_i
            S = np.abs(acts[i]) @ np.abs(Ws[i]).T + bs[i]
            var += Ws[i].shape[1] * np.einsum("noh,nh->no", Jz ** 2, S ** 2)
            J = Jz @ Ws[i]  # dL/da_{i-1}
        var += 4.0 * np.einsum("nok,nk->no", J ** 2, Habs[sl] ** 2)  # the gathers
        out[sl] = U32 * np.sqrt(var)
    return out


def directional(H, zs, W, dH, dW, db):
    """Derivative of every hidden pre-activation and of the output along
    (dH, dW, db) at the current ReLU pattern. dW/db: lists (None = 0)."""
    dzs, a, da = [], H, dH
    for i in range(len(W)):
        Wi = np.asarray(W[i], np.float64)
        dz = da @ Wi.T
        if dW[i] is not None:
            dz = dz + a @ np.asarray(dW[i], np.float64).T
        if db[i] is not None:
            dz = dz + np.asarray(db[i], np.float64)
        if i == len(W) - 1:
            return dzs, dz
        dzs.append(dz)
        a, da = np.maximum(zs[i], 0.0), np.where(zs[i] > 0.0, dz, 0.0)


def kink_distance(zs, dzs):
    """Per query, the step along the direction before the first hidden unit
    changes branch (|z| / |dz| over units that move; inf if none moves)."""
    d = np.full(zs[0].shape[0], np.inf)
    for z, dz in zip(zs, dzs):
        mov = np.abs(dz) > 0.0
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.where(mov, np.abs(z) / np.where(mov, np.abs(dz), 1.0), np.inf)
        d = np.minimum(d, t.min(axis=1))
    return d


def loss_terms(out, T, B):
    """Per-query contribution sum_c (L - T)^2 / (3B)."""
    r = out - T
    return (r * r).sum(axis=1) / (3.0 * B)


def noise_floor(r, sigma, step, B):
    """Six standard deviations of the FP32-rounding noise of the difference
    quotient over the queries the step moves."""
    var = 2.0 * np.sum((2.0 * r * sigma) ** 2)  # two independent evaluations
    return 6.0 * np.sqrt(var) / (3.0 * B) / step


def encode_abs(otree, x, d):
    """The gather with |T| in place of every table entry: sum_k w_k |T_k|."""
    t = oracle.Tree(otree.nodes, otree.level_offset, list(otree.res), otree.C,
                    [np.abs(np.asarray(f, np.float32)) for f in otree.feat])
    return oracle.encode(t, x, d)[0]


class Problem:
    """The FP64 picture of one frozen-target batch: encoding, pre-activations,
    rounding model and residuals of every LHS query."""

    def __init__(self, cfg, otree, W, bias, x, d, T):
        self.cfg, self.otree, self.W, self.bias, self.T = cfg, otree, W, bias, T
        self.x, self.d, self.B = x, d, len(x)
        self.H, self.idx = oracle.encode(otree, x, d)
        self.zs, self.out = forward64(self.H, W, bias)
        self.sigma = output_sigma(self.H, encode_abs(otree, x, d), self.zs, W, bias)
        self.r = self.out - T
        self.st = oracle.octa(d)

    def entry(self, kind, l, flat, v0, h_weight=1e-3, h_feat=0.05):
        """Step and corrections for one table entry ("feat", level, flat
        index) or weight ("W", layer, flat index) whose FP32 value is v0.
        Returns dict(up, dn, shift, nu, moved, kinks, h): the exact FP64
        difference quotient equals the derivative plus `shift`."""
        W, nl, B = self.W, len(self.W), self.B
        dW = [None] * nl
        if kind == "feat":
            R, C_ = self.cfg.res[l], self.cfg.C
            node, tex, c = flat // (R * R * C_), (flat // C_) % (R * R), flat % C_
            sel = np.nonzero(self.idx[:, l] == self.otree.level_offset[l] + node)[0]
            ij, w = oracle.taps(self.st[sel], R)
            wsum = (w * ((ij[:, :, 0] == tex % R) & (ij[:, :, 1] == tex // R))).sum(axis=1)
            sel, wsum = sel[wsum != 0.0], wsum[wsum != 0.0]
            dH = np.zeros((len(sel), self.H.shape[1]))
            dH[:, l * C_ + c] = wsum
            h = h_feat
        else:
            sel = np.arange(B)
            dH = np.zeros((B, self.H.shape[1]))
            dW[l] = np.zeros(np.shape(W[l]))
            dW[l].reshape(-1)[flat] = 1.0
            h = h_weight
        up, dn = float(np.float32(v0 + h)), float(np.float32(v0 - h))
        step = up - dn
        zsel = [z[sel] for z in self.zs]
        dzs, dout = directional(self.H[sel], zsel, W, dH, dW, [None] * nl)
        dist = kink_distance(zsel, dzs) if len(sel) and dzs else np.full(len(sel), np.inf)
        X = np.nonzero(dist <= max(up - v0, v0 - dn) * (1 + 1e-9))[0]
        shift = 0.0
        if len(X):
            ls = []
            for v in (up, dn):
                if kind == "feat":
                    Hx, Wx = self.H[sel[X]] + (v - v0) * dH[X], W
                else:
                    Hx, Wx = self.H[sel[X]], [np.array(w_, np.float64) for w_ in W]
                    Wx[l].reshape(-1)[flat] = v
                ls.append(loss_terms(forward64(Hx, Wx, self.bias)[1], self.T[sel[X]], B).sum())
            gX = (2.0 * self.r[sel[X]] * dout[X]).sum() / (3.0 * B)
            shift += (ls[0] - ls[1]) / step - gX
        keep = np.setdiff1d(np.arange(len(sel)), X)
        gamma = (dout[keep] ** 2).sum() / (3.0 * B)
        shift += 2.0 * gamma * ((up + dn) / 2.0 - v0)
        nu = noise_floor(self.r[sel], self.sigma[sel], step, B)
        return dict(up=up, dn=dn, shift=shift, nu=nu, moved=len(sel), kinks=len(X), h=h)

    def direction(self, v_tables, Pp, Pm, eps):
        """For the tables Pp and Pm (= fl32(theta +- eps v)): the exact FP64
        effect of ReLU branch changes on loss(Pp) - loss(Pm) beyond its
        first-order prediction, and the rounding floor: (shift, nu, kinks)."""
        otree, nl = self.otree, len(self.W)
        vt = oracle.Tree(otree.nodes, otree.level_offset, list(otree.res), otree.C, v_tables)
        dH = oracle.encode(vt, self.x, self.d)[0]
        dzs, dout = directional(self.H, self.zs, self.W, dH, [None] * nl, [None] * nl)
        dist = kink_distance(self.zs, dzs)
        X = np.nonzero(dist <= eps * (1 + 1e-6))[0]
        shift = 0.0
        if len(X):
            tp = oracle.Tree(otree.nodes, otree.level_offset, list(otree.res), otree.C, Pp)
            tm = oracle.Tree(otree.nodes, otree.level_offset, list(otree.res), otree.C, Pm)
            lp = loss_terms(forward64(oracle.encode(tp, self.x[X], self.d[X])[0], self.W, self.bias)[1],
                            self.T[X], self.B)
            lm = loss_terms(forward64(oracle.encode(tm, self.x[X], self.d[X])[0], self.W, self.bias)[1],
                            self.T[X], self.B)
            shift = (lp.sum() - lm.sum()) - (2.0 * self.r[X] * dout[X]).sum() / (3.0 * self.B) * 2.0 * eps
        nu = noise_floor(self.r, self.sigma, 1.0, self.B)
        return shift, nu, len(X)
