"""Row-sampled evaluation of the linearised space-time form for large grids.
Test infrastructure (see package doc).

For a test function B_i (one unknown row), (J x)_i is the sum over the Gauss
points of the space-time elements in supp B_i of the integrand of the
bilinear form (Section 3.1.1):

  omega [ C_m B_i d_t x_h + sum_l sigma_l d_l B_i d_l x_h + c B_i x_h
          + C_m sum_k tau_k theta d_t^k B_i d_t^k x_h ],

with x_h evaluated from the coefficients of the basis functions that overlap
those elements, and c, theta the low-rank coefficient fields (or a constant c
for the preconditioner operator of Section 3.2).  Nothing here is shared with
the full-grid evaluator: points, basis values and coefficient interpolation
are recomputed per row.
"""
from __future__ import annotations

import numpy as np

from .operators1d import eval_spline, tau_splines
from .splines import bspline_all, breakpoints, greville, gauss_rule


class RowSampler:
    def __init__(self, prob, knots=None):
        if any(getattr(prob, "map_kind", (0, 0, 0))[:prob.d]):
            raise NotImplementedError("row sampling is for the identity geometry")
        d = prob.d
        kn = knots if knots is not None else prob.uniform_knots()
        self.P = prob
        self.d = d
        self.kn = [np.asarray(k, float) for k in kn[:d]] + [prob.T * np.asarray(kn[d], float)]
        self.p = [prob.p_s] * d + [prob.p_t]
        self.n = [len(k) - p - 1 for k, p in zip(self.kn, self.p)]
        self.taus = tau_splines(self.kn[d], prob.p_t)
        self.gs = [greville(self.kn[l], self.p[l]) for l in range(d)]
        self.gt = greville(self.kn[d], self.p[d])[1:]

    def _local(self, l, b):
        """Gauss points/weights of the elements in the support of basis b (dir l)
        and the index range of basis functions non-zero there."""
        kn, p = self.kn[l], self.p[l]
        z = breakpoints(kn)
        lo, hi = kn[b], kn[b + p + 1]
        g, w = gauss_rule(p + 1)
        pts, wts = [], []
        for e in range(len(z) - 1):
            if z[e] >= lo and z[e + 1] <= hi:
                h = z[e + 1] - z[e]
                pts.append(z[e] + h * g)
                wts.append(h * w)
        pts, wts = np.concatenate(pts), np.concatenate(wts)
        j0 = max(b - p, 0)
        j1 = min(b + p, self.n[l] - 1)
        return pts, wts, j0, j1

    def apply_rows(self, x_unk, rows, theta=None, coef=None, coef_const=None):
        """(J x) at the given unknown rows.  theta/coef: (U, s, V) low-rank
        factors on the Greville grid (or None); coef_const: constant reaction."""
        N_s = int(np.prod(self.n[: self.d]))
        return self._rows(np.concatenate([np.zeros(N_s), x_unk]), rows, theta, coef, coef_const, None)

    def residual_rows(self, u_full, w_full, rows, theta=None, f=None):
        """N(u) of eq. (3.4) at the given unknown rows (full vectors u, w with
        their initial layer): the same form with the reaction term replaced by
        the exact ionic current I_ion(u_h, w_h) at the Gauss points, minus the
        source f(xs, t) when given."""
        return self._rows(u_full, rows, theta, None, None, (w_full, f))

    def _rows(self, x_full, rows, theta, coef, coef_const, ionic):
        P, d = self.P, self.d
        N_s = int(np.prod(self.n[:d]))
        shape = [self.n[d]] + [self.n[l] for l in range(d - 1, -1, -1)]
        X = np.asarray(x_full).reshape(shape)
        Wf = np.asarray(ionic[0]).reshape(shape) if ionic is not None else None
        out = np.zeros(len(rows))
        for ri, row in enumerate(rows):
            it, isp = divmod(int(row), N_s)
            bt = it + 1
            idx = []
            r = isp
            for l in range(d):
                idx.append(r % self.n[l])
                r //= self.n[l]
            loc = [self._local(l, idx[l]) for l in range(d)] + [self._local(d, bt)]
            # per-direction basis values on local points: E[l][k] (npts x nloc), and test row
            E, Bi = [], []
            for l in range(d + 1):
                pts, wts, j0, j1 = loc[l]
                b = idx[l] if l < d else bt
                nd = 1 if l < d else P.p_t
                Em = [bspline_all(self.kn[l], self.p[l], pts, k)[:, j0:j1 + 1] for k in range(nd + 1)]
                E.append(Em)
                Bi.append([Em[k][:, b - j0] for k in range(nd + 1)])
            # local coefficient block, axes (t, x_d, ..., x_1)
            sl = [slice(loc[d][2], loc[d][3] + 1)] + [slice(loc[l][2], loc[l][3] + 1) for l in range(d - 1, -1, -1)]
            Xl = X[tuple(sl)]

            def field(ders, src=None):   # ders[l]: derivative order per direction
                F = Xl if src is None else src
                for a, l in enumerate([d] + list(range(d - 1, -1, -1))):
                    F = np.moveaxis(np.tensordot(E[l][ders[l]], F, axes=([1], [a])), 0, a)
                return F

            def test(ders):
                T = Bi[d][ders[d]]
                for l in range(d - 1, -1, -1):
                    T = np.multiply.outer(T, Bi[l][ders[l]])
                return T

            W = loc[d][1]
            for l in range(d - 1, -1, -1):
                W = np.multiply.outer(W, loc[l][1])
            z0 = [0] * (d + 1)
            dt1 = z0.copy(); dt1[d] = 1
            acc = P.Cm * np.sum(W * test(z0) * field(dt1))
            for l in range(d):
                dl = z0.copy(); dl[l] = 1
                acc += P.sigma[l] * np.sum(W * test(dl) * field(dl))
            # coefficient fields at local points
            def lowrank_field(f):
                U, s, V = f
                tp = loc[d][0]
                out_f = 0.0
                for rr in range(len(s)):
                    tf = np.interp(tp, self.gt, U[:, rr])
                    Vr = V[:, rr].reshape([self.n[l] for l in range(d - 1, -1, -1)])
                    for a, l in enumerate(range(d - 1, -1, -1)):
                        Hl = np.stack([np.interp(loc[l][0], self.gs[l], e) for e in np.eye(self.n[l])], axis=1)
                        Vr = np.moveaxis(np.tensordot(Hl, Vr, axes=([1], [a])), 0, a)
                    out_f = out_f + s[rr] * np.multiply.outer(tf, Vr)
                return out_f
            if ionic is not None:
                uh, wh = field(z0), field(z0, Wf[tuple(sl)])
                g = P.c1 * uh * (uh - P.a) * (uh - 1.0) + P.c2 * uh * wh
                if ionic[1] is not None:
                    grids = np.meshgrid(*([loc[d][0]] + [loc[l][0] for l in range(d - 1, -1, -1)]), indexing="ij")
                    g = g - ionic[1]([grids[d - l] for l in range(d)], grids[0])
                acc += np.sum(W * g * test(z0))
            else:
                if coef_const is not None:
                    cf = coef_const
                elif coef is not None and len(coef[1]):
                    cf = lowrank_field(coef)
                else:
                    cf = 0.0
                acc += np.sum(W * cf * test(z0) * field(z0))
            if theta is not None and len(theta[1]):
                th = lowrank_field(theta)
                tq = loc[d][0]
                for k in range(1, P.p_t + 1):
                    kk, q, c = self.taus[k - 1]
                    tau = eval_spline(kk, q, c, tq)
                    dk = z0.copy(); dk[d] = k
                    tauf = tau.reshape([-1] + [1] * d)
                    acc += P.Cm * np.sum(W * tauf * th * test(dk) * field(dk))
            out[ri] = acc
        return out
