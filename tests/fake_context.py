"""A CPU stand-in for paper_1205_2288_amd.Context built on the oracle's arithmetic.

Test infrastructure only: it lets the product's host scheduler (driver.TSBTS) run
without a GPU, so that its era / pass / block-step logic can be compared with the
oracle's own scheduler decision by decision.  Its semantics follow include/tsbts.h:
prediction (Taylor for active particles, Hermite from the finished history in later
passes), force on an active set, corrector with history recording, criterion, energy.
"""
import numpy as np
import torch

import oracle
from oracle import adjoint as oadj


def _np(x):
    return x.detach().cpu().numpy() if isinstance(x, torch.Tensor) else x


class FakeContext:
    def __init__(self, n, eps):
        self.n = n
        self.eps = eps
        self.device = torch.device("cpu")
        self.recording = False
        self.hist = None

    # ------------------------------------------------------------------ plumbing
    def bind(self, r, v, m, a=None, t_last=None, dt=None):
        n = self.n
        f = lambda x, shape: torch.as_tensor(np.array(_np(x), dtype=np.float64)).reshape(shape)  # noqa
        self.r = f(r, (3, n))
        self.v = f(v, (3, n))
        self.m = f(m, (n,))
        self.a = torch.zeros((3, n), dtype=torch.float64) if a is None else f(a, (3, n))
        self.t_last = torch.zeros(n, dtype=torch.float64) if t_last is None else f(t_last, (n,))
        self.dt = torch.zeros(n, dtype=torch.float64) if dt is None else f(dt, (n,))
        return self

    def host_buffer(self, n, dtype):
        return torch.empty(n, dtype=dtype)

    def synchronize(self, stream=None):
        pass

    def idx(self, active):
        return torch.as_tensor(np.asarray(active), dtype=torch.int32).reshape(-1)

    # ------------------------------------------------------------------ entry points
    def predict(self, t_block, use_history=False):
        r, v, a = self.r.numpy(), self.v.numpy(), self.a.numpy()
        tl, dt = self.t_last.numpy(), self.dt.numpy()
        rp, vp = oracle.taylor(r, v, a, t_block - tl)
        active = tl + dt == t_block
        if use_history:
            h = self.hist
            j = np.flatnonzero(~active)
            key = h["pid"] * (1 << 40) + h["tk"]
            k = np.searchsorted(key, j * (1 << 40) + h["tk_of"](t_block), side="right") - 1
            exact = h["t"][k] == t_block
            rp[:, j[exact]] = h["r"][:, k[exact]]
            vp[:, j[exact]] = h["v"][:, k[exact]]
            inner = ~exact & (k + 1 < h["off"][j + 1])
            ji, k0 = j[inner], k[inner]
            k1 = k0 + 1
            rr, vv = oracle.hermite(h["t"][k0], h["r"][:, k0], h["v"][:, k0], h["a"][:, k0],
                                    h["t"][k1], h["r"][:, k1], h["v"][:, k1], h["a"][:, k1],
                                    t_block)
            rp[:, ji] = rr
            vp[:, ji] = vv
        self.pred_r, self.pred_v, self.pred_t = rp, vp, t_block

    def force(self, active, t_block, with_pot=True, acc=None, pot=None):
        assert t_block == self.pred_t
        idx = np.asarray(active, dtype=np.int32)
        a, p = oracle.force(self.pred_r, self.m.numpy(), self.eps, idx)
        if acc is None:
            acc = torch.empty((3, idx.size), dtype=torch.float64)
        acc.copy_(torch.from_numpy(a))
        if with_pot:
            pot = torch.from_numpy(p) if pot is None else pot.copy_(torch.from_numpy(p))
        return acc, pot

    def correct(self, active, t_block, acc_new):
        idx = np.asarray(active, dtype=np.int64)
        an = acc_new.numpy()
        r, v, a, tl = self.r.numpy(), self.v.numpy(), self.a.numpy(), self.t_last.numpy()
        h = t_block - tl[idx]
        r[:, idx] = self.pred_r[:, idx]
        v[:, idx] = v[:, idx] + 0.5 * (a[:, idx] + an) * h
        a[:, idx] = an
        tl[idx] = t_block
        self.pred_v[:, idx] = v[:, idx]
        if self.recording:
            self.records.append((idx.copy(), np.full(idx.size, t_block), r[:, idx].copy(),
                                 v[:, idx].copy(), a[:, idx].copy()))

    def load_positions(self, r, m=None, t_label=0.0):
        self.pred_r = np.array(_np(r), dtype=np.float64).reshape(3, self.n)
        if m is not None:
            self.m = torch.as_tensor(np.array(_np(m), dtype=np.float64)).reshape(self.n)
        self.pred_t = t_label

    def force_backward(self, active, t_block, grad_acc, grad_pot=None, grad_r=None,
                       grad_m=None):
        assert t_block == self.pred_t
        idx = np.asarray(active, dtype=np.int32)
        gp = None if grad_pot is None else torch.as_tensor(grad_pot).numpy()
        gr, gm = oracle.force_backward(self.pred_r, self.m.numpy(), self.eps, idx,
                                       torch.as_tensor(grad_acc).numpy(), gp)
        if grad_r is None:
            grad_r = torch.zeros((3, self.n), dtype=torch.float64)
        if grad_m is None:
            grad_m = torch.zeros(self.n, dtype=torch.float64)
        grad_r += torch.from_numpy(gr)
        grad_m += torch.from_numpy(gm)
        return grad_r, grad_m

    def block_adjoint(self, phase, active, t_block, rbar, vbar, abar, pbar, seeds):
        dt, tl = self.dt.numpy(), self.t_last.numpy()
        rb, vb, ab, pb = (x.numpy() for x in (rbar, vbar, abar, pbar))
        if phase == 0:
            idx = np.asarray(active, dtype=np.int64)
            half = 0.5 * dt[idx]
            seeds.numpy()[...] = ab[:, idx] + half * vb[:, idx]
            pb[...] = 0.0
            pb[:, idx] = rb[:, idx]
            ab[:, idx] = half * vb[:, idx]
            rb[:, idx] = 0.0
        else:
            h = t_block - tl
            rb += pb
            vb += h * pb
            ab += 0.5 * h * h * pb

    def timestep(self, active, eta, dtc=None):
        idx = np.asarray(active, dtype=np.int32)
        d = oracle.timestep(self.pred_r, self.pred_v, self.m.numpy(), self.eps, eta, idx)
        if dtc is None:
            dtc = torch.empty(idx.size, dtype=torch.float64)
        return dtc.copy_(torch.from_numpy(d))

    def set_dt(self, active, dt_new):
        self.dt.numpy()[np.asarray(active, dtype=np.int64)] = np.asarray(dt_new)

    def history_begin(self):
        n = self.n
        self.records = [(np.arange(n), self.t_last.numpy().copy(), self.r.numpy().copy(),
                         self.v.numpy().copy(), self.a.numpy().copy())]
        self.recording = True

    def history_end(self):
        pid = np.concatenate([x[0] for x in self.records])
        order = np.argsort(pid, kind="stable")
        tt = np.concatenate([x[1] for x in self.records])[order]
        self.hist = {
            "pid": pid[order],
            "tk": np.round(tt * 2.0 ** 20).astype(np.int64),
            "tk_of": lambda t: int(round(t * 2.0 ** 20)),
            "t": tt,
            "r": np.concatenate([x[2] for x in self.records], axis=1)[:, order],
            "v": np.concatenate([x[3] for x in self.records], axis=1)[:, order],
            "a": np.concatenate([x[4] for x in self.records], axis=1)[:, order],
            "off": np.concatenate([[0], np.cumsum(np.bincount(pid, minlength=self.n))]),
        }
        self.recording = False

    def history_clear(self):
        self.hist = None
        self.recording = False

    def history_layout(self):
        h = self.hist
        return (h["t"].size, torch.as_tensor(h["off"].astype(np.int32)),
                torch.as_tensor(h["t"].copy()))

    def interp_adjoint(self, t_block, pbar, hbar):
        h = self.hist
        tl, dt = self.t_last.numpy(), self.dt.numpy()
        pb, hb = pbar.numpy(), hbar.numpy()
        for j in np.flatnonzero(tl + dt != t_block):
            lo, hi = h["off"][j], h["off"][j + 1]
            ks = [k for k in range(lo, hi) if h["t"][k] <= t_block]
            k = ks[-1] if ks else lo
            if h["t"][k] == t_block:
                hb[0:3, k] += pb[:, j]
            elif k + 1 < hi:
                w = oadj.hermite_weights(h["t"][k], h["t"][k + 1], t_block)
                hb[0:3, k] += w[0] * pb[:, j]
                hb[3:6, k] += w[1] * pb[:, j]
                hb[0:3, k + 1] += w[2] * pb[:, j]
                hb[3:6, k + 1] += w[3] * pb[:, j]
            else:
                continue
            pb[:, j] = 0.0

    def record_adjoint(self, active, t_block, layout, hbar, rbar, vbar):
        _, off, t = (np.asarray(_np(x)) for x in layout)
        hb, rb, vb = hbar.numpy(), rbar.numpy(), vbar.numpy()
        for i in np.asarray(_np(active), dtype=np.int64):
            for k in range(off[i], off[i + 1]):
                if t[k] == t_block:
                    rb[:, i] += hb[0:3, k]
                    vb[:, i] += hb[3:6, k]

    def adjoint_accumulate(self, rbar, vbar, abar, rbar_acc, vbar_acc, abar_acc):
        rbar_acc += rbar
        vbar_acc += vbar
        abar_acc += abar

    def energy(self, r=None, v=None, m=None, out=None):
        k, w = oracle.energy(self.r.numpy(), self.v.numpy(), self.m.numpy(), self.eps)
        res = torch.tensor([k, w], dtype=torch.float64)
        return res if out is None else out.copy_(res)

    def close(self):
        pass
