"""Training of LDBP on the GPU (Sec. IV-B, IV-C) with data from the GPU split-step channel.

Every iteration draws a batch with the library's own kernels -- Philox symbols and amplifier
noise, RRC transmitter, split-step channel with amplifiers, low-pass + decimation -- then runs the
LDBP forward (with block checkpoints), the receiver MSE after matched filter and genie phase, the
hand-written adjoints (receiver, then LDBP) and an Adam step on the taps and Kerr coefficients.
The training power of each waveform is drawn uniformly from a power set (Sec. IV-B).

Progressive pruning (Sec. IV-C): filters start with ``t_init`` taps and lose their outermost
symmetric pair at scheduled iterations until they have ``t_final`` (or, with ``t_final_alt``, until
even-numbered layers have ``t_final`` and odd-numbered ones ``t_final_alt``, the alternating 5/3-tap
model of Sec. V-A).  Symbols are 16-QAM or, with ``symbols = "gauss"``, the i.i.d. circularly-symmetric
Gaussian symbols of the paper's simulations (Table I).  Events go round-robin over
the layers; event e of E fires at iteration floor(prune_frac * iters * (e/E)^2), so more taps go
early.  A pruned pair is removed from the packed filters (equivalent to a zero mask on it) so the
kernels stop paying for it.

With ``essm_kappa >= 0`` the model is the generalised enhanced SSM (Sec. III-D): every nonlinear
step filters the power with a real filter of 2 kappa + 1 taps before the phase, the filters start as
unit filters and train with the rest; ``essm_shared`` ties them to one filter applied in every step
(the conventional ESSM, whose gradient is the sum of the per-step filter gradients), and
``train_taps = False`` keeps the linear steps at their initialisation.

Batches are a pure function of (seed, iteration) -- with ``data_pool`` > 0, of (seed, iteration mod
data_pool), a fixed training set of that many batches for configurations whose channel simulation
would dominate every iteration -- so a run resumed from a checkpoint continues bit for bit like an
uninterrupted one.
"""
from __future__ import annotations

import json
import math
from dataclasses import asdict, dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import essm as E
from . import init as I
from . import ldbp as L
from . import ssm as SS
from . import txrx as TX


@dataclass
class TrainConfig:
    nwave: int = 32
    nsym: int = 8192
    rho_a: int = 4
    rho_d: int = 2
    rs: float = 10.7e9
    rolloff: float = 0.1
    nspan: int = 10
    span_km: float = 100.0
    channel_steps: int = 100          # uniform steps per span in the channel simulation
    ldbp_steps: int = 5               # LDBP layers per span (log step sizes)
    t_init: int = 25
    t_final: int = 3
    iters: int = 5000
    prune_frac: float = 0.2           # pruning events fall in the first prune_frac of the iterations
    lr: float = 1e-3
    lr_schedule: str = "constant"     # "cosine": after the last pruning event, decay to lr_final by a half cosine
    lr_final: float = 1e-4
    powers_dbm: Sequence[float] = (2.0, 3.0, 4.0)
    alpha_db_km: float = 0.2
    beta2_ps2_km: float = -21.683
    gamma_w_km: float = 1.3
    nf_db: float = 5.0
    npol: int = 1
    symmetric: bool = True
    train_c: bool = True
    ckpt_every: int = 2
    seed: int = 301
    complex128: bool = False
    unit_init: bool = False
    random_init: bool = False         # random filters (normalised) instead of least squares
    init_method: str = "inband"       # least-squares design: "inband", "full" or "multiobjective"
    ssm: str = "asymmetric"           # "symmetric": l = M + 1 with merged half-steps, last step linear
    train_taps: bool = True
    essm_kappa: int = -1              # >= 0: filtered nonlinear steps with 2 kappa + 1 real taps
    essm_shared: bool = False         # one filter in every nonlinear step (conventional ESSM)
    symbols: str = "qam16"            # "qam16", or "gauss": i.i.d. circularly-symmetric Gaussian symbols
    t_final_alt: int = 0              # > 0: odd-numbered layers prune to this length instead of t_final
    peak_normalise: bool = False      # scale every initial filter to unit peak gain (non-expansive cascade)
    data_pool: int = 0                # > 0: training batches cycle through this many fixed batches
    tie_spans: bool = False           # one span's filters and coefficients shared by every span
    channel_group: int = 4            # training batches simulated by one channel call (same data)


def pruning_plan(t_init: Sequence[int], t_final: Sequence[int], iters: int, frac: float):
    """(iteration, layer) pairs: round-robin over layers, front-loaded quadratic timing."""
    cur = list(t_init)
    layers = []
    while any(c > f for c, f in zip(cur, t_final)):
        for i in range(len(cur)):
            if cur[i] > t_final[i]:
                cur[i] -= 2
                layers.append(i)
    E = len(layers)
    when = [int(math.floor(frac * iters * ((e + 1) / E) ** 2)) for e in range(E)]
    return list(zip(when, layers))


class Trainer:
    def __init__(self, cfg: TrainConfig, device="cuda:0"):
        self.cfg = cfg
        self.dev = torch.device(device)
        self.cdt = torch.complex128 if cfg.complex128 else torch.complex64
        self.rdt = torch.float64 if cfg.complex128 else torch.float32
        self.alpha = I.db_per_km_to_alpha(cfg.alpha_db_km)
        self.beta2 = I.ps2_per_km_to_beta2(cfg.beta2_ps2_km)
        self.gamma = cfg.gamma_w_km / 1e3
        self.span = cfg.span_km * 1e3
        self.kerr_scale = 8.0 / 9.0 if cfg.npol == 2 else 1.0
        self.fs_a = cfg.rho_a * cfg.rs
        self.fs_d = cfg.rho_d * cfg.rs
        self.n_a = cfg.rho_a * cfg.nsym
        self.n_d = cfg.rho_d * cfg.nsym
        self.channel = SS.Link(fs=self.fs_a, alpha=self.alpha, beta2=self.beta2, gamma=self.gamma,
                               span_len=self.span, nspan=cfg.nspan, nstep=cfg.channel_steps, edfa_gain=True,
                               ase_var=I.ase_variance(self.alpha, self.span, cfg.nf_db, self.fs_a),
                               kerr_scale=self.kerr_scale)
        if cfg.ssm == "symmetric":
            taps, c = I.ldbp_parameters_symmetric(self.span, cfg.nspan, cfg.ldbp_steps, cfg.t_init, self.fs_d,
                                                  self.alpha, self.beta2, self.gamma, kerr_scale=self.kerr_scale,
                                                  method="inband" if cfg.init_method == "multiobjective"
                                                  else cfg.init_method)
        else:
            taps, c = I.ldbp_parameters(self.span, cfg.nspan, cfg.ldbp_steps, cfg.t_init, self.fs_d, self.alpha,
                                        self.beta2, self.gamma, kerr_scale=self.kerr_scale, unit_taps=cfg.unit_init,
                                        random_seed=cfg.seed if cfg.random_init else None, method=cfg.init_method)
        if cfg.random_init and cfg.symmetric:
            raise ValueError("random filters are not symmetric: use symmetric=False with random_init")
        self.reps = 1
        if cfg.tie_spans:
            # every span of the backpropagation is the same operation (same step lengths and positions
            # in the span), so one span's ldbp_steps layers serve all spans; their gradient is the sum
            # over the copies
            if cfg.ssm != "asymmetric" or cfg.essm_kappa >= 0 or cfg.t_final != cfg.t_init:
                raise ValueError("tie_spans needs the asymmetric LDBP model without pruning")
            self.reps = cfg.nspan
            taps, c = taps[:cfg.ldbp_steps], c[:cfg.ldbp_steps]
        if cfg.peak_normalise:
            # least-squares filters whose gain exceeds one outside the signal band expand the out-of-band
            # noise at every step; over many short steps the cascade blows up unless each is non-expansive
            taps = [I.unit_peak_gain(h) for h in taps]
        if cfg.symmetric:
            # the least-squares fit of an even response is symmetric up to rounding; make it exact, since
            # the folded kernels read only one side of each filter
            taps = [0.5 * (h + h[::-1]) for h in taps]
        self.ntap = [len(h) for h in taps]
        self.taps = torch.from_numpy(np.concatenate(taps)).to(self.dev, self.cdt)
        self.c = torch.from_numpy(c).to(self.dev, self.rdt)
        self.m_t = torch.zeros(2 * self.taps.numel(), dtype=self.rdt, device=self.dev)
        self.v_t = torch.zeros_like(self.m_t)
        self.m_c = torch.zeros_like(self.c)
        self.v_c = torch.zeros_like(self.c)
        # symmetric SSM: the last step is linear only, its coefficient stays 0
        self.c_mask = None
        if cfg.ssm == "symmetric":
            self.c_mask = torch.ones_like(self.c)
            self.c_mask[-1] = 0
        self.essm = cfg.essm_kappa >= 0
        if self.essm:
            ne = 2 * cfg.essm_kappa + 1
            self.nl_ntap = [ne] * len(self.ntap)
            unit = torch.zeros(ne, dtype=self.rdt, device=self.dev)
            unit[cfg.essm_kappa] = 1.0
            self.eta = unit if cfg.essm_shared else unit.repeat(len(self.ntap))
            self.m_e = torch.zeros_like(self.eta)
            self.v_e = torch.zeros_like(self.eta)
        self.t = 0
        self.it = 0
        targets = [cfg.t_final if (i % 2 == 0 or cfg.t_final_alt <= 0) else cfg.t_final_alt
                   for i in range(len(self.ntap))]
        self.plan = pruning_plan(self.ntap, targets, cfg.iters, cfg.prune_frac) \
            if any(t < cfg.t_init for t in targets) else []
        self.events_done = 0
        self._mirror = None
        self._pool = {}
        self._group, self._group_at = None, -1   # batches simulated together (channel_group)
        self._history: List[dict] = []
        self._pending = []   # (iteration, loss on the GPU, taps) not yet copied to the host

    # ------------------------------------------------------------------ data
    def powers(self, it: int) -> torch.Tensor:
        g = np.random.Generator(np.random.PCG64([self.cfg.seed, it, 7]))
        p = g.choice(np.asarray(self.cfg.powers_dbm, dtype=np.float64), size=self.cfg.nwave)
        return torch.from_numpy(10.0 ** (p / 10.0 - 3.0)).to(self.dev)

    def batch(self, it: int, p_watt: Optional[torch.Tensor] = None):
        """Received waveforms r [nwave, n_d(, 2)], transmitted symbols, powers: a function of (seed, it)."""
        cfg = self.cfg
        p = self.powers(it) if p_watt is None else p_watt
        shape = (cfg.nwave, cfg.nsym) if cfg.npol == 1 else (cfg.nwave, cfg.nsym, 2)
        if cfg.symbols == "gauss":
            s = TX.randn(shape, cfg.seed, 2 * it, dtype=self.cdt, device=self.dev)
            x = TX.tx_shape_symbols(s, p, cfg.rho_a, cfg.rs, cfg.rolloff, npol=cfg.npol)
        else:
            words = TX.randbits(int(np.prod(shape)), cfg.seed, 2 * it, device=self.dev).view(shape)
            x = TX.tx_shape(words, p, cfg.rho_a, cfg.rs, cfg.rolloff, npol=cfg.npol, dtype=self.cdt)
        noise = TX.randn((cfg.nspan,) + tuple(x.shape), cfg.seed, 2 * it + 1, dtype=self.cdt, device=self.dev)
        y = SS.ssm_channel(x, self.channel, noise=noise, npol=cfg.npol, y=x)
        del noise
        r = TX.rx_lpf_decimate(y, self.n_d, npol=cfg.npol)
        if cfg.symbols != "gauss":
            s = TX.qam16_symbols(words, dtype=self.cdt)
        return r, s, p

    def batches(self, its: Sequence[int]):
        """batch(it) for every it of `its`, their channel simulations run as one call over all their
        waveforms (the split-step kernels treat every waveform alike, so each batch is bit for bit the
        one batch(it) returns; one call over several batches keeps more of the GPU busy)."""
        cfg = self.cfg
        if len(its) == 1:
            return [self.batch(its[0])]
        shape = (cfg.nwave, cfg.nsym) if cfg.npol == 1 else (cfg.nwave, cfg.nsym, 2)
        xs, noises, syms, ps = [], [], [], []
        for it in its:
            p = self.powers(it)
            if cfg.symbols == "gauss":
                s = TX.randn(shape, cfg.seed, 2 * it, dtype=self.cdt, device=self.dev)
                xs.append(TX.tx_shape_symbols(s, p, cfg.rho_a, cfg.rs, cfg.rolloff, npol=cfg.npol))
            else:
                words = TX.randbits(int(np.prod(shape)), cfg.seed, 2 * it, device=self.dev).view(shape)
                xs.append(TX.tx_shape(words, p, cfg.rho_a, cfg.rs, cfg.rolloff, npol=cfg.npol, dtype=self.cdt))
                s = TX.qam16_symbols(words, dtype=self.cdt)
            noises.append(TX.randn((cfg.nspan,) + tuple(xs[-1].shape), cfg.seed, 2 * it + 1, dtype=self.cdt,
                                   device=self.dev))
            syms.append(s)
            ps.append(p)
        x = torch.cat(xs, 0)
        noise = torch.stack(noises, 1).reshape((cfg.nspan, x.shape[0]) + tuple(x.shape[1:]))
        del xs, noises
        y = SS.ssm_channel(x, self.channel, noise=noise, npol=cfg.npol, y=x)
        del noise
        r = TX.rx_lpf_decimate(y, self.n_d, npol=cfg.npol)
        return [(r[k * cfg.nwave:(k + 1) * cfg.nwave], syms[k], ps[k]) for k in range(len(its))]

    def train_batch(self, it: int):
        """The batch of training iteration `it`: batch(it) (simulated `channel_group` iterations at a
        time), or with a data pool the pool's batch it mod data_pool, simulated once and kept on the GPU."""
        if self.cfg.data_pool <= 0:
            G = max(1, self.cfg.channel_group)
            g0 = it - it % G
            if self._group_at != g0:
                self._group = self.batches(list(range(g0, g0 + G)))
                self._group_at = g0
            return self._group[it - g0]
        k = it % self.cfg.data_pool
        if k not in self._pool:
            self._pool[k] = self.batch(k)
        return self._pool[k]

    # ------------------------------------------------------------------ model
    def mirror(self) -> torch.Tensor:
        if self._mirror is None:
            mir, off = [], 0
            for T in self.ntap:
                mir.extend(off + T - 1 - j for j in range(T))
                off += T
            self._mirror = torch.tensor(mir, dtype=torch.int32, device=self.dev)
        return self._mirror

    def _prune(self, layer: int):
        """Removes the outermost pair of filter `layer` from the packed taps and the Adam moments."""
        keep, off = [], 0
        for i, T in enumerate(self.ntap):
            if i == layer:
                keep.extend(range(off + 1, off + T - 1))
            else:
                keep.extend(range(off, off + T))
            off += T
        idx = torch.tensor(keep, dtype=torch.int64, device=self.dev)
        self.taps = self.taps.index_select(0, idx).contiguous()
        self.m_t = self.m_t.view(-1, 2).index_select(0, idx).reshape(-1).contiguous()
        self.v_t = self.v_t.view(-1, 2).index_select(0, idx).reshape(-1).contiguous()
        self.ntap[layer] -= 2
        self._mirror = None

    def eta_per_step(self) -> torch.Tensor:
        """The filters of the nonlinear steps back to back (the shared one repeated in every step)."""
        return self.eta.repeat(len(self.ntap)) if self.cfg.essm_shared else self.eta

    def model_taps(self) -> torch.Tensor:
        """Packed taps of every layer of the model (the span's taps repeated when spans are tied)."""
        return self.taps.repeat(self.reps) if self.reps > 1 else self.taps

    def model_c(self) -> torch.Tensor:
        return self.c.repeat(self.reps) if self.reps > 1 else self.c

    def model_ntap(self) -> List[int]:
        return list(self.ntap) * self.reps

    def _fwd(self, r, **kw):
        if self.essm:
            return E.essm_forward(r, self.taps, self.c, self.eta_per_step(), self.ntap, self.nl_ntap,
                                  npol=self.cfg.npol, **kw)
        return L.ldbp_forward(r, self.model_taps(), self.model_c(), self.model_ntap(), npol=self.cfg.npol, **kw)

    def forward(self, r: torch.Tensor, ckpt: bool = False):
        cfg = self.cfg
        sym = 1 if cfg.symmetric else 0
        if not ckpt:
            return self._fwd(r, plan=(0, 0, 0, sym)), None
        S = max(1, min(cfg.ckpt_every, len(self.ntap) * self.reps))
        nslot = L.num_checkpoints(len(self.ntap) * self.reps, S)
        ck = torch.empty((nslot,) + tuple(r.shape), dtype=r.dtype, device=r.device) if nslot else None
        z = self._fwd(r, ckpt=ck, ckpt_every=S if ck is not None else 0,
                      plan=(S, 0, 0, sym) if ck is None else (0, 0, 0, sym))
        return z, ck

    def learning_rate(self, it: int) -> float:
        """Adam step size at iteration `it` (constant, or a half-cosine decay from the last pruning event
        to the end of training)."""
        cfg = self.cfg
        if cfg.lr_schedule != "cosine":
            return cfg.lr
        t0 = self.plan[-1][0] if self.plan else 0
        if it < t0 or cfg.iters <= t0:
            return cfg.lr
        f = min(1.0, (it - t0) / (cfg.iters - t0))
        return cfg.lr_final + 0.5 * (cfg.lr - cfg.lr_final) * (1.0 + math.cos(math.pi * f))

    @property
    def history(self) -> List[dict]:
        """{"it", "loss", "taps"} per training iteration (losses copied from the GPU in groups)."""
        self._flush()
        return self._history

    def _flush(self):
        if self._pending:
            vals = torch.stack([v for _, v, _ in self._pending]).cpu().tolist()   # one synchronisation
            for (it, _, nt), v in zip(self._pending, vals):
                self._history.append({"it": it, "loss": float(v), "taps": nt})
            self._pending = []

    def step(self, sync: bool = True):
        """One training iteration; returns the batch loss (mean MSE over frames): a float (sync=True), or
        without synchronising the GPU, the loss as a device scalar (sync=False)."""
        cfg = self.cfg
        while self.events_done < len(self.plan) and self.plan[self.events_done][0] <= self.it:
            self._prune(self.plan[self.events_done][1])
            self.events_done += 1
        r, s, p = self.train_batch(self.it)
        z, ck = self.forward(r, ckpt=True)
        S = max(1, min(cfg.ckpt_every, len(self.ntap) * self.reps))
        mse, _, gz = TX.rx_mse(z, s, p, cfg.rho_d, cfg.rs, cfg.rolloff, npol=cfg.npol, want_grad=True)
        if self.essm:
            _, gt, gc, ge = E.essm_backward(r, self.taps, self.c, self.eta_per_step(), self.ntap, self.nl_ntap, gz,
                                            npol=cfg.npol, ckpt=ck, ckpt_every=S, need_gx=False,
                                            symmetric=cfg.symmetric)
            if cfg.essm_shared:
                ge = TX.sum_rows(ge, len(self.ntap))
        else:
            _, gt, gc = L.ldbp_backward(r, self.model_taps(), self.model_c(), self.model_ntap(), gz, npol=cfg.npol,
                                        ckpt=ck, ckpt_every=S, need_gx=False, symmetric=cfg.symmetric)
            if self.reps > 1:
                gt, gc = TX.sum_rows(gt, self.reps), TX.sum_rows(gc, self.reps)
        self.t += 1
        lr = self.learning_rate(self.it)
        if cfg.train_taps:
            TX.adam_(self.taps, gt, self.m_t, self.v_t, self.t, lr=lr,
                     mirror=self.mirror() if cfg.symmetric else None)
        if cfg.train_c:
            TX.adam_(self.c, gc, self.m_c, self.v_c, self.t, lr=lr, mask=self.c_mask)
        if self.essm:
            TX.adam_(self.eta, ge, self.m_e, self.v_e, self.t, lr=lr)
        loss = mse.mean()
        self._pending.append((self.it, loss, int(sum(self.ntap)) * self.reps))
        if len(self._pending) >= 256:
            self._flush()
        self.it += 1
        if sync:
            self._flush()
            return self._history[-1]["loss"]
        return loss

    def train(self, iters: Optional[int] = None, log=None):
        n = self.cfg.iters - self.it if iters is None else iters
        for _ in range(n):
            self.step(sync=log is not None)
            if log is not None:
                log.write(json.dumps(self._history[-1]) + "\n")
        return self.history

    # ------------------------------------------------------------------ evaluation
    def evaluate(self, nbatch: int = 4, p_dbm: Optional[float] = None, offset: int = 1_000_000):
        """Effective SNR [dB] (symbols / total squared error) of LDBP on held-out batches."""
        err, cnt = 0.0, 0
        for b in range(nbatch):
            p = None if p_dbm is None else torch.full((self.cfg.nwave,), I.dbm_to_w(p_dbm), dtype=torch.float64,
                                                      device=self.dev)
            r, s, pp = self.batch(offset + b, p)
            z, _ = self.forward(r)
            mse, _, _ = TX.rx_mse(z, s, pp, self.cfg.rho_d, self.cfg.rs, self.cfg.rolloff, npol=self.cfg.npol)
            err += float(mse.sum().item())
            cnt += mse.numel()
        return 10.0 * math.log10(cnt / err)

    def dbp_link(self, steps_per_span: int, log_steps: bool = True) -> SS.Link:
        steps = I.log_step_sizes(self.span, steps_per_span, self.alpha) if log_steps else None
        return SS.Link(fs=self.fs_d, alpha=self.alpha, beta2=self.beta2, gamma=self.gamma, span_len=self.span,
                       nspan=self.cfg.nspan, nstep=steps_per_span, step_len=steps, edfa_gain=True,
                       kerr_scale=self.kerr_scale)

    def evaluate_fft_dbp(self, steps_per_span: int, nbatch: int = 4, p_dbm: Optional[float] = None,
                         offset: int = 1_000_000, gamma_zero: bool = False):
        link = self.dbp_link(steps_per_span)
        if gamma_zero:
            link.gamma = 0.0
        err, cnt = 0.0, 0
        for b in range(nbatch):
            p = None if p_dbm is None else torch.full((self.cfg.nwave,), I.dbm_to_w(p_dbm), dtype=torch.float64,
                                                      device=self.dev)
            r, s, pp = self.batch(offset + b, p)
            z = SS.fft_dbp(r, link, npol=self.cfg.npol)
            mse, _, _ = TX.rx_mse(z, s, pp, self.cfg.rho_d, self.cfg.rs, self.cfg.rolloff, npol=self.cfg.npol)
            err += float(mse.sum().item())
            cnt += mse.numel()
        return 10.0 * math.log10(cnt / err)

    # ------------------------------------------------------------------ checkpoints
    def state_dict(self):
        st = {"cfg": asdict(self.cfg), "taps": self.taps.cpu(), "c": self.c.cpu(), "ntap": list(self.ntap),
              "m_t": self.m_t.cpu(), "v_t": self.v_t.cpu(), "m_c": self.m_c.cpu(), "v_c": self.v_c.cpu(),
              "t": self.t, "it": self.it, "events_done": self.events_done}
        if self.essm:
            st.update(eta=self.eta.cpu(), m_e=self.m_e.cpu(), v_e=self.v_e.cpu())
        return st

    def load_state_dict(self, st):
        self.taps = st["taps"].to(self.dev)
        self.c = st["c"].to(self.dev)
        self.ntap = [int(t) for t in st["ntap"]]
        self.m_t, self.v_t = st["m_t"].to(self.dev), st["v_t"].to(self.dev)
        self.m_c, self.v_c = st["m_c"].to(self.dev), st["v_c"].to(self.dev)
        self.t, self.it, self.events_done = int(st["t"]), int(st["it"]), int(st["events_done"])
        if self.essm:
            self.eta, self.m_e, self.v_e = st["eta"].to(self.dev), st["m_e"].to(self.dev), st["v_e"].to(self.dev)
        self._mirror = None

    def save(self, path: str):
        torch.save(self.state_dict(), path)

    def load(self, path: str):
        self.load_state_dict(torch.load(path, weights_only=True))
