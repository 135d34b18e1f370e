"""Surrogate screening with the simulator as arbiter and fallback.

* ``Pool``: a population of robots stepped together as one batched simulation; one rollout
  draw sets every robot's actuation (phases, amplitudes), restarts from the rest state, runs
  the rollout and reads each robot's centre-of-mass displacement from the FP64 diagnostics.
* ``Surrogate``: the MFMA perceptron trained on (features -> displacement), with the inputs
  and targets standardised by training statistics; flags candidates whose features fall
  outside the training range (out of distribution), which are then simulated, not predicted.
* ``screen``: rank candidates by predicted forward (x) displacement; the top-k and the flagged
  candidates go to the simulator, whose result is final.

Marshalling and bookkeeping only: features, rollouts, training and prediction all run in the
native library.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

import workloads as W

from . import cronos as CR
from . import problem as PR


class Pool:
    def __init__(self, n_robots: int, seed: int = 4, steps: int = 5000, first_robot: int = 0, stream=None,
                 lo: int = 500, hi: int = 50_000, tune_steps: int = 0):
        self.workload = W.population(n_robots, seed=seed, lo=lo, hi=hi, first_robot=first_robot)
        self.workload = dataclasses.replace(self.workload, steps=steps)
        self.seed, self.steps, self.n = seed, steps, n_robots
        self.first_robot = first_robot
        self.sim, self.lat, self.x0 = PR.create(self.workload, stream=stream, tune_steps=tune_steps)
        self.com0 = np.array([d["com"] for d in CR.cronos_diagnostics(self.sim)])
        self.sim_seconds = 0.0
        self.rollouts_done = 0

    def actuation(self, draw: int):
        return W.population_actuation(self.seed, self.n, W.POP_GROUPS, draw=draw, first_robot=self.first_robot)

    def features(self, phase, amp) -> np.ndarray:
        w = self.workload
        return CR.cronos_features(w.bodies, w.material_k, w.spacing, W.POP_GROUPS, phase, amp)

    def rollout(self, phase, amp) -> np.ndarray:
        """Centre-of-mass displacement [n_robots][3] after `steps` steps with this actuation."""
        CR.cronos_set_state(self.sim, self.x0, np.zeros_like(self.x0), 0)
        CR.cronos_set_actuation(self.sim, phase, amp, self.workload.freq_hz)
        t0 = time.perf_counter()
        CR.cronos_step(self.sim, self.steps)
        diags = CR.cronos_diagnostics(self.sim)      # blocks until the rollout is done
        self.sim_seconds += time.perf_counter() - t0
        self.rollouts_done += self.n
        return np.array([d["com"] for d in diags]) - self.com0

    def draw(self, draw: int):
        ph, am = self.actuation(draw)
        return self.features(ph, am), self.rollout(ph, am)

    def close(self):
        self.sim.close()


@dataclasses.dataclass
class Standardiser:
    mean: np.ndarray
    std: np.ndarray

    @staticmethod
    def fit(a: np.ndarray) -> "Standardiser":
        std = a.std(axis=0)
        return Standardiser(a.mean(axis=0), np.where(std > 1e-12, std, 1.0))

    def apply(self, a):
        return (a - self.mean) / self.std

    def invert(self, a):
        return a * self.std + self.mean


class Surrogate:
    def __init__(self, X: np.ndarray, D: np.ndarray, epochs: int = 150, batch: int = 1024, lr: float = 2e-3,
                 seed: int = 4, max_rows: int = 4096, width: int = 768, lr_final: float = 0.0):
        """width: hidden layer width (three hidden layers); lr_final: end of the cosine
        learning-rate schedule (None: constant lr)."""
        self.xs, self.ds = Standardiser.fit(X), Standardiser.fit(D)
        Xn = self.xs.apply(X)
        self.lo, self.hi = Xn.min(axis=0), Xn.max(axis=0)
        sizes = (X.shape[1], width, width, width, D.shape[1])
        self.net = CR.cronos_mlp_create(W.mlp_init(seed, sizes), max_rows=max_rows)
        self.n_params = sum(sizes[l] * sizes[l + 1] + sizes[l + 1] for l in range(4))
        t0 = time.perf_counter()
        self.train_loss = CR.cronos_mlp_train(self.net, Xn.astype(np.float32), self.ds.apply(D).astype(np.float32),
                                              batch=batch, epochs=epochs, lr=lr, seed=seed, lr_final=lr_final)
        self.train_seconds = time.perf_counter() - t0

    def predict(self, X: np.ndarray) -> np.ndarray:
        y = CR.cronos_mlp_forward(self.net, self.xs.apply(X).astype(np.float32))
        return self.ds.invert(y.astype(np.float64))

    def out_of_distribution(self, X: np.ndarray, margin: float = 0.25) -> np.ndarray:
        Xn = self.xs.apply(X)
        span = self.hi - self.lo
        return ((Xn < self.lo - margin * span) | (Xn > self.hi + margin * span)).any(axis=1)


def rms_relative_error(pred: np.ndarray, true: np.ndarray) -> float:
    """||pred - true||_RMS / ||true||_RMS over candidates (vectors of displacement)."""
    return float(np.sqrt(((pred - true) ** 2).sum(axis=1).mean()) / np.sqrt((true ** 2).sum(axis=1).mean()))


def screen(pred: np.ndarray, flagged: np.ndarray, top_k: int, axis: int = 0) -> np.ndarray:
    """Indices handed to the simulator: the top_k by predicted displacement along `axis`, plus
    every flagged candidate."""
    order = np.argsort(-pred[:, axis], kind="stable")
    chosen = np.zeros(len(pred), bool)
    chosen[order[:top_k]] = True
    chosen |= flagged
    return np.nonzero(chosen)[0]
