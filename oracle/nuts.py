"""Oracle No-U-Turn sampler (test infrastructure only).

Section 3.3 of the paper runs its HMC with the No-U-Turn sampler (NUTS) of
Hoffman & Gelman (JMLR 15, 2014) and tunes the step by their dual averaging.
This module takes the efficient NUTS of that paper with dual averaging in
its own steps and notation, on the Hamiltonian of Section 3.1 (eq:Hamiltonian,
eq:M_ab):

  * momenta r0 ~ N(0, M); slice variable u ~ Uniform[0, exp(-H(theta, r0))];
  * theta- = theta+ = theta, r- = r+ = r0, n = 1, s = 1, j = 0; then while
    s = 1, double the trajectory in a random direction v_j: BuildTree from
    the end on that side with 2^j leapfrog steps of v_j eps;
  * BuildTree (height 0): one leapfrog step to (theta', r'); n' = I[u <=
    exp(-H')], s' = I[u < exp(Delta_max - H')], alpha' = min(1, exp(H0 - H'));
    (height j): the first half, and if its s' = 1 the second half from the
    end reached; the second half's sample replaces the first's with
    probability n''/(n' + n''); s' = s'' I[(theta+ - theta-).r- >= 0]
    I[(theta+ - theta-).r+ >= 0] over the subtree's ends;
  * after a doubling with s' = 1 the chain moves to its sample with
    probability min(1, n'/n); n += n'; s = s' times the same no-U-turn test
    over the whole trajectory;
  * dual averaging on the statistic alpha / n_alpha of all leaves built.

Readings (the paper states none of them):
  * ln u = ln U - H0 with U in (0, 1] from the shared counter-based stream, so
    a leaf is in the slice iff ln U <= H0 - H'; Delta_max = 1000.
  * The no-U-turn test uses the plain dot product (theta+ - theta-).r of the
    independent real coordinates (pair-weighted on the kz = 0 plane): with
    the mass matrix M of eq:M_ab this is Hoffman & Gelman's test after the
    change of variables M^(1/2) theta that makes the mass the identity.
  * At most `max_depth` doublings per iteration (10 by default).
  * "With probability p" is decided as U p_den <= p_num with one uniform U
    from the counter-based stream (purposes NUTS_DIR, NUTS_MERGE, NUTS_TOP):
    v_j = -1 iff U <= 1/2.
  * A leaf whose Hamiltonian is not finite is outside the slice and ends the
    tree (s' = 0); its alpha' is 0.

The sampler is written against a small target interface (gradient, leapfrog
step, kinetic energy, momenta, dot product), so that it can be pinned on
Gaussian targets with known answers as well as run on the posterior.
"""
import math
from dataclasses import dataclass, field

import numpy as np

from . import hmc, philox
from .model import exact_sum, mode_variance, pair_weight

DELTA_MAX = 1000.0


def uniform(seed, iteration, purpose, index):
    """One uniform in (0, 1] of the counter-based stream."""
    w = philox.draw_words(seed, iteration, purpose, np.array([index], dtype=np.uint64))
    return float(philox.uniform53(w[0, 0], w[0, 1]))


def merge_index(doubling, height, position):
    return ((doubling * 16 + height) << 32) | position


# ----------------------------------------------------------------------------
# Targets
# ----------------------------------------------------------------------------

class PosteriorTarget:
    """The posterior of Section 2 with the mass matrix of eq:M_ab."""

    def __init__(self, prob):
        self.prob = prob
        self.w_half = 0.5 * pair_weight(prob.n_grid)

    def gradient(self, q):
        return hmc.gradient(self.prob, q)

    def leapfrog(self, q, p, eps, cached):
        return hmc.leapfrog(self.prob, q, p, eps, 1, cached)

    def kinetic(self, p):
        return hmc.kinetic(self.prob, p)

    def momenta(self, seed, iteration):
        return hmc.draw_momenta(self.prob, seed, iteration)

    def dot(self, q_plus, q_minus, p):
        """(theta+ - theta-) . r over the independent real coordinates."""
        dm = q_plus.modes - q_minus.modes
        terms = [(self.w_half * (dm.real * p.modes.real + dm.imag * p.modes.imag)).ravel()]
        if self.prob.sample_distances:
            terms.append((q_plus.dist - q_minus.dist) * p.dist)
        if self.prob.sample_sigma_nl:
            terms.append([(q_plus.s - q_minus.s) * p.s])
        if self.prob.sample_cosmology:
            terms.append((np.asarray(q_plus.cosmo) - np.asarray(q_minus.cosmo)) * np.asarray(p.cosmo))
        return exact_sum(np.concatenate(terms))


@dataclass
class VecState:
    x: np.ndarray

    def copy(self):
        return VecState(self.x.copy())


class GaussianTarget:
    """Psi(x) = x^T A x / 2 (A = C^-1) with mass matrix diag(1 / minv):
    a target whose distribution is known, for pins of the sampler."""

    def __init__(self, cov, minv):
        self.cov = np.asarray(cov, dtype=float)
        self.prec = np.linalg.inv(self.cov)
        self.minv = np.asarray(minv, dtype=float)

    def gradient(self, q):
        g = self.prec @ q.x
        return (0.5 * float(q.x @ g), g)

    def leapfrog(self, q, p, eps, cached):
        pm = p.x - 0.5 * eps * cached[1]
        x = q.x + eps * self.minv * pm
        c = self.gradient(VecState(x))
        return VecState(x), VecState(pm - 0.5 * eps * c[1]), c

    def kinetic(self, p):
        return 0.5 * float(np.sum(self.minv * p.x * p.x))

    def momenta(self, seed, iteration):
        idx = np.arange(len(self.minv), dtype=np.uint64)
        z, _ = philox.normal_pair(philox.draw_words(seed, iteration, philox.PURPOSE_MODES, idx))
        return VecState(z / np.sqrt(self.minv))

    def dot(self, q_plus, q_minus, p):
        return float((q_plus.x - q_minus.x) @ p.x)


# ----------------------------------------------------------------------------
# The tree
# ----------------------------------------------------------------------------

@dataclass
class Leaf:
    q: object             # coordinates theta
    p: object             # momenta r (synchronised with theta)
    cached: tuple         # (Psi, gradient...) at theta
    where: tuple          # (doubling, position in it) of the leaf; (-1, 0) for the start


@dataclass
class Tree:
    minus: Leaf
    plus: Leaf
    cand: Leaf
    n: int
    s: int
    alpha: float
    n_alpha: int


class _Iteration:
    def __init__(self, target, eps, seed, it, ln_u, h0):
        self.t, self.eps, self.seed, self.it, self.ln_u, self.h0 = target, eps, seed, it, ln_u, h0
        self.leaves = 0

    def no_u_turn(self, minus, plus):
        d1 = self.t.dot(plus.q, minus.q, minus.p)
        d2 = self.t.dot(plus.q, minus.q, plus.p)
        return int(d1 >= 0.0 and d2 >= 0.0)

    def build(self, start, v, height, doubling, position):
        if height == 0:
            q1, p1, c1 = self.t.leapfrog(start.q, start.p, v * self.eps, start.cached)
            self.leaves += 1
            h1 = c1[0] + self.t.kinetic(p1)
            if not math.isfinite(h1):
                h1 = math.inf
            leaf = Leaf(q1, p1, c1, (doubling, position))
            n1 = int(self.ln_u <= -h1)
            s1 = int(self.ln_u < DELTA_MAX - h1)
            alpha = 0.0 if not math.isfinite(h1) else min(1.0, math.exp(self.h0 - h1))
            return Tree(leaf, leaf, leaf, n1, s1, alpha, 1)
        tree = self.build(start, v, height - 1, doubling, 2 * position)
        if tree.s == 1:
            edge = tree.minus if v < 0 else tree.plus
            right = self.build(edge, v, height - 1, doubling, 2 * position + 1)
            if right.n > 0:
                u = uniform(self.seed, self.it, philox.PURPOSE_NUTS_MERGE, merge_index(doubling, height, position))
                if u * (tree.n + right.n) <= right.n:
                    tree.cand = right.cand
            if v < 0:
                tree.minus = right.minus
            else:
                tree.plus = right.plus
            tree.alpha += right.alpha
            tree.n_alpha += right.n_alpha
            tree.s = right.s * self.no_u_turn(tree.minus, tree.plus)
            tree.n += right.n
        return tree


@dataclass
class NutsStep:
    q: object
    cached: tuple
    depth: int            # doublings done
    leaves: int           # leapfrog steps (gradient evaluations)
    alpha: float          # alpha / n_alpha of the iteration
    where: tuple          # (doubling, position) of the new state's leaf; (-1, 0) if it did not move
    h0: float


def nuts_iteration(target, q, cached, eps, seed, it, max_depth=10):
    """One NUTS transition from (q, cached)."""
    r0 = target.momenta(seed, it)
    h0 = cached[0] + target.kinetic(r0)
    u = uniform(seed, it, philox.PURPOSE_ACCEPT, 0)
    ln_u = math.log(u) - h0
    run = _Iteration(target, eps, seed, it, ln_u, h0)
    start = Leaf(q, r0, cached, (-1, 0))
    minus = plus = sample = start
    n, s, j = 1, 1, 0
    alpha, n_alpha = 0.0, 0
    while s == 1 and j < max_depth:
        v = -1 if uniform(seed, it, philox.PURPOSE_NUTS_DIR, j) <= 0.5 else 1
        tree = run.build(minus if v < 0 else plus, v, j, j, 0)
        if v < 0:
            minus = tree.minus
        else:
            plus = tree.plus
        if tree.s == 1 and tree.n > 0:
            if uniform(seed, it, philox.PURPOSE_NUTS_TOP, j) * n <= tree.n:
                sample = tree.cand
        n += tree.n
        alpha += tree.alpha
        n_alpha += tree.n_alpha
        s = tree.s * run.no_u_turn(minus, plus)
        j += 1
    return NutsStep(sample.q, sample.cached, j, run.leaves, alpha / n_alpha, sample.where, h0)


@dataclass
class NutsResult:
    state: object
    eps: float
    depth: np.ndarray
    leaves: np.ndarray
    alpha: np.ndarray
    where: np.ndarray     # (n_iter, 2): doubling and position of each iteration's leaf
    mode_sum: object = None
    n_mean: int = 0


def nuts_run(target, q0, n_iter, eps0, seed, warmup=0, target_accept=0.65, max_depth=10, callback=None):
    """n_iter NUTS iterations from q0; the first `warmup` adapt eps by dual
    averaging on alpha / n_alpha, after which it is frozen at the averaged
    value.  Post-warm-up states are summed into mode_sum (posterior target)."""
    q = q0.copy()
    cached = target.gradient(q)
    eps = float(eps0)
    da = hmc.DualAveraging(eps0, target_accept) if warmup > 0 else None
    depth = np.zeros(n_iter, dtype=np.int32)
    leaves = np.zeros(n_iter, dtype=np.int32)
    alpha = np.zeros(n_iter)
    where = np.zeros((n_iter, 2), dtype=np.int64)
    mode_sum = np.zeros_like(q.modes) if hasattr(q, "modes") else None
    n_mean = 0
    for it in range(n_iter):
        step = nuts_iteration(target, q, cached, eps, seed, it, max_depth)
        q, cached = step.q, step.cached
        depth[it], leaves[it], alpha[it] = step.depth, step.leaves, step.alpha
        where[it] = step.where
        if it < warmup:
            eps = da.update(step.alpha)
            if it == warmup - 1:
                eps = da.final()
        else:
            if mode_sum is not None:
                mode_sum += q.modes
            n_mean += 1
        if callback is not None:
            callback(it, q, step)
    return NutsResult(q, eps, depth, leaves, alpha, where, mode_sum, n_mean)
