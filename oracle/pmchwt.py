"""Dense static-mode PMCHWT operator, right-hand side and solve (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Blocks (eq. Zpq_delta, Sec. II.A), per particle unknowns [J_e (N); J_m (N)]:
  Z^{mu mu} = [[z- T- + z+ T+ ,  K- + K+       ],
               [-(K- + K+)    ,  T-/z- + T+/z+ ]]      (self, both media)
  Z^{mu nu} = [[z- T- , K-], [-K-, T-/z-]]             (mu != nu, exterior only)
with T, K of ``operators`` expressed in the static modes by sampling
psi_i = sum_j m_ij xi_j at the quadrature points (the same numbers as
M {A}_xi M^T of eq. BasisTransformation).  Units: k- = 2 pi, z- = 1,
k+ = k- sqrt(eps_r), z+ = z- / sqrt(eps_r).

Right-hand side (Sec. II): V = -[<psi, E_inc>; <psi, H_inc>] for
E_inc = pol exp(-j k khat . r), H_inc = khat x E_inc / z-.

Background medium (Sec. II: particles (eps+, mu+) in (eps-, mu-), mu = 1):
with eps_bg = eps- and every eps_r relative to vacuum, k- = k0 sqrt(eps-),
z- = 1 / sqrt(eps-), k+ = k0 sqrt(eps+), z+ = 1 / sqrt(eps+) (vacuum
wavelengths and the vacuum impedance as units).  eps_bg = 1 is the vacuum
case above.
"""
from __future__ import annotations

import numpy as np

from .basis import MeshBasis
from .operators import SampledBasis, SelfSingular, direct_TK, self_TK
from .static_modes import static_modes

K0 = 2.0 * np.pi


class ParticleClass:
    """One particle shape: mesh, static modes and sampled basis."""

    def __init__(self, verts, tris, edges, n_perp, n_par, eps_r, M=None):
        self.mb = MeshBasis(verts, tris, edges)
        self.sing = SelfSingular(self.mb)
        if M is None:
            M, self.gamma_perp, self.gamma_par = static_modes(self.mb, n_perp, n_par, self.sing)
        self.M = np.asarray(M, float)
        self.n_modes = self.M.shape[0]
        self.bs = SampledBasis(self.mb, self.M)
        self.eps_r = complex(eps_r)

    @property
    def n(self):
        return 2 * self.n_modes


def assemble_block(T, K, zeta):
    return np.block([[zeta * T, K], [-K, T / zeta]])


def self_block(pc: ParticleClass, k0: float = K0, eps_bg: complex = 1.0):
    """Z_s of eq. Zpq_delta with delta = 1 (exterior: the background)."""
    k_out, z_out = k0 * np.sqrt(eps_bg), 1.0 / np.sqrt(eps_bg)
    k_in = k0 * np.sqrt(pc.eps_r)
    z_in = 1.0 / np.sqrt(pc.eps_r)
    To, Ko = self_TK(pc.bs, pc.sing, k_out)
    Ti, Ki = self_TK(pc.bs, pc.sing, k_in)
    Kt = Ko + Ki
    return np.block([[z_out * To + z_in * Ti, Kt], [-Kt, To / z_out + Ti / z_in]])


def pair_block(pp: ParticleClass, pq: ParticleClass, offset, k0: float = K0, eps_bg: complex = 1.0):
    """Z^{mu nu} for distinct particles, offset = r_nu - r_mu."""
    T, K = direct_TK(pp.bs, pq.bs, offset, k0 * np.sqrt(eps_bg))
    return assemble_block(T, K, 1.0 / np.sqrt(eps_bg))


class DenseProblem:
    """Particles at ``centers`` with class ids into ``classes``; blocks are
    memoised by (class_mu, class_nu, centre offset)."""

    def __init__(self, classes, centers, class_id, k0: float = K0, eps_bg: complex = 1.0):
        self.classes = classes
        self.centers = np.asarray(centers, float)
        self.class_id = np.asarray(class_id, int)
        self.k0 = k0                                    # vacuum wavenumber
        self.eps_bg = complex(eps_bg)
        kb = k0 * np.sqrt(self.eps_bg)
        self.k = kb.real if kb.imag == 0 else kb        # background wavenumber
        self.zeta = 1.0 / np.sqrt(self.eps_bg)          # background impedance / vacuum impedance
        self._cache = {}

    @property
    def n_particles(self):
        return len(self.centers)

    def block(self, mu, nu):
        cm, cn = self.class_id[mu], self.class_id[nu]
        off = self.centers[nu] - self.centers[mu]
        key = self._key(mu, nu)
        if key not in self._cache:
            if mu == nu:
                self._cache[key] = self_block(self.classes[cm], self.k0, self.eps_bg)
            else:
                self._cache[key] = pair_block(self.classes[cm], self.classes[cn], off, self.k0, self.eps_bg)
        return self._cache[key]

    def _key(self, mu, nu):
        off = self.centers[nu] - self.centers[mu]
        return (self.class_id[mu], self.class_id[nu], tuple(np.round(off, 9)))

    def prefetch(self, pairs, workers: int = 0):
        """Compute the blocks of the (mu, nu) pairs in parallel worker
        processes (fork; one BLAS thread each).  Pure speed-up of ``block``."""
        import multiprocessing as mp
        todo = {}
        for mu, nu in pairs:
            k = self._key(mu, nu)
            if k not in self._cache and k not in todo:
                todo[k] = (mu, nu)
        if not todo:
            return
        workers = workers or min(len(todo), len(__import__("os").sched_getaffinity(0)))
        global _PREFETCH_PROB
        _PREFETCH_PROB = self
        items = list(todo.items())
        if workers <= 1:
            for k, (mu, nu) in items:
                self.block(mu, nu)
            return
        ctx = mp.get_context("fork")
        with ctx.Pool(workers, initializer=_limit_threads) as pool:
            for k, blk in zip([k for k, _ in items], pool.map(_prefetch_one, [v for _, v in items], chunksize=1)):
                self._cache[k] = blk

    def dense(self):
        P = self.n_particles
        n = [self.classes[c].n for c in self.class_id]
        off = np.concatenate([[0], np.cumsum(n)])
        Z = np.zeros((off[-1], off[-1]), complex)
        for mu in range(P):
            for nu in range(P):
                Z[off[mu]:off[mu + 1], off[nu]:off[nu + 1]] = self.block(mu, nu)
        return Z

    def matvec_rows(self, x, rows):
        """y_mu = sum_nu Z^{mu nu} x_nu for the particles in ``rows`` only;
        x is [P][n] (or [P][n][R])."""
        x = np.asarray(x)
        out = []
        for mu in rows:
            acc = 0
            for nu in range(self.n_particles):
                acc = acc + self.block(mu, nu) @ x[nu]
            out.append(acc)
        return np.array(out)

    def rhs(self, khat, pol):
        """V for a plane wave exp(-j k khat . r) pol; returns [P][n]."""
        khat = np.asarray(khat, float)
        pol = np.asarray(pol, complex)
        hpol = np.cross(khat, pol) / self.zeta           # H_inc / E amplitude
        out = []
        for mu in range(self.n_particles):
            pc = self.classes[self.class_id[mu]]
            X = pc.bs.X + self.centers[mu][None, :]
            ph = np.exp(-1j * self.k * (X @ khat)) * pc.bs.W
            Ev = sum(pc.bs.Psi[c] @ (ph * pol[c]) for c in range(3))
            Hv = sum(pc.bs.Psi[c] @ (ph * hpol[c]) for c in range(3))
            out.append(-np.concatenate([Ev, Hv]))
        return np.array(out)


_PREFETCH_PROB = None


def _limit_threads():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _prefetch_one(pair):
    mu, nu = pair
    return _PREFETCH_PROB.block(mu, nu)


def solve_dense(prob: DenseProblem, V):
    """LU solve of the dense system; V is [P][n] (or [P][n][R])."""
    Z = prob.dense()
    sh = np.asarray(V).shape
    x = np.linalg.solve(Z, np.asarray(V).reshape(Z.shape[0], -1))
    return x.reshape(sh)
