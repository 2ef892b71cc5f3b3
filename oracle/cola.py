"""COLA time stepping in the frame comoving with 2LPT observers (FP64).

Test infrastructure only (see the package docstring).

Eq. 1 splits the displacement into the LPT trajectory and a residual; Eq. 2 moves the LPT
acceleration to the right-hand side and discretises only the residual's time derivative.
The paper gives no discrete scheme, so the oracle uses the kick-drift-kick leapfrog that
follows from Eq. 2 with canonical momentum p = a^2 dx/dt and H0 = 1:

  dx/dt = p / a^2,   dp/dt = -grad Phi = (3/2) Omega_m g / a,   g = IFFT[i k delta_k/k^2].

On the 2LPT path x_LPT = q + D1 Psi1 + D2 Psi2 the growth equations give
  d(a^2 dD1/dt)/dt = (3/2) Omega_m D1 / a,   d(a^2 dD2/dt)/dt = (3/2) Omega_m (D2 - D1^2) / a,
so the residual momentum p_res = p - a^2 (dD1/dt Psi1 + dD2/dt Psi2) obeys

  dp_res/dt = (3/2) (Omega_m / a) [ g - D1 Psi1 - (D2 - D1^2) Psi2 ],

whose bracket vanishes order by order in LPT.  With dt = da / (a E):

  kick   p_res += (3/2) Omega_m K(a, b) [bracket at the node],  K  = ∫ da / (a^2 E)
  drift  x     += p_res Dr(a, b) + (D1(b) - D1(a)) Psi1 + (D2(b) - D2(a)) Psi2,
                                                               Dr = ∫ da / (a^3 E)

Nodes a_0..a_{n-1} follow Eq. 3; half-nodes are arithmetic mid-points.  The particle
starts on the 2LPT path (p_res = 0 at a_0).  Each node gets one force evaluation, so a
run of n nodes costs n forces and n-1 drifts.  The state at a node is "synced": p_res
holds its value at that node.  A step j -> j+1 is

  p_res += (3/2) Om K(a_j, a_{j+1/2}) B(x_j);  drift a_j -> a_{j+1};  force at x_{j+1};
  p_res += (3/2) Om K(a_{j+1/2}, a_{j+1}) B(x_{j+1}),

always applying the two half-kicks around a node separately, so that stopping at any
node and resuming gives bitwise the same result.
"""

import numpy as np

from . import cosmology, lpt, pm


class Problem:
    """Box, particle grid, PM_grid factor and time stepping (Table 1 parameters)."""

    def __init__(self, box, n_part, pm_factor, z_init, n_steps, a_final=1.0,
                 sampling="linear", sampling_power=None):
        self.box = float(box)
        self.n_part = int(n_part)
        self.pm_factor = int(pm_factor)
        self.z_init = float(z_init)
        self.n_steps = int(n_steps)
        self.a_final = float(a_final)
        self.sampling = sampling
        self.sampling_power = sampling_power
        self.accel = None  # force law override, accel(pos, n_mesh, box) -> (3, N)

    @property
    def n_mesh(self):
        return self.n_part * self.pm_factor

    @property
    def a_init(self):
        return 1.0 / (1.0 + self.z_init)

    def nodes(self):
        return cosmology.time_nodes(self.a_init, self.n_steps, self.a_final,
                                    self.sampling, self.sampling_power)


class Schedule:
    """FP64 per-node coefficients: D1, D2 at nodes and the kick/drift integrals."""

    def __init__(self, problem, cosmo):
        om = cosmo.omega_m
        self.omega_m = om
        self.a = problem.nodes()
        self.a_half = cosmology.half_nodes(self.a)
        gf = cosmology.growth_factors(self.a, om)
        self.d1, self.d2 = gf[0], gf[1]
        n = self.a.size
        # kick from a node to the next half-node, and from a half-node to the next node
        self.k_out = np.array([cosmology.kick_integral(self.a[j], self.a_half[j], om)
                               for j in range(n - 1)])
        self.k_in = np.array([cosmology.kick_integral(self.a_half[j], self.a[j + 1], om)
                              for j in range(n - 1)])
        self.drift = np.array([cosmology.drift_integral(self.a[j], self.a[j + 1], om)
                               for j in range(n - 1)])


class State:
    """Particle state in SoA form, each array (3, N) with Lagrangian index order."""

    def __init__(self, disp, p_res, psi1, psi2, node=0, q=None):
        self.q = q  # Lagrangian positions (3, N); None means the cubic grid q = index * L / N_p
        self.disp = disp
        self.p_res = p_res
        self.psi1 = psi1
        self.psi2 = psi2
        self.node = node
        self.force = None  # g at the current node, if evaluated

    def copy(self):
        s = State(self.disp.copy(), self.p_res.copy(), self.psi1.copy(), self.psi2.copy(),
                  self.node, self.q)
        s.force = None if self.force is None else self.force.copy()
        return s


def lagrangian_positions(n_part, box, n_mesh):
    """q = index * L / N_p + H / 2 with H = L / n_mesh, shape (3, N).

    The lattice sits half a force-mesh cell off the mesh nodes, so that every particle
    starts at a cell centre.  On a node the CIC weights have a kink and the deposit
    responds one-sidedly to a small displacement; at a centre the response is linear and
    symmetric.  This is a uniform translation of the whole periodic system.
    """
    return lpt.lagrangian_grid(n_part, box).reshape(3, -1) + 0.5 * box / n_mesh


def positions(state, problem):
    """Eulerian positions q + disp, wrapped into [0, box)."""
    box = problem.box
    if state.q is not None:
        return np.mod(state.q + state.disp, box)
    return np.mod(lagrangian_positions(problem.n_part, box, problem.n_mesh) + state.disp, box)


def initial_state(problem, cosmo, seed, amplitude=None):
    """2LPT initial conditions at a_0 with p_res = 0 (the particle starts on the 2LPT path)."""
    ic = lpt.initial_conditions(problem.n_part, problem.box, seed, cosmo, problem.a_init,
                                amplitude)
    n = problem.n_part ** 3
    psi1 = ic["psi1"].reshape(3, n)
    psi2 = ic["psi2"].reshape(3, n)
    disp = ic["disp"].reshape(3, n)
    return State(disp, np.zeros((3, n)), psi1, psi2, node=0)


def bracket(g, d1, d2, psi1, psi2):
    """g - D1 Psi1 - (D2 - D1^2) Psi2: the force not already carried by the 2LPT frame."""
    return g - d1 * psi1 - (d2 - d1 * d1) * psi2


def evaluate_force(state, problem):
    """Acceleration g at the particles: the PM force, or problem.accel(pos, n_mesh, box) when the
    problem carries another force law (the learned correction)."""
    accel = getattr(problem, "accel", None) or pm.pm_accel
    state.force = accel(positions(state, problem), problem.n_mesh, problem.box)
    return state.force


def step(state, problem, sched, j_end):
    """Advance a synced state from its node to node j_end (in place)."""
    om = sched.omega_m
    while state.node < j_end:
        j = state.node
        if state.force is None:
            evaluate_force(state, problem)
        b = bracket(state.force, sched.d1[j], sched.d2[j], state.psi1, state.psi2)
        state.p_res = state.p_res + 1.5 * om * sched.k_out[j] * b
        state.disp = (state.disp + state.p_res * sched.drift[j]
                      + (sched.d1[j + 1] - sched.d1[j]) * state.psi1
                      + (sched.d2[j + 1] - sched.d2[j]) * state.psi2)
        state.node = j + 1
        evaluate_force(state, problem)
        b = bracket(state.force, sched.d1[j + 1], sched.d2[j + 1], state.psi1, state.psi2)
        state.p_res = state.p_res + 1.5 * om * sched.k_in[j] * b
    return state


def lpt_momentum_coefficients(a, om):
    """a^2 dD/dt = a^3 E(a) dD/da for D1 and D2: the momentum of the 2LPT path is
    p_LPT = c1 Psi1 + c2 Psi2."""
    gf = cosmology.growth_factors([a], om)
    e = float(cosmology.hubble_e(a, om))
    return a ** 3 * e * gf[2, 0], a ** 3 * e * gf[3, 0]


def step_pm_only(state, problem, sched, j_end):
    """Plain particle-mesh leapfrog (LPT frame switched off), for comparison with COLA.

    Here state.p_res holds the full momentum p = a^2 dx/dt; kicks use g alone and drifts
    p alone (Appendix B compares such runs with COLA).
    """
    om = sched.omega_m
    while state.node < j_end:
        j = state.node
        if state.force is None:
            evaluate_force(state, problem)
        state.p_res = state.p_res + 1.5 * om * sched.k_out[j] * state.force
        state.disp = state.disp + state.p_res * sched.drift[j]
        state.node = j + 1
        evaluate_force(state, problem)
        state.p_res = state.p_res + 1.5 * om * sched.k_in[j] * state.force
    return state


def redshift_space_positions(state, problem, cosmo, a, los=2, frame="cola"):
    """Eq. 5, plane-parallel along axis los: s = x + v_los / (a H(a)), v = a dx/dt.

    With p = a^2 dx/dt and H0 = 1 the shift is p_los / (a^2 E(a)).  The state must be synced at
    a node of scale factor a.  In the COLA frame the full momentum is p_res plus the 2LPT
    momentum a^2 (dD1/dt Psi1 + dD2/dt Psi2); with the frame switched off p_res is p itself.
    """
    p = state.p_res
    if frame == "cola":
        c1, c2 = lpt_momentum_coefficients(a, cosmo.omega_m)
        p = p + c1 * state.psi1 + c2 * state.psi2
    e = float(cosmology.hubble_e(a, cosmo.omega_m))
    disp = state.disp.copy()
    disp[los] = disp[los] + p[los] / (a * a * e)
    return positions(State(disp, None, None, None, q=state.q), problem)


def displacement_at(state, problem, sched, a_out):
    """Displacement at a_out in [a_j, a_{j+1}) without touching the state.

    The momentum is first brought to the half-node with the node's own force (the kick
    the next step would apply), then drifted from a_j to a_out.  The main integration is
    unchanged, so outputs between nodes do not alter the run.
    """
    j = state.node
    a_j = sched.a[j]
    if a_out == a_j:
        return state.disp.copy()
    if not (j + 1 < sched.a.size and a_j < a_out < sched.a[j + 1]):
        raise ValueError("a_out must lie in [a_j, a_{j+1})")
    om = sched.omega_m
    if state.force is None:
        evaluate_force(state, problem)
    b = bracket(state.force, sched.d1[j], sched.d2[j], state.psi1, state.psi2)
    p_half = state.p_res + 1.5 * om * sched.k_out[j] * b
    d1o, d2o = cosmology.growth_factors([a_out], om)[:2, 0]
    dr = cosmology.drift_integral(a_j, a_out, om)
    return (state.disp + p_half * dr + (d1o - sched.d1[j]) * state.psi1
            + (d2o - sched.d2[j]) * state.psi2)


def run(problem, cosmo, seed, amplitude=None, outputs=()):
    """Full run from the 2LPT initial conditions; returns (state, {a_out: disp})."""
    sched = Schedule(problem, cosmo)
    state = initial_state(problem, cosmo, seed, amplitude)
    snaps = {}
    outs = sorted(outputs)
    for a_out in outs:
        j = int(np.searchsorted(sched.a, a_out, side="right") - 1)
        j = min(j, sched.a.size - 1)
        step(state, problem, sched, j)
        snaps[a_out] = displacement_at(state, problem, sched, a_out)
    step(state, problem, sched, sched.a.size - 1)
    return state, snaps
