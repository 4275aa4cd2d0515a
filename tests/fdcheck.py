"""Finite-difference reference for the gradient tests: a ladder of central
differences of the oracle and, per component, the value the ladder
converges to."""
import numpy as np

NAMES = ("M", "R_e", "i", "Phi", "N_H", "theta1", "zeta1", "logT1", "theta2", "zeta2", "logT2", "dphi2")
LADDER = (1e-4, 3e-5, 1e-5, 3e-6, 1e-6, 3e-7, 1e-7, 3e-8)


def converged_fd(fds):
    """fds: {step: FD vector}.  Per component the mean of the adjacent pair
    of steps (in decreasing order) whose values agree best, and that pair's
    relative disagreement."""
    steps = sorted(fds, reverse=True)
    ref, delta = np.zeros(12), np.full(12, np.inf)
    for a, b in zip(steps[:-1], steps[1:]):
        d = np.abs(fds[a] - fds[b]) / np.maximum(np.abs(fds[b]), 1e-300)
        better = d < delta
        delta[better] = d[better]
        ref[better] = 0.5 * (fds[a] + fds[b])[better]
    return ref, delta


def fd_gate(g, fds, tol=1e-5, kinked=False):
    """Per component (true relative error against the converged difference,
    bound, delta).  Smooth model: bound = tol + delta.  Kinked model (the
    piecewise-cubic stencils of the atmosphere table: every step crosses
    stencil kinks and the differences wander): the differences over the
    steps <= 1e-5 bracket the derivative, and the bound is tol plus the
    distance from the converged value to the far end of that bracket."""
    ref, delta = converged_fd(fds)
    rel = np.abs(g - ref) / np.abs(ref)
    if not kinked:
        return rel, tol + delta, delta
    small = np.array([fds[s] for s in fds if s <= 1e-5])
    reach = np.maximum(np.abs(small.max(axis=0) - ref), np.abs(small.min(axis=0) - ref)) / np.abs(ref)
    return rel, tol + np.maximum(delta, reach), delta


def report(g, fds, rel, bound, delta):
    ref, _ = converged_fd(fds)
    for n in range(12):
        print("%-7s gpu %+.9e  fd %+.9e  rel err %.1e  bound %.1e  (fd converged to %.1e)"
              % (NAMES[n], g[n], ref[n], rel[n], bound[n], delta[n]), flush=True)
