"""The whole gradient of J = 1/2 sum (rho(T) - target)^2 with respect to
every initial degree of freedom (A, X, Y, V planes of all 8 variables), from
the tangent oracle along each basis direction: a column-by-column build of
the reverse product, with no reverse code involved.  Test support only."""
import numpy as np


def basis_gradient(oracle, prob, u0, dts, target=1.0, chunk=256, progress=None):
    shapes = [a.shape for a in u0]
    uT, _ = oracle.tangent_run(prob, u0, [], dts)
    r = uT[0][0] - target
    grad = [np.zeros(s) for s in shapes]
    todo = [(q, f) for q, s in enumerate(shapes) for f in range(int(np.prod(s)))]
    for lo in range(0, len(todo), chunk):
        part = todo[lo:lo + chunk]
        dirs = []
        for q, f in part:
            v = [np.zeros(s) for s in shapes]
            v[q].flat[f] = 1.0
            dirs.append(tuple(v))
        _, du = oracle.tangent_run(prob, u0, dirs, dts)
        for (q, f), dv in zip(part, du):
            grad[q].flat[f] = float(np.sum(r * dv[0][0]))
        if progress:
            progress(lo + len(part), len(todo))
    return tuple(grad), uT
