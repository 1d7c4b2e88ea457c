"""Write tests/golden/adjoint_reference_alfven_perturbed_256.json: the FP64
CPU reference of the adjoint workload's gradient, from the oracle only.

Workload: the perturbed Alfven wave on 256^2 (inputs.alfven_perturbed),
kappa 1, 400 SSP-RK3 steps.  The dt sequence is the plain oracle's own (CFL
0.2 from each step's state) and is stored: it is data of the frozen-dt
gradient, fed to the GPU run as is.  The tangent oracle then runs the 400
steps with exact directional derivatives along the first 8 directions of
inputs.adjoint_directions; stored per direction: dJ = sum (rho(T) - 1)
drho(T), J = 1/2 sum (rho(T) - 1)^2 over the cell averages.

Takes about half an hour on 8 cores.  Run: python tests/golden/make_adjoint_reference.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle as orc  # noqa: E402
from paper_2506_04857_amd import inputs as I  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_reference_alfven_perturbed_256.json")


def main(n=256, nsteps=I.ADJOINT_STEPS, ndirs=8):
    prob = I.alfven_perturbed(n)
    u0 = I.sample(prob)
    t0 = time.time()
    u, dts = u0, []
    for _ in range(nsteps):
        u, d = orc.step(prob, u)
        dts.append(d)
    print(f"oracle forward: {time.time() - t0:.0f} s", flush=True)
    dirs = I.adjoint_directions(prob, ndirs)
    t0 = time.time()
    uT, du = orc.tangent_run(prob, u0, dirs, dts)
    print(f"tangent oracle: {time.time() - t0:.0f} s", flush=True)
    assert all(np.array_equal(a, b) for a, b in zip(uT, u))
    r = uT[0][0] - I.adjoint_objective_target(prob)
    out = {
        "workload": f"alfven_perturbed {n}x{n}, kappa {prob.kappa}, {nsteps} SSP-RK3 steps",
        "objective": "J = 1/2 sum over cells (rho(T) - 1)^2",
        "directions": f"inputs.adjoint_directions(prob, {ndirs}) (default_rng(3506 + k), unit Gaussian, 32 planes)",
        "dts": [float(d) for d in dts],
        "J": float(0.5 * np.sum(r * r)),
        "dJ": [float(np.sum(r * dv[0][0])) for dv in du],
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
