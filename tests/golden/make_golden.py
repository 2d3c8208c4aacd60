"""Write tests/golden/oracle_4x4x4x4_seed0.json from the FP64 oracle only.

The workload is the small plain-Wilson case: 4^4 lattice, periodic space,
antiperiodic time, kappa = 0.12, links from the seeded SU(3) generator (seed
0), one complex Gaussian source drawn after the links.  The paper prints no
worked example for this operator, so these values are regression anchors for
the oracle (its correctness is pinned by the closed-form, invariant and
brute-force tests), and a reference for the GPU path at the same inputs.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2302_00850_amd.synth import Synth, bc_phases  # noqa: E402


def main():
    dims = (4, 4, 4, 4)
    kappa = 0.12
    bc = bc_phases((0, 0, 0, np.pi))
    s = Synth(0)
    U = s.gauge(dims).numpy()
    b = s.gaussian_spinor(dims)[0].numpy()
    Mb = oracle.apply_M(U, b, kappa, bc)
    x, it, res = oracle.cg(U, b, kappa, bc, system=0, tol=1e-10)
    x_e, it_e, res_e = oracle.cg(U, b, kappa, bc, system=1, tol=1e-10)
    out = {
        "source": "tests/golden/make_golden.py (FP64 oracle); workload: 4^4, kappa 0.12, "
                  "theta = (0,0,0,pi), synthetic SU(3) links mixed 0.3 toward 1, seed 0",
        "plaquette": oracle.plaquette(U),
        "norm2_b": float(np.vdot(b, b).real),
        "norm2_Mb": float(np.vdot(Mb, Mb).real),
        "Mb_site0": [[float(z.real), float(z.imag)] for z in Mb[0, 0, 0, 0].ravel()],
        "cg_full_iterations": it,
        "cg_full_true_residual": res,
        "norm2_x_full": float(np.vdot(x, x).real),
        "cg_schur_iterations": it_e,
        "cg_schur_true_residual": res_e,
        "norm2_x_schur": float(np.vdot(x_e, x_e).real),
    }
    path = os.path.join(HERE, "oracle_4x4x4x4_seed0.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
