"""Write the FP64 oracle reference of the 128^2 sinusoidal problem (S8,
sigma_t = 1 + 0.5 sin sin, c = 0.9, GRF source of seed 2, vacuum faces).

Calls only the oracle and the seeded input generators.  It solves the
problem the FP32 library receives (fields rounded to FP32) by source
iteration until the relative L2 change is below 1e-12; at the observed
contraction rate (about 0.9) that leaves the reference within about 1e-11
of the discrete solution, far inside the 1e-5 parity bar.  It also records
the oracle's zero-start iteration counts at 1e-6 under the plain change
rule and under the error-bound rule tested every 16 iterations.

    python tests/golden/make_sinusoid_128_ref.py

Output: tests/golden/sinusoid_128_S8_ref.npz with
    phi          the scalar flux (FP32 copy of the FP64 solution)
    iters_ref    source iterations of that solve
    resid_ref    its last relative change
    tol_ref      1e-12
    iters_change zero-start iterations to a 1e-6 relative change
    iters_bound  zero-start iterations under the error-bound rule at 1e-6
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2509_01416_amd import inputs as I  # noqa: E402

OUT = os.path.join(HERE, "sinusoid_128_S8_ref.npz")
TOL_REF = 1e-12


def main() -> None:
    wl = I.sinusoid_128()
    inst, quad = wl.instances[0], wl.quad
    ref = oracle.solve_instance(inst, quad, tol=TOL_REF, f32_inputs=True)
    ch = oracle.solve_instance(inst, quad, tol=wl.tol, f32_inputs=True)
    bd = oracle.solve_instance(inst, quad, tol=wl.tol, norm="bound", stride=16,
                               f32_inputs=True)
    assert ref.status == ch.status == bd.status == oracle.OK
    np.savez_compressed(
        OUT, phi=ref.phi.astype(np.float32), iters_ref=np.int32(ref.iterations),
        resid_ref=np.float64(ref.residual), tol_ref=np.float64(TOL_REF),
        iters_change=np.int32(ch.iterations), iters_bound=np.int32(bd.iterations))
    print(f"wrote {OUT}: {ref.iterations} iterations to {TOL_REF:g}, "
          f"{ch.iterations} (change rule) and {bd.iterations} (bound rule) to {wl.tol:g}")


if __name__ == "__main__":
    main()
