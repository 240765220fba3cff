"""Write ke_increments_k3.txt: relative kinetic-energy change of the first two
IMEX-HDG steps (ARS(2,2,2), dt = 1e-3, n_R = 3, k = 3, seed-0 stream-function
data, zero forcing) computed by the oracle on the 64 x 64 mesh, where the flow
is resolved and the increments have converged under mesh refinement (the
32 x 32 run differs by a few percent).  Calls only the oracle."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import hdg_inputs as hi  # noqa: E402
from oracle.forms import Discretisation  # noqa: E402
from oracle.imex import IMEXHDG, ars222  # noqa: E402


def main(n=64):
    par = hi.stream_function_params(0)
    X, C = hi.unit_square_mesh(n)
    d = Discretisation(X, C, 3)
    st = IMEXHDG(d, 1e-3, ars222(), 3)
    Q, p, lam = st.initial_state(lambda x, y: hi.streamfunction_velocity(par, x, y))
    e = [d.kinetic_energy(Q)]
    for s in range(2):
        Q, p, lam = st.step(Q, p, lam, s * 1e-3)
        e.append(d.kinetic_energy(Q))
    inc = np.diff(e) / e[0]
    with open(os.path.join(HERE, "ke_increments_k3.txt"), "w") as fh:
        fh.write(f"# written by make_ke_golden.py (oracle, {n}x{n} mesh, k=3, ARS(2,2,2), dt=1e-3, n_R=3, seed 0)\n")
        fh.write(f"# initial kinetic energy {e[0]:.15e}\n")
        for v in inc:
            fh.write(f"{v:.6e}\n")


if __name__ == "__main__":
    main()
