"""Write oracle-only expected values for the GPU parity tests.

Calls only the oracle (and the seeded shape generators).  Output:
tests/golden/small_fp64_oracle.npz with the 14 observables of the 32 x 32
Gaussian workload (dx = 0.2 fm, peak T = 0.4 GeV, width 2 fm, eta/s = 0.08,
tau 0.5 -> 2.0 fm/c in 150 steps) at steps 0, 1, 10 and 150, plus the
initial energy density array.

Run: python tests/golden/make_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import step as st  # noqa: E402
from oracle.eos import HBARC, TanhEntropyEoS  # noqa: E402
from oracle.lattice import Lattice  # noqa: E402
from paper_1108_5561_amd import workloads as wl  # noqa: E402


def main():
    w = wl.WORKLOADS["small"]
    lat = Lattice(5, 5, 4, 1.0)
    eos = TanhEntropyEoS(g=37.0, Tc=0.17, width=0.02, kappa=2.0)
    prm = st.Params(dx=w["dx"], eta_over_s=w["eta_over_s"])
    e_peak = float(eos.eps(0.4)) / HBARC ** 3
    e0 = e_peak * wl.gaussian_shape(w["nx"], w["ny"], w["dx"], 2.0)
    F, l = st.init_state(lat, eos, e0)
    dtau = (w["tau1"] - w["tau0"]) / w["steps"]
    tau = w["tau0"]
    out = {"e0": e0, "obs_0": st.observables(lat, eos, prm, F, l)}
    t0 = time.time()
    for i in range(1, w["steps"] + 1):
        F, l = st.heun_step(lat, eos, prm, F, l, tau, dtau)
        tau += dtau
        if i in (1, 10, w["steps"]):
            out[f"obs_{i}"] = st.observables(lat, eos, prm, F, l)
            print(f"step {i} tau {tau:.4f} ({time.time() - t0:.1f} s)", flush=True)
    np.savez_compressed(os.path.join(os.path.dirname(__file__), "small_fp64_oracle.npz"), **out)


if __name__ == "__main__":
    main()
