"""Writes the oracle's state of the isentropic vortex on the 204,800-triangle
mesh (320 x 320 split squares of [0, 10]^2, +-0.1h jitter, seed 3; strength 5
on the background (1, 1, 1, 1)) at T = 2, with the fixed step
dt = 0.3 * min inradius / max signal speed of the initial state and the last
step clipped to T.

Calls only the oracle and the seeded input generator:

    python tests/golden/make_c3_vortex_T2.py [threads]

Output c3_vortex_T2_oracle.npz (caller cell order): wbar [4][N], the
derivative averages grad [2][4][S] on the sampled cells idx [S] (every 8th
cell), dt, the number of full steps and the clipped last step.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import OracleMesh  # noqa: E402
from workloads import vortex_workload  # noqa: E402

OUT = os.path.join(HERE, "c3_vortex_T2_oracle.npz")


def main(nthreads=0):
    wl = vortex_workload()
    om = OracleMesh.from_workload(wl)
    dt = om.max_dt(wl.state0, wl.cfl)
    n = int(np.floor(wl.T / dt + 1e-12))
    rem = wl.T - n * dt
    s = wl.state0.copy()
    t0 = time.time()
    done = 0
    while done < n:
        k = min(100, n - done)
        s = om.run(s, dt, k, nthreads, t=done * dt)
        done += k
        print(f"{done}/{n} steps, {time.time() - t0:.0f} s", flush=True)
    if rem > 1e-14 * wl.T:
        s = om.step(s, rem, nthreads, t=n * dt)
    idx = np.arange(0, om.N, 8)
    np.savez_compressed(OUT, wbar=s[0], grad=s[1:, :, idx], idx=idx, dt=dt, nsteps=n, rem=rem)
    print("wrote", OUT, flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 0)
