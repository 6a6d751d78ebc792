"""Write tests/golden/longrun_<name>.npz: a sample of the FP64 oracle's end state after the full
step count of each long run in ``tests/longrun.py`` (the 1D dusty shock at every t_stop over
2000 steps, the 3D box over 200 steps), started from the FP32 state those runs load on the
device.  Calls only the oracle.

    python tests/golden/make_longrun_oracle.py [name ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O      # noqa: E402
from tests import longrun as LR     # noqa: E402


def main(names):
    for name in names:
        make, steps, stride = LR.RUNS[name]
        prob = make()
        p = prob.params
        sg, sd = LR.fp32_state(prob)
        og, od = LR.to_oracle(sg), LR.to_oracle(sd)
        t0 = time.time()
        # the gas rho left by the step is the summation density the last step used, as on the
        # device
        O.step(p, og, od, steps)
        print(f"{name}: {steps} steps in {time.time() - t0:.1f} s on {O.num_threads()} threads", flush=True)
        out = {}
        for pre, ph in (("g_", og), ("d_", od)):
            s = LR.sample(dict(cell=ph.cell, off=ph.off, vel=ph.vel, id=ph.id, rho=ph.rho,
                               energy=ph.energy), stride)
            for k, v in s.items():
                if pre == "d_" and k in ("rho", "energy"):
                    continue
                out[pre + k] = v
        out["steps"] = np.array(steps)
        out["stride"] = np.array(stride)
        np.savez_compressed(LR.golden_path(name), **out)


if __name__ == "__main__":
    main(sys.argv[1:] or list(LR.RUNS))
