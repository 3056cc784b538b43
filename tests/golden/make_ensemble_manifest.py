"""Write ensemble48_manifest.json: the 48-configuration batched workload
(lattice sizes drawn uniformly from 8^4, 12^4, 16^4, 24^4; seeds 100..147;
eps uniform in [0.2, 0.35]; Haar-random gauge).  The draw uses numpy's PCG64
stream seeded with 48; the file is the input specification both the tests and
the benchmark read, and holds no expected value."""
import json
import os

import numpy as np


def main():
    rng = np.random.default_rng(48)
    sizes = rng.choice([8, 12, 16, 24], size=48)
    eps = rng.uniform(0.2, 0.35, size=48)
    configs = [{"index": i, "seed": 100 + i, "dims": [int(sizes[i])] * 4, "eps": round(float(eps[i]), 6),
                "haar": True} for i in range(48)]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ensemble48_manifest.json")
    with open(out, "w") as f:
        json.dump({"description": "48 SU(3) configurations for the batched persistent launch",
                   "configs": configs}, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
