"""A seeded random sweep of plan shapes against the FP64 oracle: transform
sizes of every supported family (2^K, 3^K, 5^K, 7^K, mixed radices, N from 2
to 2^14), 1..200 radii up to 0.999 (a zero radius in some), 1..5 steps, both
modes; each free-running and replayed along the oracle's trajectory."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests.parity_tools import TOL, compare, compare_replay

torch = pytest.importorskip("torch")
from paper_1711_08604_amd import Plan  # noqa: E402
from paper_1711_08604_amd.afd import workspace_bytes  # noqa: E402

pytestmark = pytest.mark.gpu

SIZES = ([2 ** k for k in range(1, 15)] + [3 ** k for k in range(1, 9)] + [5 ** k for k in range(1, 7)]
         + [7 ** k for k in range(1, 5)] + [6, 10, 14, 24, 40, 56, 96, 160, 384, 640, 1000, 1536, 2560, 6144, 10240,
                                           12288])


def _cases(count=80, seed=2024):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        n = int(rng.choice(SIZES))
        m = int(rng.integers(1, max(2, min(200, 400_000 // n))))
        steps = int(rng.integers(1, 6))
        rmax = float(rng.choice([0.3, 0.8, 0.95, 0.99, 0.999]))
        prec = str(rng.choice(["fp64", "fp32"]))
        radii = np.sort(rng.uniform(0, rmax, m))
        if rng.random() < 0.3:
            radii[0] = 0.0
        g, _, _ = W.random_kernel_signal(rng, n, int(rng.integers(1, 8)), 0.95)
        out.append((n, radii, steps, prec, W.add_noise(rng, g, 30.0)))
    return out


def test_random_shapes():
    for i, (n, radii, steps, prec, g) in enumerate(_cases()):
        print(f"case {i}: N={n} M={radii.shape[0]} steps={steps} {prec}", flush=True)
        assert workspace_bytes(n, radii, prec) > 0
        ref = O.decompose(g, radii, steps)
        with Plan(n, radii, precision=prec) as plan:
            x = torch.from_numpy(g).to("cuda:0")
            compare(plan.decompose(x, steps), ref, TOL[prec], signal=g, radii=radii)
            compare_replay(plan.replay(x, steps, ref.index.astype(np.int32)), ref, prec, radii=radii)
