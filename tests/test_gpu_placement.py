"""Learned placement on the GPU: operation timings this engine records on both
devices train the MLP with the library's GPU kernels, and on held-out batches
the placements it chooses must take less measured time than those of the
analytic cost model (Eq. 7-9) it replaces."""
import os

import numpy as np
import pytest

from gpu_helpers import log

pytestmark = pytest.mark.gpu


def test_learned_placement_gains_over_analytic():
    from paper_2111_04289_amd import placement
    cores = min(16, os.cpu_count() or 1)
    pool = placement.Pool(1 << 22, static_rows=1 << 16)
    for op in placement.OPS:  # warm both devices
        cfg = {"op": op, "rows": 4096, "sel": 0.3, "window_s": 10, "slide_s": 1}
        cols = pool.batch(np.random.default_rng(0), 4096)
        placement.run_gpu(pool, cfg, cols)
        placement.run_cpu(pool, cfg, cols, cores)
    recs = placement.collect(pool, 1500, 1, cores, 1 << 21, 1 << 22)
    held = placement.collect(pool, 300, 2, cores, 1 << 21, 1 << 21)
    net, losses = placement.train(recs, epochs=400)
    log(f"loss {losses[0]:.3f} -> {losses[-1]:.3f}")
    assert losses[-1] < 0.5 * losses[0]
    ev = placement.evaluate(held, net.get_params(), cores)
    log(str(ev))
    t = ev["total_ms"]
    assert t["learned"] < t["analytic"], ev
    assert ev["mispredictions"]["learned"] <= ev["mispredictions"]["analytic"], ev
