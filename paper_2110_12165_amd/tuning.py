"""Launch configurations of the benchmark workloads on gfx950.

``bench_options(workload, variant)`` returns the keyword options of
``HMatrix.build`` for one of the three product variants:

* ``batched_f32`` — FP32 factors, batched panels (tuned schedule);
* ``batched_f64`` — FP64 factors, batched panels (tuned schedule);
* ``plain_f64``   — FP64 factors, natural layout, two plain launches.

The batched schedule (waves per workgroup, unit size, split or persistent
launch) is the fastest one measured on an MI355X for that workload by a
sweep over the schedules hmat_autotune also searches.
"""
from __future__ import annotations

from synth import WORKLOADS

# workload -> (wg_waves phase 2, wg_waves phase 1, kernel): fastest measured on MI355X
TUNED = {
    "dip30_480x256": (8, 4, "split"),
}


def bench_options(workload: str, variant: str) -> dict:
    w = WORKLOADS[workload]
    base = dict(aca_eps=w["aca_eps"], eta=w["eta"], leaf=w["leaf"], lattice=w["lattice"])
    wg, wg1, kern = TUNED.get(workload, (8, 4, "split"))
    if variant == "batched_f32":
        return dict(base, prec="f32", kernel=kern, wg_waves=wg, wg_waves_p1=wg1)
    if variant == "batched_f64":
        return dict(base, prec="f64", kernel=kern, wg_waves=wg, wg_waves_p1=wg1)
    if variant == "plain_f64":
        return dict(base, prec="f64", kernel="plain")
    raise ValueError(f"unknown variant {variant}")
