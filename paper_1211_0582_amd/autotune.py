"""Autotuner: picks the fastest kernel variant per (order, precision, size).

The paper tunes its work decomposition, memory layout and flux-gather
granularity by timing generated variants and keeping the fastest (Sections
3-4).  Here the variants are ahead-of-time kernels selected at run time
(dg_set_variant): the vector-ALU kernel and the matrix-core kernel in each of
its tuning configurations (waves per tile, operator prefetch depth,
occupancy target, flux interleave, split lift, 4-row tail).  For each
(N, precision) and mesh-size bucket this driver builds a seeded mesh of the
bucket's size, times every variant built for it -- one LSERK step (five
fused stages, the production path) with HIP events, and one right-hand side
with the library's timing core (dg_time_rhs) -- and records the winner by
step time in a JSON cache:

    {"<arch>": {"<precision>": {"<N>": {"<bucket>": {"K": K, "variant": name,
        "step_ms": {name: t}, "rhs_ms": {name: t}}}}}}

Buckets: "small" (K < 20,000 elements: the batch's problems; tuned on the
8^3 x 6 cube, K = 3,072) and "large" (tuned on the 24^3 x 6 cube, K = 82,944).
The cache path is $DG_AUTOTUNE_CACHE, else autotune_cache.json next to this
file.  ``python -m paper_1211_0582_amd.autotune [--orders 1-9] [--precisions fp64,fp32]``
"""
from __future__ import annotations

import argparse
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))

#: element count below which a problem belongs to the "small" bucket
SMALL_K = 20000
#: cube resolution k (K = 6 k^3) of the tuning mesh of each bucket
BUCKET_K = {"small": 8, "large": 24}


def cache_path() -> str:
    return os.environ.get("DG_AUTOTUNE_CACHE", os.path.join(HERE, "autotune_cache.json"))


def _arch() -> str:
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def bucket(K: int) -> str:
    return "small" if K < SMALL_K else "large"


def load(path: str | None = None) -> dict:
    path = path or cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save(cache: dict, path: str | None = None) -> None:
    path = path or cache_path()
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(N: int, precision, K: int | None = None, arch: str | None = None, path: str | None = None):
    """Variant name recorded for (N, precision) and K's bucket on this GPU
    architecture (the other bucket if that one is missing), or None."""
    from . import dg
    if isinstance(precision, int):
        precision = {v: k for k, v in dg.PRECISIONS.items()}[precision]
    entry = load(path).get(arch or _arch(), {}).get(precision, {}).get(str(N))
    if not entry:
        return None
    want = bucket(K) if K is not None else "large"
    for b in (want, "large" if want == "small" else "small"):
        if b in entry:
            return entry[b]["variant"]
    return None


def record(cache: dict, arch: str, precision: str, N: int, bkt: str, K: int, step_ms: dict, rhs_ms: dict) -> str:
    best = min(step_ms, key=step_ms.get)
    cache.setdefault(arch, {}).setdefault(precision, {}).setdefault(str(N), {})[bkt] = {
        "K": int(K), "variant": best, "step_ms": step_ms, "rhs_ms": rhs_ms}
    return best


def _time_steps(torch, p, du, res, dt, nsteps, reps):
    stream = torch.cuda.current_stream()
    p.rk_step(du, res, 0.0, dt, nsteps, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        p.rk_step(du, res, 0.0, dt, nsteps, stream)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / (reps * nsteps)


def tune(orders, precisions, buckets=("small", "large"), reps: int = 5, path: str | None = None,
         verbose=True, sizes: dict | None = None) -> dict:
    import torch

    import dg_inputs as I
    from . import dg
    arch = _arch()
    cache = load(path)
    sizes = dict(BUCKET_K, **(sizes or {}))
    for prec in precisions:
        for N in orders:
            for bkt in buckets:
                VX, EToV = I.kuhn_cube(sizes[bkt], 0.1, 0)
                try:
                    p = dg.Problem(N, VX, EToV, prec)
                except dg.DgError as e:
                    if e.status == dg.DG_EUNSUPPORTED:  # no kernel at all for (N, precision)
                        break
                    raise
                xyz = p.nodes()
                u = I.cavity_mode(xyz[..., 0], xyz[..., 1], xyz[..., 2]) + \
                    I.field_noise((6, p.info.K, p.info.Np), 1e-3, 1)
                du = p.pack(u)
                res = p.zeros_state()
                out = p.zeros_state()
                dt = 0.5 * p.info.dt_cfl1
                step_ms, rhs_ms = {}, {}
                for v in range(dg.dg_variant_count()):
                    name = dg.dg_variant_name(v)
                    try:
                        p.set_variant(v)
                    except dg.DgError as e:
                        if e.status == dg.DG_EUNSUPPORTED:
                            continue
                        raise
                    rhs_ms[name] = dg.dg_time_rhs(p.handle, du, out, 3, 4 * reps)
                    step_ms[name] = _time_steps(torch, p, du, res, dt, 2, reps)
                best = record(cache, arch, prec, N, bkt, p.info.K, step_ms, rhs_ms)
                if verbose:
                    print(f"autotune {arch} {prec} N={N} {bkt} K={p.info.K}: " +
                          ", ".join(f"{n} {t * 1e3:.1f} us" for n, t in step_ms.items()) + f" -> {best}",
                          flush=True)
                p.close()
                del du, res, out
                save(cache, path)
    return cache


def _orders(spec: str):
    if "-" in spec:
        a, b = spec.split("-")
        return list(range(int(a), int(b) + 1))
    return [int(x) for x in spec.split(",")]


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--orders", default="1-9")
    ap.add_argument("--precisions", default="fp64,fp32,f16x3,bf16x3")
    ap.add_argument("--buckets", default="small,large")
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    tune(_orders(a.orders), a.precisions.split(","), a.buckets.split(","), a.reps)
