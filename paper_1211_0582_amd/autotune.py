"""Autotuner: picks the fastest right-hand-side kernel per (order, precision).

The paper tunes its work decomposition, memory layout and flux-gather
granularity by timing generated variants and keeping the fastest (Sections
3-4).  Here the variants are ahead-of-time kernels selected at run time
(dg_set_variant); this driver times every variant built for an (N, precision)
on a seeded mesh of about ``dofs`` nodal values per field with the library's
timing core (dg_time_rhs) and records the winner in a JSON cache:

    {"<arch>": {"<precision>": {"<N>": {"variant": name, "ms": {name: time}}}}}

The cache path is $DG_AUTOTUNE_CACHE, else autotune_cache.json next to this
file.  ``python -m paper_1211_0582_amd.autotune [--orders 1-9] [--precisions fp64,fp32]``
"""
from __future__ import annotations

import argparse
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def cache_path() -> str:
    return os.environ.get("DG_AUTOTUNE_CACHE", os.path.join(HERE, "autotune_cache.json"))


def _arch() -> str:
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


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


def lookup(N: int, precision, arch: str | None = None, path: str | None = None):
    """Variant name recorded for (N, precision) on this GPU architecture, or None."""
    from . import dg
    if isinstance(precision, int):
        precision = {v: k for k, v in dg.PRECISIONS.items()}[precision]
    entry = load(path).get(arch or _arch(), {}).get(precision, {}).get(str(N))
    return None if entry is None else entry["variant"]


def record(cache: dict, arch: str, precision: str, N: int, times: dict) -> str:
    best = min(times, key=times.get)
    cache.setdefault(arch, {}).setdefault(precision, {})[str(N)] = {"variant": best, "ms": times}
    return best


def tune(orders, precisions, dofs: float = 2e6, reps: int = 20, path: str | None = None, verbose=True) -> dict:
    import dg_inputs as I
    from . import dg
    arch = _arch()
    cache = load(path)
    for prec in precisions:
        for N in orders:
            k = max(2, I.k_for_dofs(N, dofs))
            VX, EToV = I.kuhn_cube(k, 0.1, 0)
            try:
                p = dg.Problem(N, VX, EToV, prec)
            except dg.DgError as e:
                if e.status == dg.DG_EUNSUPPORTED:  # no kernel at all for (N, precision)
                    continue
                raise
            xyz = p.nodes()
            u = I.cavity_mode(xyz[..., 0], xyz[..., 1], xyz[..., 2]) + \
                I.field_noise((6, p.info.K, p.info.Np), 1e-3, 1)
            du = p.pack(u)
            out = p.zeros_state()
            times = {}
            for v in range(dg.dg_variant_count()):
                name = dg.dg_variant_name(v)
                try:
                    p.set_variant(v)
                except dg.DgError as e:
                    if e.status == dg.DG_EUNSUPPORTED:
                        continue
                    raise
                times[name] = dg.dg_time_rhs(p.handle, du, out, 3, reps)
            best = record(cache, arch, prec, N, times)
            if verbose:
                print(f"autotune {arch} {prec} N={N} K={p.info.K}: " +
                      ", ".join(f"{n} {t * 1e3:.1f} us" for n, t in times.items()) + f" -> {best}", flush=True)
            p.close()
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
    ap.add_argument("--precisions", default="fp64,fp32")
    ap.add_argument("--dofs", type=float, default=2e6)
    ap.add_argument("--reps", type=int, default=20)
    a = ap.parse_args()
    tune(_orders(a.orders), a.precisions.split(","), a.dofs, a.reps)
