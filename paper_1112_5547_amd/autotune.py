"""Autotuner of the fused step's launch shape.

For a lattice type, size, precision and forcing scheme it times every
compiled transverse tile with a set of march-chunk lengths on a scratch
lattice (HIP events on the lattice's stream), keeps the fastest, and caches
the choice in a JSON table keyed by "q:nx:ny:nz:precision" ("precision+guo"
for the Guo forcing, whose kernels are separate instantiations).  Lattices
look their configuration up by exact key, then by the nearest tuned size of
the same type, precision and forcing, then (Guo) of the same precision.

The tuned schedule feeds both single-lattice launches (Lattice.set_kernel)
and batches (Batch.set_tiles with a tile whose block size D2Q9 and D3Q19
members share).
"""
from __future__ import annotations

import json
import math
import os
from typing import Dict, Iterable, List, Optional, Tuple

import numpy as np

from .lattice import Lattice, tiles

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def _pkey(precision: str, forcing: str = "shift") -> str:
    return precision if forcing == "shift" else f"{precision}+{forcing}"


def _key(q, nx, ny, nz, precision, forcing: str = "shift"):
    return f"{q}:{nx}:{ny}:{nz}:{_pkey(precision, forcing)}"


def load(path: str = CACHE) -> Dict[str, dict]:
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def save(table: Dict[str, dict], path: str = CACHE):
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(q: int, nx: int, ny: int, nz: int, precision: str,
           table: Optional[Dict[str, dict]] = None,
           forcing: str = "shift") -> Optional[Tuple[int, int, int, int]]:
    """(variant, tx, ty, mb) for the lattice, or None if nothing of its type is tuned."""
    table = load() if table is None else table
    k = _key(q, nx, ny, nz, precision, forcing)
    if k in table:
        e = table[k]
        return (e["variant"], e["tx"], e["ty"], e["mb"])
    pk = _pkey(precision, forcing)
    if forcing != "shift" and not any(key.split(":")[0] == str(q) and key.split(":")[4] == pk
                                      for key in table):
        pk = precision                 # nothing tuned for this scheme: the shift's choice
    best, bd = None, math.inf
    for key, e in table.items():
        kq, kx, ky, kz, kp = key.split(":")
        if int(kq) != q or kp != pk:
            continue
        d = abs(math.log(int(kx) * int(ky) * int(kz) / (nx * ny * nz)))
        if d < bd:
            bd, best = d, e
    if best is None:
        return None
    march = nz if q == 19 else ny
    return (best["variant"], best["tx"], best["ty"], max(1, min(best["mb"], march)))


def _mb_candidates(march: int) -> List[int]:
    c = sorted({m for m in (4, 8, 16, 24, 32, 48, 64, 96, 128, 256, march) if 1 <= m <= march})
    return c


def tune(q: int, nx: int, ny: int, nz: int = 1, *, precision: str = "fp64", G: float = 1.6,
         tau: float = 1.0, steps: int = 20, warmup: int = 3, mbs: Optional[Iterable[int]] = None,
         include_twopass: bool = True, verbose: bool = False, forcing: str = "shift") -> dict:
    """Times the candidates on a scratch spinodal lattice; returns the best entry
    plus the full table of timings (ms per step)."""
    rng = np.random.default_rng(0)
    shape = (nz, ny, nx)
    rA = 0.5 + rng.uniform(-0.01, 0.01, shape)
    rB = 0.5 + rng.uniform(-0.01, 0.01, shape)
    lat = Lattice(q, nx, ny, nz, tau_A=tau, G=G, precision=precision, forcing=forcing)
    lat.init(rA, rB)
    march = nz if q == 19 else ny
    mbs = list(mbs) if mbs is not None else _mb_candidates(march)
    results = []
    cands = [(v, tx, ty, mb) for v in (0, 2, 3) for (tx, ty) in tiles(q) for mb in mbs]
    if include_twopass:
        cands.append((1, tiles(q)[0][0], tiles(q)[0][1], mbs[0]))
    for cand in cands:
        lat.set_kernel(*cand)
        lat.step(warmup)
        ms = lat.time_steps(steps) / steps
        results.append({"variant": cand[0], "tx": cand[1], "ty": cand[2], "mb": cand[3], "ms": ms})
        if verbose:
            print(f"  {cand} {ms:.4f} ms/step", flush=True)
    lat.close()
    best = min(results, key=lambda r: r["ms"])
    n = nx * ny * nz
    entry = dict(best)
    entry["mlups"] = n / (best["ms"] * 1e-3) / 1e6
    entry["candidates"] = results
    return entry


def tune_and_store(specs, path: str = CACHE, **kw) -> Dict[str, dict]:
    table = load(path)
    for (q, nx, ny, nz, prec) in specs:
        e = tune(q, nx, ny, nz, precision=prec, **kw)
        table[_key(q, nx, ny, nz, prec)] = {k: v for k, v in e.items() if k != "candidates"}
    save(table, path)
    return table


def apply(lat: Lattice, table: Optional[Dict[str, dict]] = None) -> bool:
    """Sets the tuned configuration on a lattice; False if none is known."""
    nz, ny, nx = lat.shape
    cfg = lookup(lat.q, nx, ny, nz, lat.precision, table, getattr(lat, "forcing", "shift"))
    if cfg is None:
        return False
    lat.set_kernel(*cfg)
    return True


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="tune the fused step's tile and march chunk")
    ap.add_argument("specs", nargs="+",
                    help="q:nx:ny:nz:precision[+guo], e.g. 19:256:256:256:fp64")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--store", action="store_true")
    ap.add_argument("--table", default=CACHE, help="JSON table to update (default: packaged)")
    a = ap.parse_args()
    specs = []
    for s in a.specs:
        q, x, y, z, p = s.split(":")
        specs.append((int(q), int(x), int(y), int(z), p))
    table = load(a.table)
    for spec in specs:
        prec, _, forcing = spec[4].partition("+")
        forcing = forcing or "shift"
        e = tune(*spec[:4], precision=prec, forcing=forcing, steps=a.steps, verbose=True)
        best = {k: v for k, v in e.items() if k != "candidates"}
        print(json.dumps(best), flush=True)
        table[_key(*spec[:4], prec, forcing)] = best
    if a.store:
        save(table, a.table)


BATCH_CFGS = [(256, 64, 4), (256, 32, 8), (512, 64, 8), (128, 32, 4)]


def tune_batch(jobs, *, precision: str = "fp32_shifted", mode: str = "fused",
               epoch: int = 50, mbs=(0, 64, 256), verbose: bool = False) -> dict:
    """Chooses the shared block shape (D2Q9 tile width = D3Q19 tile area) and
    the march chunks of a batch by timing one epoch of the given jobs on
    scratch lattices for each candidate.  Returns the fastest as
    {"tx9", "tx19", "ty19", "mb9", "mb19", "ms"}."""
    import time

    import torch

    from .batch import Batch
    lats = []
    for j in jobs:
        lat = Lattice(j.lattice, j.nx, j.ny, j.nz, tau_A=j.tau, G=j.G, precision=precision)
        fl = j.fields()
        lat.init(fl.rho_A, fl.rho_B)
        lats.append(lat)
    best = None
    for (nt, tx19, ty19) in BATCH_CFGS:
        for mb in mbs:
            b = Batch()
            b.set_tiles(nt, tx19, ty19, mb, mb)
            for lat in lats:
                b.add(lat, 10 ** 9)
            b.run(epoch, mode)       # warm-up and graph capture
            b.poll()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.run(epoch, mode)
            b.poll()
            ms = (time.perf_counter() - t0) * 1e3
            for lat in lats:
                b.remove(lat)
            b.close()
            cand = {"tx9": nt, "tx19": tx19, "ty19": ty19, "mb9": mb, "mb19": mb, "ms": ms}
            if verbose:
                print("  batch", cand, flush=True)
            if best is None or ms < best["ms"]:
                best = cand
    for lat in lats:
        lat.close()
    return best
