"""Python handle of a batch of lattices (marshalling over the C ABI)."""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional

from . import _abi
from ._abi import check, lib
from .lattice import Lattice

MODES = {"per_lattice": _abi.LBM_BATCH_PER_LATTICE, "fused": _abi.LBM_BATCH_FUSED,
         "persistent": _abi.LBM_BATCH_PERSISTENT}


class Batch:
    """Independent lattices advanced together on one stream.

    hbm_budget: bytes of member state admitted (0 = unlimited).  Members keep
    their own state; a member's results are bitwise the same as running it
    alone, whatever the mode.
    """

    def __init__(self, hbm_budget: int = 0, use_torch: bool = True):
        self._b = ctypes.c_void_p()
        self._stream = None
        stream = None
        if use_torch:
            import torch
            self._stream = torch.cuda.Stream()
            stream = ctypes.c_void_p(self._stream.cuda_stream)
        check(lib().lbm_batch_create(ctypes.byref(self._b), int(hbm_budget), stream), "batch_create")
        self._members: Dict[int, Lattice] = {}

    def close(self):
        """Releases the batch.  The native object is freed even when destroy
        reports an error (an unread persistent-launch give-up), so the handle
        is dropped before the status is checked."""
        self._members.clear()
        if self._b:
            b, self._b = self._b, ctypes.c_void_p()
            check(lib().lbm_batch_destroy(b), "batch_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, lat: Lattice, steps: int) -> bool:
        """Admit a lattice; False when the memory budget has no room."""
        rc = lib().lbm_batch_add(self._b, lat.handle, int(steps))
        if rc == _abi.LBM_EBUDGET:
            return False
        check(rc, "batch_add")
        self._members[lat.handle.value] = lat
        return True

    def remove(self, lat: Lattice):
        check(lib().lbm_batch_remove(self._b, lat.handle), "batch_remove")
        self._members.pop(lat.handle.value, None)

    def run(self, epoch_steps: int, mode: str = "fused"):
        check(lib().lbm_batch_run(self._b, int(epoch_steps), MODES[mode]), "batch_run")

    def run_noalloc(self, epoch_steps: int, mode: str = "fused"):
        """The same epoch without device allocations: the fused form's tables go
        to the library's fixed per-GPU scratch array (calls on one GPU must not
        overlap)."""
        check(lib().lbm_batch_run_noalloc(self._b, int(epoch_steps), MODES[mode]),
              "batch_run_noalloc")

    def poll(self) -> List[Lattice]:
        """Waits for queued work; returns members whose steps are complete."""
        n = max(1, len(self._members))
        arr = (ctypes.c_void_p * n)()
        nd = ctypes.c_int()
        check(lib().lbm_batch_poll(self._b, arr, n, ctypes.byref(nd)), "batch_poll")
        return [self._members[arr[i]] for i in range(nd.value)]

    def stats(self):
        m, b, pend = ctypes.c_int(), ctypes.c_size_t(), ctypes.c_double()
        check(lib().lbm_batch_stats(self._b, ctypes.byref(m), ctypes.byref(b), ctypes.byref(pend)),
              "batch_stats")
        return {"members": m.value, "bytes_used": b.value, "pending_site_updates": pend.value}

    def set_tiles(self, tx9: int = 0, tx19: int = 0, ty19: int = 0, mb9: int = 0, mb19: int = 0):
        check(lib().lbm_batch_set_tiles(self._b, tx9, tx19, ty19, mb9, mb19), "batch_set_tiles")

    def set_spin_limit(self, spins: int):
        """Grid-barrier polls before a persistent launch gives up (0: default)."""
        check(lib().lbm_batch_set_spin_limit(self._b, int(spins)), "batch_set_spin_limit")

    @property
    def members(self) -> List[Lattice]:
        return list(self._members.values())
