"""Binding of the library's adaptive keyframe scheduler (CaRtGS Sec. III-C-2,
Eqs. (5)-(8)); the selection logic runs in libgs.so."""
from __future__ import annotations

import ctypes
from typing import List, Sequence

from . import _lib as L


class KeyframeScheduler:
    """Pool of keyframes with remaining-iteration counts and last losses.

    r0: iterations given to a new keyframe (8 on Replica, 2 on TUM / VECtor
    in the paper); d: divisor of d_k = max(1, k // d) (4 in the paper)."""

    def __init__(self, capacity: int = 4096, r0: int = 8, d: int = 4):
        self._r = (ctypes.c_int32 * capacity)()
        self._l = (ctypes.c_double * capacity)()
        self.c = L.GsScheduler()
        self._check(L.lib().gs_sched_init(ctypes.byref(self.c), self._r, self._l, capacity, r0, d))

    def _check(self, st):
        if st != L.GS_OK:
            raise L.GsError(st, L.lib().gs_sched_last_error().decode())

    def add_keyframe(self) -> int:
        out = ctypes.c_int32()
        self._check(L.lib().gs_sched_add_keyframe(ctypes.byref(self.c), ctypes.byref(out)))
        return out.value

    def select(self, uniforms: Sequence[float]) -> List[int]:
        b = len(uniforms)
        u = (ctypes.c_double * max(b, 1))(*uniforms)
        ids = (ctypes.c_int32 * max(b, 1))()
        n = ctypes.c_int32()
        self._check(L.lib().gs_sched_select(ctypes.byref(self.c), b, u, ids, ctypes.byref(n)))
        return list(ids[:n.value])

    def select_batch(self, uniforms: Sequence[float]) -> List[int]:
        """Fill a batch of len(uniforms) slots by successive draws: when the
        eligible keyframes run out part-way, the next draw refills the counts
        by Eq. (8) first, so a keyframe may take two slots of one batch."""
        ids = self.select(uniforms)
        while len(ids) < len(uniforms):
            more = self.select(uniforms[len(ids):])
            if not more:
                break
            ids += more
        return ids

    def report(self, i: int, loss: float):
        self._check(L.lib().gs_sched_report(ctypes.byref(self.c), int(i), float(loss)))

    @property
    def remaining(self) -> List[int]:
        return list(self._r[:self.c.count])

    @property
    def losses(self) -> List[float]:
        return list(self._l[:self.c.count])

    @property
    def refills(self) -> int:
        return int(self.c.refills)
