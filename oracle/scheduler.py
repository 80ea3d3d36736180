"""Adaptive keyframe selection of CaRtGS Sec. III-C-2, Eqs. (5)-(8) --
TEST INFRASTRUCTURE (plain Python reference of the library's scheduler).

State: per keyframe i the remaining optimisation count r_i and the last
loss l_i.  A new keyframe enters with r^0 iterations and loss l_new
(Eqs. (5)-(7); the paper leaves l_{k+1} open, read here as +inf so that a
fresh keyframe ranks first at the next refill).  Each iteration picks a
keyframe uniformly among those with r_i > 0, decrements its r and stores
its new loss.  When no keyframe has r_i > 0, every r_i is reset by Eq. (8):
2 for the d_k largest losses, 1 otherwise, with d_k = max(1, floor(k / d)).
Ties in the top-d_k ranking go to the lower keyframe index.

Random draws are inputs: a uniform u in [0, 1) picks position floor(u m)
of the m eligible keyframes in index order.  A batch of B keyframes per
iteration draws B times without replacement (B = 1 is the paper's rule).
"""
from __future__ import annotations

import math
from typing import List, Sequence


class Scheduler:
    def __init__(self, r0: int = 8, d: int = 4):
        self.r0, self.d = int(r0), int(d)
        self.r: List[int] = []
        self.l: List[float] = []
        self.refills = 0

    def add_keyframe(self, loss: float = math.inf) -> int:
        self.r.append(self.r0)
        self.l.append(float(loss))
        return len(self.r) - 1

    def refill(self):
        k = len(self.r)
        dk = max(1, k // self.d)
        # top-d_k largest losses, ties to the lower index
        order = sorted(range(k), key=lambda i: (-self.l[i], i))
        top = set(order[:dk])
        self.r = [2 if i in top else 1 for i in range(k)]
        self.refills += 1

    def select(self, uniforms: Sequence[float]) -> List[int]:
        """Pick len(uniforms) distinct keyframes (fewer if fewer are eligible)."""
        if not self.r:
            return []
        if not any(x > 0 for x in self.r):
            self.refill()
        eligible = [i for i, x in enumerate(self.r) if x > 0]
        out = []
        for u in uniforms:
            if not eligible:
                break
            j = min(int(math.floor(u * len(eligible))), len(eligible) - 1)
            out.append(eligible.pop(j))
        for i in out:
            self.r[i] -= 1
        return out

    def report(self, i: int, loss: float):
        self.l[i] = float(loss)
