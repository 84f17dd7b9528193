"""Closed form of <Z_u Z_v> for depth p=1 (oracle step O10).

An independent pin for the statevector code.  For unit weights it is the published
p=1 MaxCut edge formula (Wang, Hadfield, Jiang, Rieffel, Phys. Rev. A 97, 022304
(2018)); the weighted form follows by conjugating Z_u Z_v through one QAOA layer
with the conventions of Sec. 2.2 (U_P = exp(-i gamma H), U_B = prod exp(-i beta X))
and the MaxCut H of Sec. 2.4.

With N'_u = N(u) minus {v}, N'_v = N(v) minus {u}, L = N'_u intersect N'_v and
c_xy = cos(gamma w_xy):
  <ZZ> = -1/2 sin(4 beta) sin(gamma w_uv) [prod_{k in N'_u} c_uk + prod_{k in N'_v} c_vk]
         + 1/2 sin^2(2 beta) prod_{k in N'_u - L} c_uk prod_{k in N'_v - L} c_vk
           [prod_{k in L} cos gamma (w_uk - w_vk) - prod_{k in L} cos gamma (w_uk + w_vk)]
"""
from __future__ import annotations

import numpy as np


def zz_p1(n, edges, weights, u: int, v: int, gamma: float, beta: float) -> float:
    wmap = {}
    for i, (a, b) in enumerate(np.asarray(edges).reshape(-1, 2).tolist()):
        wab = 1.0 if weights is None else float(weights[i])
        wmap[(a, b)] = wab
        wmap[(b, a)] = wab
    nbr = {x: set() for x in range(n)}
    for (a, b) in wmap:
        nbr[a].add(b)
    nu = nbr[u] - {v}
    nv = nbr[v] - {u}
    common = nu & nv
    wuv = wmap[(u, v)]
    cu = np.prod([np.cos(gamma * wmap[(u, k)]) for k in nu]) if nu else 1.0
    cv = np.prod([np.cos(gamma * wmap[(v, k)]) for k in nv]) if nv else 1.0
    term1 = -0.5 * np.sin(4 * beta) * np.sin(gamma * wuv) * (cu + cv)
    cu_only = np.prod([np.cos(gamma * wmap[(u, k)]) for k in nu - common]) if nu - common else 1.0
    cv_only = np.prod([np.cos(gamma * wmap[(v, k)]) for k in nv - common]) if nv - common else 1.0
    dif = np.prod([np.cos(gamma * (wmap[(u, k)] - wmap[(v, k)])) for k in common]) if common else 1.0
    summ = np.prod([np.cos(gamma * (wmap[(u, k)] + wmap[(v, k)])) for k in common]) if common else 1.0
    term2 = 0.5 * np.sin(2 * beta) ** 2 * cu_only * cv_only * (dif - summ)
    return float(term1 + term2)
