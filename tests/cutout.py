"""Cut-outs of a grid around sample zones, for checking multi-step results at
full size against the oracle one small block at a time (index bookkeeping
only; none of the method's arithmetic).

A zone's new value after one step depends on the zones within three of it
along every axis (reconstruction radius two plus one face neighbour), so
after s steps on a cut-out whose edges lie at least 3 s zones beyond the
sampled zones, those zones hold exactly the whole-grid result.  Along an
outflow axis the cut-out stops at the domain boundary, where it keeps the
real boundary condition; along a periodic axis it wraps.  Edges that cut
through the domain get an outflow boundary, which only reaches zones that
are not sampled."""
import numpy as np

import icgen


def cutout(pb, lo, hi, hw):
    """Block of pb holding the zones lo..hi (inclusive, (i, j, k)) plus hw
    zones on every side.  Returns (problem, where) with where(i, j, k) the
    position (i', j', k') of a zone of the original grid inside the block."""
    ids, bcs = [], []
    for ax in range(pb.ndim):
        n = pb.n[ax]
        a, b = lo[ax] - hw, hi[ax] + hw
        if pb.bc[ax] == "periodic":
            if b - a + 1 >= n:
                ids.append(np.arange(n))
                bcs.append("periodic")
            else:
                ids.append(np.arange(a, b + 1) % n)
                bcs.append("outflow")
        else:
            ids.append(np.arange(max(a, 0), min(b, n - 1) + 1))
            bcs.append("outflow")
    if pb.ndim == 3:
        U = pb.U[:, ids[2]][:, :, ids[1]][:, :, :, ids[0]]
        nn = (len(ids[0]), len(ids[1]), len(ids[2]))
    else:
        U = pb.U[:, ids[1]][:, :, ids[0]]
        nn = (len(ids[0]), len(ids[1]), 1)
        bcs.append("outflow")
    pos = [{int(g): p for p, g in enumerate(a)} for a in ids]

    def where(i, j, k=0):
        out = [pos[0][i], pos[1][j]]
        out.append(pos[2][k] if pb.ndim == 3 else 0)
        return tuple(out)

    sub = icgen.Problem(U=np.ascontiguousarray(U), ndim=pb.ndim, n=nn, h=pb.h, origin=pb.origin,
                        bc=tuple(bcs), gamma=pb.gamma, meta=dict(pb.meta, cutout=(tuple(lo), tuple(hi), hw)))
    return sub, where
