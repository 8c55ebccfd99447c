"""Host-side tile simulator (test infrastructure).

Executes a chain of toy loops twice in numpy: once untiled (every loop over its
full range, in program order) and once following the library's plan exactly
as the device pipeline would: per tile, a NaN-poisoned slot buffer per field,
the edge copy from the previous tile's slot, the planned uploads, every loop
over its planned rows of that tile, then the planned downloads.  Any missing
upload or edge row, or a wrong skew, shows up as a NaN or a difference.

The toy kernels are defined here (not in the library and not in the oracle):
  AVG      out = c0 * mean_k in(p + o_k) + c1
  INC_ADD  out = out + c * in
  MIRROR   dst_q = sign_q * src_q(p + o_q)
  FILL     dst = value
"""
import numpy as np

K_MIRROR, K_FILL, K_AVG, K_INC_ADD = 1, 2, 4, 5


class ToyLoop:
    def __init__(self, kid, rng, dats, consts):
        self.kid, self.rng, self.dats, self.consts = kid, rng, dats, consts  # dats: (field, access, offsets)


def apply_loop(loop, get, put, rows):
    """Run one toy loop over x-range x its rows (a (lo, hi) along y)."""
    (x0, x1), _ = loop.rng
    j0, j1 = rows
    if j1 <= j0 or x1 <= x0:
        return
    J, I = np.meshgrid(np.arange(j0, j1), np.arange(x0, x1), indexing="ij")
    if loop.kid == K_AVG:
        (fo, _, _), (fi, _, offs) = loop.dats
        s = np.zeros(J.shape)
        for (ox, oy) in offs:
            s = s + get(fi, I + ox, J + oy)
        put(fo, I, J, loop.consts[0] * (s / float(len(offs))) + loop.consts[1])
    elif loop.kid == K_INC_ADD:
        (fo, _, _), (fi, _, _) = loop.dats
        put(fo, I, J, get(fo, I, J) + loop.consts[0] * get(fi, I, J))
    elif loop.kid == K_MIRROR:
        vals = []
        for q in range(len(loop.dats) // 2):
            fs, _, offs = loop.dats[2 * q + 1]
            ox, oy = offs[0]
            vals.append(loop.consts[q] * get(fs, I + ox, J + oy))
        for q in range(len(loop.dats) // 2):
            put(loop.dats[2 * q][0], I, J, vals[q])
    elif loop.kid == K_FILL:
        put(loop.dats[0][0], I, J, np.full(J.shape, loop.consts[0]))
    else:
        raise ValueError(loop.kid)


def run_untiled(loops, host, H):
    arr = {f: a.copy() for f, a in host.items()}

    def get(f, I, J):
        return arr[f][J + H, I + H]

    def put(f, I, J, v):
        arr[f][J + H, I + H] = v

    for lp in loops:
        apply_loop(lp, get, put, lp.rng[1])
    return arr


def run_tiled(loops, host, plan, H, slots):
    """Follow the plan; returns the host arrays after all downloads."""
    T = plan["ntiles"]
    res = plan["resident"]
    arr = {f: a.copy() for f, a in host.items()}
    ncols = {f: a.shape[1] for f, a in host.items()}
    used = sorted(set(f for lp in loops for (f, _, _) in lp.dats))
    cap = {f: int(max(res[f, t, 1] - res[f, t, 0] for t in range(T))) for f in used}
    slot = {}  # (s, f) -> array
    up = {t: [r for r in plan["up"] if r[1] == t] for t in range(T)}
    down = {t: [r for r in plan["down"] if r[1] == t] for t in range(T)}
    edge = {t: [r for r in plan["edge"] if r[1] == t] for t in range(T)}
    for t in range(T):
        s = t % slots
        for f in used:
            slot[(s, f)] = np.full((max(cap[f], 1), ncols[f]), np.nan)
        if t > 0:
            ps = (t - 1) % slots
            for f, _, r0, r1 in edge[t]:
                A0, A1 = res[f, t - 1, 0], res[f, t, 0]
                slot[(s, f)][r0 - A1:r1 - A1] = slot[(ps, f)][r0 - A0:r1 - A0]
        for f, _, r0, r1 in up[t]:
            A = res[f, t, 0]
            slot[(s, f)][r0 - A:r1 - A] = arr[f][r0:r1]

        def get(f, I, J, t=t, s=s):
            A, B = res[f, t, 0], res[f, t, 1]
            r = J + H
            assert (r >= A).all() and (r < B).all(), "read outside the rows held for tile %d" % t
            return slot[(s, f)][r - A, I + H]

        def put(f, I, J, v, t=t, s=s):
            A, B = res[f, t, 0], res[f, t, 1]
            r = J + H
            assert (r >= A).all() and (r < B).all(), "write outside the rows held for tile %d" % t
            slot[(s, f)][r - A, I + H] = v

        for i, lp in enumerate(loops):
            a, b = plan["loop_rows"][i, t]
            apply_loop(lp, get, put, (a, b))
        for f, _, r0, r1 in down[t]:
            A = res[f, t, 0]
            arr[f][r0:r1] = slot[(s, f)][r0 - A:r1 - A]
    return arr


# ---- the same in 3D: loops tiled along z, arrays indexed [k, j, i]

def apply_loop3(loop, get, put, rows):
    """Run one toy loop over its x and y ranges x its planes (a (lo, hi) along z)."""
    (x0, x1), (y0, y1), _ = loop.rng
    k0, k1 = rows
    if k1 <= k0 or x1 <= x0 or y1 <= y0:
        return
    K, J, I = np.meshgrid(np.arange(k0, k1), np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
    if loop.kid == K_AVG:
        (fo, _, _), (fi, _, offs) = loop.dats
        s = np.zeros(K.shape)
        for (ox, oy, oz) in offs:
            s = s + get(fi, I + ox, J + oy, K + oz)
        put(fo, I, J, K, loop.consts[0] * (s / float(len(offs))) + loop.consts[1])
    elif loop.kid == K_INC_ADD:
        (fo, _, _), (fi, _, _) = loop.dats
        put(fo, I, J, K, get(fo, I, J, K) + loop.consts[0] * get(fi, I, J, K))
    elif loop.kid == K_MIRROR:
        vals = []
        for q in range(len(loop.dats) // 2):
            fs, _, offs = loop.dats[2 * q + 1]
            ox, oy, oz = offs[0]
            vals.append(loop.consts[q] * get(fs, I + ox, J + oy, K + oz))
        for q in range(len(loop.dats) // 2):
            put(loop.dats[2 * q][0], I, J, K, vals[q])
    elif loop.kid == K_FILL:
        put(loop.dats[0][0], I, J, K, np.full(K.shape, loop.consts[0]))
    else:
        raise ValueError(loop.kid)


def run_untiled3(loops, host, H):
    arr = {f: a.copy() for f, a in host.items()}

    def get(f, I, J, K):
        return arr[f][K + H, J + H, I + H]

    def put(f, I, J, K, v):
        arr[f][K + H, J + H, I + H] = v

    for lp in loops:
        apply_loop3(lp, get, put, lp.rng[2])
    return arr


def run_tiled3(loops, host, plan, H, slots):
    """Follow the plan along z; returns the host arrays after all downloads."""
    T = plan["ntiles"]
    res = plan["resident"]
    arr = {f: a.copy() for f, a in host.items()}
    used = sorted(set(f for lp in loops for (f, _, _) in lp.dats))
    cap = {f: int(max(res[f, t, 1] - res[f, t, 0] for t in range(T))) for f in used}
    slot = {}
    up = {t: [r for r in plan["up"] if r[1] == t] for t in range(T)}
    down = {t: [r for r in plan["down"] if r[1] == t] for t in range(T)}
    edge = {t: [r for r in plan["edge"] if r[1] == t] for t in range(T)}
    for t in range(T):
        s = t % slots
        for f in used:
            slot[(s, f)] = np.full((max(cap[f], 1),) + host[f].shape[1:], np.nan)
        if t > 0:
            ps = (t - 1) % slots
            for f, _, r0, r1 in edge[t]:
                A0, A1 = res[f, t - 1, 0], res[f, t, 0]
                slot[(s, f)][r0 - A1:r1 - A1] = slot[(ps, f)][r0 - A0:r1 - A0]
        for f, _, r0, r1 in up[t]:
            A = res[f, t, 0]
            slot[(s, f)][r0 - A:r1 - A] = arr[f][r0:r1]

        def get(f, I, J, K, t=t, s=s):
            A, B = res[f, t, 0], res[f, t, 1]
            r = K + H
            assert (r >= A).all() and (r < B).all(), "read outside the planes held for tile %d" % t
            return slot[(s, f)][r - A, J + H, I + H]

        def put(f, I, J, K, v, t=t, s=s):
            A, B = res[f, t, 0], res[f, t, 1]
            r = K + H
            assert (r >= A).all() and (r < B).all(), "write outside the planes held for tile %d" % t
            slot[(s, f)][r - A, J + H, I + H] = v

        for i, lp in enumerate(loops):
            a, b = plan["loop_rows"][i, t]
            apply_loop3(lp, get, put, (a, b))
        for f, _, r0, r1 in down[t]:
            A = res[f, t, 0]
            arr[f][r0:r1] = slot[(s, f)][r0 - A:r1 - A]
    return arr


# ---- ring slabs: one ring per field, stored row (plane) r at position r mod R

def run_tiled_ring(loops, host, plan, H, slots, ndim=2):
    """Follow a ring-slab plan (OOC_FLAG_RING) in 2D (ndim=2: rows) or 3D
    (planes): per field one ring of plan["ring_rows"] rows, stored row r at
    position r mod R.  The rows a tile brings in are NaN-poisoned before its
    uploads; the rows two tiles share stay where they are (no edge copy).
    Also checks that each ring holds the rows of any `slots` consecutive
    tiles (the tiles the pipeline can have in flight)."""
    T = plan["ntiles"]
    res = plan["resident"]
    R = plan["ring_rows"]
    assert plan["ring"]
    arr = {f: a.copy() for f, a in host.items()}
    used = sorted(set(f for lp in loops for (f, _, _) in lp.dats))
    ring = {f: np.full((max(int(R[f]), 1),) + host[f].shape[1:], np.nan) for f in used}
    up = {t: [r for r in plan["up"] if r[1] == t] for t in range(T)}
    down = {t: [r for r in plan["down"] if r[1] == t] for t in range(T)}
    pos = lambda f, r: np.asarray(r) % int(R[f])
    for t in range(T):
        for f in used:
            A, B = res[f, t]
            if B <= A:
                continue
            held = [res[f, u] for u in range(max(0, t - slots + 1), t + 1) if res[f, u, 1] > res[f, u, 0]]
            assert max(b for _, b in held) - min(a for a, _ in held) <= R[f], \
                "ring of field %d too small for %d tiles in flight at tile %d" % (f, slots, t)
            prev = t > 0 and res[f, t - 1, 1] > res[f, t - 1, 0]
            new0 = max(A, res[f, t - 1, 1]) if prev else A
            if new0 < B:
                ring[f][pos(f, np.arange(new0, B))] = np.nan
        for f, _, r0, r1 in up[t]:
            ring[f][pos(f, np.arange(r0, r1))] = arr[f][r0:r1]

        if ndim == 2:
            def get(f, I, J, t=t):
                r = J + H
                assert (r >= res[f, t, 0]).all() and (r < res[f, t, 1]).all()
                return ring[f][pos(f, r), I + H]

            def put(f, I, J, v, t=t):
                r = J + H
                assert (r >= res[f, t, 0]).all() and (r < res[f, t, 1]).all()
                ring[f][pos(f, r), I + H] = v

            for i, lp in enumerate(loops):
                apply_loop(lp, get, put, tuple(plan["loop_rows"][i, t]))
        else:
            def get(f, I, J, K, t=t):
                r = K + H
                assert (r >= res[f, t, 0]).all() and (r < res[f, t, 1]).all()
                return ring[f][pos(f, r), J + H, I + H]

            def put(f, I, J, K, v, t=t):
                r = K + H
                assert (r >= res[f, t, 0]).all() and (r < res[f, t, 1]).all()
                ring[f][pos(f, r), J + H, I + H] = v

            for i, lp in enumerate(loops):
                apply_loop3(lp, get, put, tuple(plan["loop_rows"][i, t]))
        for f, _, r0, r1 in down[t]:
            arr[f][r0:r1] = ring[f][pos(f, np.arange(r0, r1))]
    return arr
