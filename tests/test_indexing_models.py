"""CPU models of the multi-step kernels' and the fused reverse step's index
arithmetic (no GPU).

The stationary multi-step kernel (stepk.hpp) stages a region of 2048
positions, advances it up to 16 steps in LDS and writes its tile; the halo it
recomputes must hold everything the tile's nodes depend on.  The model below
follows the kernel's placement of a block (its tile, the last tile of a
Dirichlet or Neumann instance moved back to end at node N - 1, the halo
upstream of one-sided windows), marks which region positions hold valid
values after each stencil application (interior windows, the Dirichlet pass
over the kernel's list of clamped nodes, held ends, Neumann mirrors), and
checks that every node of every tile is valid after the launch's steps, that
every window read stays inside the LDS array with its margins, and that each
node of the grid is written by some block.  Run with the placement of every
tile at b * tile, the model finds the instances whose last tile starts next to
a Dirichlet end -- the error the placement fixes.
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest

REGION = 2048
MARGIN = 16


def stepk_apps(scheme, nonlin):
    rk2n = scheme == "etd2rk" and nonlin != "none"
    return (2 if rk2n else 1) * (2 if scheme != "linear" and nonlin == "kdv" else 1)


def interior_offset(n, side):
    return {0: -((n - 1) // 2), 1: -(n - 1), 2: 0}[side]


def window_offset(i, N, n, bc, side):
    o = interior_offset(n, side)
    if bc == "dirichlet":
        o = max(o, -i)
        o = min(o, N - n - i)
    return o


def node_of(j, N, bc):
    """Vectorised: the node whose value sits at unwrapped position j."""
    j = np.asarray(j)
    if bc == "periodic":
        return j % N
    if bc == "neumann":
        P2 = 2 * (N - 1)
        m = j % P2 if P2 > 0 else np.zeros_like(j)
        return np.where(m > N - 1, P2 - m, m)
    return np.clip(j, 0, N - 1)


def edge_nodes(N, n, side):
    R = (n - 1) // 2
    if side == 0:
        return [e if e < R else N - 1 - (e - R) for e in range(n - 1)]
    if side == 1:
        return [e if e < n - 1 else N - 1 for e in range(n)]
    return [N - 1 - e if e < n - 1 else 0 for e in range(n)]


def model_block(b, N, n, bc, side, scheme, nonlin, kb, ksteps, move_back=True):
    """Validity of the region after ksteps steps; returns (tile range, ok)."""
    apps = stepk_apps(scheme, nonlin)
    R = (n - 1) // 2
    tile = REGION - 2 * kb * apps * R
    O = interior_offset(n, side)
    lhalo = kb * apps * (-O)
    tb = b * tile
    t0 = N - tile if (move_back and bc != "periodic" and N >= tile and tb > N - tile) else tb
    base = t0 - lhalo
    q = np.arange(REGION)
    j = base + q
    inside = (j >= 0) & (j <= N - 1)
    valid = inside.copy() if bc == "dirichlet" else np.ones(REGION, bool)
    at_end = base < n or base + REGION > N - n
    # every window read of the interior pass stays inside the array and margins
    assert -MARGIN <= O and O + n - 1 <= MARGIN
    edges = [i for i in edge_nodes(N, n, side) if 0 <= i - base < REGION] if (bc == "dirichlet" and at_end) else []
    if bc == "dirichlet":
        # the interior pass is right only where the node's own window is the
        # interior one; the kernel's list of clamped nodes must cover the rest
        true_off = np.minimum(np.maximum(O, -j), N - n - j)
        wrong = inside & (true_off != O)
        wrong[[i - base for i in edges]] = False
    if bc == "neumann" and at_end:
        outside = ~inside
        src = node_of(j, N, bc) - base
        src_ok = (src >= 0) & (src < REGION)
        src_c = np.clip(src, 0, REGION - 1)
    lo, hi = max(0, -O), min(REGION, REGION - (O + n - 1))  # windows inside the staged region
    for _ in range(ksteps * apps):
        bad = np.concatenate(([0], np.cumsum(~valid)))
        new = np.zeros(REGION, bool)
        qq = np.arange(lo, hi)
        new[lo:hi] = (bad[qq + O + n] - bad[qq + O]) == 0
        if bc == "dirichlet":
            new &= inside  # positions outside the grid hold no node
            new[wrong] = False
            upd = {}
            for i in edges:
                if i in (0, N - 1):
                    upd[i - base] = True  # held end
                    continue
                off = min(max(-((n - 1) // 2) if side == 0 else (-(n - 1) if side == 1 else 0), -i), N - n - i)
                b0 = min(max(i + off - base, -MARGIN), REGION + MARGIN - n)
                upd[i - base] = all(0 <= b0 + k < REGION and valid[b0 + k] for k in range(n))
            for k, v in upd.items():
                new[k] = v
        elif bc == "neumann" and at_end:
            new[outside] = src_ok[outside] & new[src_c[outside]]
        valid = new
    lo_t, hi_t = t0, min(t0 + tile, N)
    ok = bool(np.all(valid[lo_t - base:hi_t - base])) if hi_t > lo_t else True
    return (lo_t, hi_t), ok


def check_instance(N, n, bc, side, scheme, nonlin, kb, ksteps, move_back=True):
    apps = stepk_apps(scheme, nonlin)
    tile = REGION - 2 * kb * apps * ((n - 1) // 2)
    blocks = -(-N // tile)
    covered = np.zeros(N, bool)
    bad = []
    for b in range(blocks):
        (lo, hi), ok = model_block(b, N, n, bc, side, scheme, nonlin, kb, ksteps, move_back)
        covered[lo:hi] = True
        if not ok:
            bad.append(b)
    return bad, bool(covered.all())


def _sizes(n, tile):
    R = (n - 1) // 2
    out = {n, n + 1, 2 * n + 3, 700, tile - 1, tile, tile + 1, tile + 2, tile + R, tile + n, 2 * tile + 3,
           3 * tile - 1}
    return sorted(x for x in out if x >= n)


CONFIGS = [(scheme, nonlin) for scheme, nonlin in
           [("linear", "none"), ("etd1", "allen_cahn"), ("etd2rk", "allen_cahn"), ("etd1", "kdv"),
            ("etd2rk", "kdv")]]


@pytest.mark.parametrize("side", [0, 1, 2])
@pytest.mark.parametrize("bc", ["periodic", "dirichlet", "neumann"])
def test_stepk_tiles_hold_their_dependencies(side, bc):
    """Every tile node is valid after the launch's steps, for 1, 4 and 16
    steps per launch (a shorter last launch spoils less), every scheme's
    number of stencil passes, n = 3 .. 15 and sizes around the tile
    boundaries."""
    failures = []
    for n in (3, 7, 9, 15):
        for (scheme, nonlin), kb in itertools.product(CONFIGS, (1, 4, 16)):
            apps = stepk_apps(scheme, nonlin)
            tile = REGION - 2 * kb * apps * ((n - 1) // 2)
            if tile <= 0:
                continue
            for N in _sizes(n, tile):
                bad, covered = check_instance(N, n, bc, side, scheme, nonlin, kb, kb)
                if bad or not covered:
                    failures.append((n, scheme, nonlin, kb, N, bad, covered))
    assert not failures, failures[:5]


def test_model_finds_the_last_tile_error():
    """With every tile placed at b * tile the model finds the Dirichlet
    instances whose last tile starts next to the end (the clamped window of
    node N - 2 reads n - 1 nodes inwards), and with the kernel's placement it
    does not."""
    n, kb = 15, 1
    tile = REGION - 2 * kb * ((n - 1) // 2)
    for N in (tile + 2, tile + 3):
        bad, _ = check_instance(N, n, "dirichlet", 0, "linear", "none", kb, kb, move_back=False)
        assert bad, N
        bad, covered = check_instance(N, n, "dirichlet", 0, "linear", "none", kb, kb)
        assert not bad and covered, N
    # one-sided windows starting at the node, Neumann ends: the mirrors of the
    # last nodes lie before a tile that starts there
    tile4 = REGION - 2 * 4 * 4
    bad, _ = check_instance(tile4 + 3, 9, "neumann", 2, "linear", "none", 4, 4, move_back=False)
    assert bad
    bad, covered = check_instance(tile4 + 3, 9, "neumann", 2, "linear", "none", 4, 4)
    assert not bad and covered


# --------------------------------------------------------------------------
# The fused reverse step (adjoint_taylor.hip): one block of 2 x 256 threads
# per tile of 256 - 4 (n - 1) nodes, 256 weight positions, each worked on by
# two threads (its W0 and W1 sides) with the same index arithmetic; the model
# replays that arithmetic position by position: every LDS index in bounds, and
# every value read is one that was staged or computed (a staged position the
# load covered, a weight slot whose node was active, a ghat slot in the range
# step 3 fills), for every stencil size, boundary type and tile position.

ADJ_T = 256


def _map_index(j, N, bc):
    if bc == "periodic":
        return j % N
    if bc == "neumann":
        j = -j if j < 0 else j
        return 2 * (N - 1) - j if j > N - 1 else j
    return j


def _window_offset_c(i, N, n, bc):
    o = -((n - 1) // 2)
    if bc == "dirichlet":
        o = max(o, -i)
        o = min(o, N - n - i)
    return o


def _stencils_containing(j, N, n, bc):
    R = (n - 1) // 2
    ps = [j]
    if bc == "neumann":
        if 0 < j <= 2 * R:
            ps.append(-j)
        if N - 1 > j >= N - 1 - 2 * R:
            ps.append(2 * (N - 1) - j)
    out = []
    for p in ps:
        for d in range(-(n - 1), n):
            x = p + d
            i = x
            if bc == "periodic":
                i = _map_index(x, N, bc)
            elif i < 0 or i > N - 1:
                continue
            if bc == "dirichlet" and i in (0, N - 1):
                continue
            k = -d - _window_offset_c(i, N, n, bc)
            if 0 <= k < n:
                out.append((x if bc == "periodic" else i, k))
    return out


def adj_tile_problems(N, n, bc, tile):
    """Problems found in tile `tile` of an instance (empty: none)."""
    T = ADJ_T
    R = (n - 1) // 2
    H = n - 1
    HW = 2 * H
    TO = T - 2 * HW
    SU = T + 2 * H
    t0 = tile * TO
    base = t0 - HW
    per, dr = bc == "periodic", bc == "dirichlet"
    holds = lambda x: per or 0 <= x < N
    errs = []
    staged = []
    for q in range(SU):
        x = base - H + q
        staged.append(per or ((0 <= x < N) if dr else (-(N - 1) <= x <= 2 * (N - 1))))
    computed = [False] * T
    for thread in range(2 * T):  # step 2: both sides of every position
        side = 1 if thread >= T else 0
        tid = thread - side * T
        if not 0 <= tid < T:
            errs.append(("step2 slot", thread))
            continue
        x = base + tid
        active = holds(x)
        i = _map_index(x, N, bc) if active else (t0 if t0 < N else N - 1)
        xs = x if active else i
        us0 = xs - (base - H)
        o = _window_offset_c(i, N, n, bc)
        for j in [0] + [o + k for k in range(n)]:
            if not 0 <= us0 + j < SU:
                errs.append(("step2 bounds", tid))
            elif active and not staged[us0 + j]:
                errs.append(("step2 unstaged", tid))
        computed[tid] = active

    def weight_slot_ok(q):
        return 0 <= q < T and computed[q] and 0 <= q + H < SU and staged[q + H]

    ghat = [False] * T
    for tid in range(H, T - H):  # step 3 (frozen-velocity ghat; run by thread T + tid, the W1 side)
        m = base + tid
        if not holds(m):
            ghat[tid] = True  # written as 0 and read only as such
            continue
        mi = _map_index(m, N, bc)
        if mi >= 2 * (n - 1) and mi <= N - 1 - 2 * (n - 1):
            terms = [(m + d, R - d) for d in range(-R, R + 1)]
        else:
            terms = _stencils_containing(m if per else mi, N, n, bc)
        ok = True
        for x, k in terms:
            if not weight_slot_ok(x - base):
                errs.append(("step3", tid, x))
                ok = False
        ghat[tid] = ok
    for tid in range(TO):  # step 4
        j = t0 + tid
        if j >= N:
            continue
        qj = HW + tid
        inner = j >= 2 * (n - 1) and j <= N - 1 - 2 * (n - 1)
        terms = [(j + d, R - d) for d in range(-R, R + 1)] if inner else _stencils_containing(j, N, n, bc)
        for x, k in terms:
            if not weight_slot_ok(x - base):
                errs.append(("step4 gather", tid, x))
        if not (dr and j in (0, N - 1)):
            o = _window_offset_c(j, N, n, bc)
            for k in range(n):
                s = qj + H + o + k
                if not (0 <= s < SU and staged[s]):
                    errs.append(("step4 own window", tid))
        if inner:
            slots = [qj + d for d in range(-R, R + 1)]
        else:
            ps = [j]
            if bc == "neumann":
                if 0 < j <= 2 * R:
                    ps.append(-j)
                if N - 1 > j >= N - 1 - 2 * R:
                    ps.append(2 * (N - 1) - j)
            slots = []
            for p in ps:
                for d in range(-(n - 1), n):
                    x = p + d
                    m = x
                    if per:
                        m = _map_index(x, N, bc)
                    elif m < 0 or m > N - 1:
                        continue
                    l = -d - _window_offset_c(m, N, n, bc)
                    if 0 <= l < n:
                        slots.append((x if per else m) - base)
        for s in slots:
            if not (H <= s < T - H and ghat[s]):
                errs.append(("step4 ghat", tid, s))
    return errs


@pytest.mark.parametrize("bc", ["periodic", "dirichlet", "neumann"])
def test_fused_reverse_step_indexing(bc):
    failures = []
    for n in (3, 5, 9, 15):
        TO = ADJ_T - 4 * (n - 1)
        for N in sorted({n, n + 1, 2 * n + 1, 4 * n, TO - 1, TO, TO + 1, TO + n, 2 * TO + 3}):
            if N < n:
                continue
            for tile in range(-(-N // TO)):
                e = adj_tile_problems(N, n, bc, tile)
                if e:
                    failures.append((n, N, tile, e[:3]))
    assert not failures, failures[:3]
