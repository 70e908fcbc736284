"""The autotuner's search logic without a GPU: batch signatures, the candidate
set the library accepts, selection of the fastest agreeing candidate, and the
JSON cache."""
from __future__ import annotations

import json

import numpy as np

import workloads
from paper_2603_15964_amd import tune
from paper_2603_15964_amd._native import (LMEP_EXP_AUTO, LMEP_EXP_PADE, LMEP_F_PERSISTENT, LMEP_OPT_APPLY_TILE,
                                          LMEP_OPT_EXP_METHOD, LMEP_OPT_FUSE_FROZEN, LMEP_OPT_STEPS_PER_LAUNCH,
                                          LMEP_OPT_MERGE_GROUPS, LMEP_OPT_TAYLOR_REGION)


def _opts(c):
    return dict(c.options)


def test_signature_groups_and_size_classes():
    ps, _ = workloads.allen_cahn_batch(count=40, n_min=512, n_max=2000)
    s1 = tune.signature(ps)
    assert s1 == tune.signature(list(reversed(ps)))  # order does not matter
    assert len(s1.split(";")) == len({(p["n"], p["bc"]) for p in ps})
    p, _ = workloads.burgers(N=5000)
    q, _ = workloads.burgers(N=7000)
    assert tune.signature([p]) == tune.signature([q])  # same power-of-two class
    r, _ = workloads.burgers(N=9000)
    assert tune.signature([p]) != tune.signature([r])


def test_candidates_follow_what_the_library_accepts():
    frozen = [workloads.burgers(N=1000)[0]]
    c = tune.candidates(frozen)
    assert {_opts(x)[LMEP_OPT_FUSE_FROZEN] for x in c} == {0, 1}
    assert {_opts(x)[LMEP_OPT_EXP_METHOD] for x in c} == {LMEP_EXP_AUTO, LMEP_EXP_PADE}
    assert _opts(c[0])[LMEP_OPT_EXP_METHOD] == LMEP_EXP_AUTO  # the default comes first (reference result)
    # frozen velocity several steps per launch: the finite-Taylor multi-step
    # kernel only, at most 8 steps, with its region sized or forced
    pers = [x for x in c if x.flags & LMEP_F_PERSISTENT]
    assert {_opts(x)[LMEP_OPT_STEPS_PER_LAUNCH] for x in pers} == {1, 2, 4, 8}
    assert {_opts(x)[LMEP_OPT_TAYLOR_REGION] for x in pers} == {0, 256, 512}
    assert all(_opts(x)[LMEP_OPT_EXP_METHOD] == LMEP_EXP_AUTO for x in pers)
    neumann = [dict(frozen[0], bc="neumann")]
    assert not any(x.flags & LMEP_F_PERSISTENT for x in tune.candidates(neumann))
    stat = [workloads.kdv(N=4096)[0]]
    assert {_opts(x)[LMEP_OPT_EXP_METHOD] for x in tune.candidates(stat)} == {LMEP_EXP_AUTO}
    kbs = {_opts(x)[LMEP_OPT_STEPS_PER_LAUNCH] for x in tune.candidates(stat) if x.flags & LMEP_F_PERSISTENT}
    assert kbs == {1, 2, 4, 8, 16}
    assert all(LMEP_OPT_TAYLOR_REGION not in _opts(x) for x in tune.candidates(stat))
    assert all(LMEP_OPT_MERGE_GROUPS not in _opts(x) for x in tune.candidates(stat))  # one stencil size
    acb = workloads.allen_cahn_batch(count=12, n_min=600, n_max=3000)[0]
    merges = {(_opts(x)[LMEP_OPT_STEPS_PER_LAUNCH], _opts(x).get(LMEP_OPT_MERGE_GROUPS))
              for x in tune.candidates(acb) if x.flags & LMEP_F_PERSISTENT}
    assert (16, 0) in merges and (16, 1) in merges and (8, 1) in merges and (4, None) in merges
    upwind = [workloads.burgers_upwind(N=1000)[0]]  # frozen velocity: the multi-step Taylor kernel takes it
    assert any(x.flags & LMEP_F_PERSISTENT for x in tune.candidates(upwind))
    ac_upwind = [dict(workloads.allen_cahn_batch(count=1)[0][0], window="upwind")]  # one-sided stationary
    assert any(x.flags & LMEP_F_PERSISTENT for x in tune.candidates(ac_upwind))
    cheb = [workloads.allen_cahn_chebyshev()[0]]
    cc = tune.candidates(cheb)
    assert sum(1 for x in cc if x.flags & LMEP_F_PERSISTENT) == 1
    assert 64 in {_opts(x)[LMEP_OPT_APPLY_TILE] for x in cc}
    big = [dict(cheb[0], N=600, x=workloads.chebyshev(600))]
    assert not any(x.flags & LMEP_F_PERSISTENT for x in tune.candidates(big))


def test_search_picks_fastest_agreeing_and_caches(tmp_path):
    ps = [workloads.kdv(N=4096)[0]]
    cands = tune.candidates(ps)
    times = {c: 10.0 - i for i, c in enumerate(cands)}  # the last is fastest ...
    bad = cands[-1]                                       # ... but disagrees
    calls = []

    def measure(c):
        calls.append(c)
        return times[c], (np.ones(3) * (2.0 if c == bad else 1.0))

    def agree(a, b):
        return np.array_equal(a, b)

    path = str(tmp_path / "tune.json")
    r = tune.search(ps, measure, "gfx950", path, agree=agree)
    assert not r.from_cache and r.choice == cands[-2] and len(calls) == len(cands)
    data = json.load(open(path))
    assert len(data) == 1 and list(data)[0].startswith("gfx950|")
    r2 = tune.search(ps, measure, "gfx950", path, agree=agree)
    assert r2.from_cache and r2.choice == r.choice and len(calls) == len(cands)
    r3 = tune.search(ps, measure, "gfx950", path, refresh=True, agree=agree)
    assert not r3.from_cache and len(calls) == 2 * len(cands)
    r4 = tune.search(ps, measure, "gfx942", path, agree=agree)  # another architecture: its own entry
    assert not r4.from_cache and len(json.load(open(path))) == 2
