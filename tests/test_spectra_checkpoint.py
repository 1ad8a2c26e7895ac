"""Checkpoint / resume of the spectra and angular sweeps: one JSONL record per
(a, lambda, theta, phi, polarisation, variant) solve, appended as each study
group returns; a restart reads the file back and solves only what is missing.
The solver is replaced by a deterministic stand-in (host only): what is checked
is which solves run, what is stored and that the reductions come out the same
as for an uninterrupted sweep."""
import json

import pytest

import gpu_cases as G
from paper_1809_05334_amd import spectra_study as SS
from paper_1809_05334_amd.serve import Result


def fake_run(reqs, **kw):
    """Absorptances as a smooth function of the request's parameters."""
    out = []
    for rq in reqs:
        _, var, pol = rq["tag"]
        base = rq["lambda"] * 1e-3 + 0.1 * rq["theta"] + 0.01 * pol + (0.2 if var == "particle" else 0.0)
        out.append(Result(rid=rq["rid"], N=123, A=[0.0, base, 2.0 * base], R=0.1, T=0.2, iters=7))
    return out


class Counting:
    def __init__(self, fail_after=None, bad=None):
        self.calls, self.fail_after, self.bad = [], fail_after, bad or set()

    def __call__(self, reqs, **kw):
        if self.fail_after is not None and len(self.calls) >= self.fail_after:
            raise KeyboardInterrupt("interrupted")
        self.calls.append([SS.solve_key(kw["a_nm"], rq) for rq in reqs])
        res = fake_run(reqs)
        for r, rq in zip(res, reqs):
            if SS.solve_key(kw["a_nm"], rq) in self.bad:
                r.ok, r.error = False, "GMRES did not converge"
        return res


def groups():
    mesh = G.osc_small()
    return [(40.0, SS.study_requests(mesh, [(lam, 0.0) for lam in (500.0, 550.0)])),
            (40.0, SS.study_requests(mesh, [(600.0, th) for th in (0.0, 20.0, 40.0)]))]


def sweep(ckpt, run):
    out = []
    for a, reqs in groups():
        res = SS.run_with_checkpoint(a, reqs, ckpt, lambda rr, **kw: run(rr, a_nm=a, **kw))
        out.append(SS.reduce_active(reqs, res))
    return out


def test_resume_skips_recorded_solves(tmp_path):
    path = str(tmp_path / "study.jsonl")
    ref = sweep(SS.Checkpoint(""), Counting())

    first = Counting(fail_after=1)
    with pytest.raises(KeyboardInterrupt):
        sweep(SS.Checkpoint(path), first)
    g0 = groups()[0][1]
    assert len(first.calls) == 1 and len(first.calls[0]) == len(g0) == 8    # 2 lambdas x 2 variants x TE/TM
    lines = open(path).read().splitlines()
    assert len(lines) == 8
    assert all(len(json.loads(l)["key"]) == 6 for l in lines)
    with open(path, "a") as f:                      # a write cut off mid-line
        f.write('{"key": [40.0, 600.0, 0.0, 0.0, 0, "none"], "N": 12')

    second = Counting()
    got = sweep(SS.Checkpoint(path), second)
    assert len(second.calls) == 1                   # the first group came entirely from the file
    assert len(second.calls[0]) == 12               # 3 angles x 2 variants x TE/TM, the cut-off one included
    assert got == ref

    third = Counting()
    assert sweep(SS.Checkpoint(path), third) == ref
    assert third.calls == []                        # nothing left to solve


def test_failed_solves_are_not_recorded(tmp_path):
    path = str(tmp_path / "study.jsonl")
    a, reqs = groups()[0]
    bad = {SS.solve_key(a, reqs[3])}
    run = Counting(bad=bad)
    with pytest.raises(RuntimeError, match="did not converge"):
        sweep(SS.Checkpoint(path), run)
    ck = SS.Checkpoint(path)
    assert len(ck.done) == 7 and not (bad & set(ck.done))
    again = Counting()
    sweep(SS.Checkpoint(path), again)
    assert again.calls[0] == [SS.solve_key(a, reqs[3])]     # only the failed solve runs again


def test_keys_distinguish_every_parameter():
    mesh = G.osc_small()
    reqs = SS.study_requests(mesh, [(500.0, 0.0), (500.0, 20.0), (520.0, 0.0)])
    keys = {SS.solve_key(40.0, rq) for rq in reqs} | {SS.solve_key(60.0, rq) for rq in reqs}
    assert len(keys) == 2 * len(reqs)
    k = SS.solve_key(40.0, reqs[4])                          # case 1: theta 20 deg
    assert tuple(json.loads(json.dumps(list(k)))) == k      # survives the JSON round trip
    assert k[2] == pytest.approx(20.0)
