"""Batched mock ensembles through cola_ensemble_run: eager and hipGraph-captured.

Every realization of a batched class must match the same seed run alone (the batch only adds a
realization index to each launch), and every replay of the captured graph must match the eager
result.  Positions are compared at 1e-5 relative RMS and spectra at 1e-4 (the spectra's float64
bin sums are order-dependent); with the integer deposit, graph replays reproduce the eager
positions bit for bit, which the PM-only / sampled class checks.
"""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import cola as ocola, cosmology as ocosmo, power as opower  # noqa: E402
from paper_1509_04685_amd import workloads as W  # noqa: E402


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def cola():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_04685_amd as c
    yield c
    c.ensemble_release()


def rel_rms(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2) / np.mean(b ** 2)))


CLASSES = [dict(box=120.0, n_part=16, pm=3, seeds=(11, 12, 13), n_steps=6, a_out=(0.5, 1.0)),
           dict(box=150.0, n_part=24, pm=3, seeds=(21, 22), n_steps=6, a_out=(1.0,))]


def build(cola, cosmo):
    spec = []
    for c in CLASSES:
        prob = cola.make_problem(c["box"], c["n_part"], c["pm"], 19.0, c["n_steps"], n_real=len(c["seeds"]))
        n_pk = c["n_part"] * c["pm"]
        spec.append(dict(prob=prob, seeds=c["seeds"], a_out=c["a_out"], n_pk=n_pk, n_bins=n_pk // 2))
    return cola.Ensemble(spec, cosmo)


def snapshot(ens):
    return [(it["state"].x.cpu().numpy().copy(), it["out"][1].cpu().numpy().copy()) for it in ens.items]


def test_ensemble_matches_single_runs(cola):
    say("ensemble eager vs single runs")
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    ens = build(cola, cosmo)
    ens.run(graph=False)
    torch.cuda.synchronize()
    for c, it in zip(CLASSES, ens.items):
        n = c["n_part"] ** 3
        for r, seed in enumerate(c["seeds"]):
            prob = cola.make_problem(c["box"], c["n_part"], c["pm"], 19.0, c["n_steps"])
            st = cola.ParticleState(prob)
            n_pk = c["n_part"] * c["pm"]
            ws = cola.Workspace(prob, n_pk=n_pk)
            cola.ic_2lpt(prob, cosmo, [seed], st, ws)
            tab = cola.schedule_table(prob, cosmo)
            for k, a in enumerate(c["a_out"]):
                j = int((tab[:, 0] <= a * (1 + 1e-12)).sum()) - 1
                if j > st.node:
                    cola.step(prob, cosmo, st, j, ws)
                _, pk, _ = cola.power_spectrum(prob, cosmo, st, a, n_pk, n_pk // 2, ws)
                got = it["out"][1][k, r].cpu().numpy()
                ref = pk.cpu().numpy()[0]
                sel = ref > 0
                assert np.abs(got[sel] / ref[sel] - 1).max() < 1e-4
            cola.step(prob, cosmo, st, c["n_steps"] - 1, ws)
            assert rel_rms(it["state"].x[:, r * n:(r + 1) * n].cpu().numpy(), st.x.cpu().numpy()) < 1e-5
        assert it["state"].node == c["n_steps"] - 1


def test_ensemble_first_realization_matches_oracle(cola):
    say("ensemble vs oracle")
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    ens = build(cola, cosmo)
    ens.run(graph=False)
    torch.cuda.synchronize()
    c, it = CLASSES[1], ens.items[1]
    op = ocola.Problem(c["box"], c["n_part"], c["pm"], 19.0, c["n_steps"])
    oc = ocosmo.Cosmology(**W.COSMOLOGY)
    ost, _ = ocola.run(op, oc, c["seeds"][1])
    n = c["n_part"] ** 3
    x = it["state"].x[:, n:2 * n].cpu().numpy()
    assert rel_rms(x, ost.disp) < 1e-3
    k, pk, cnt = opower.power_spectrum(ocola.positions(ost, op), c["n_part"] * c["pm"], c["box"], c["n_part"] * c["pm"] // 2)
    got = it["out"][1][0, 1].cpu().numpy()
    sel = cnt > 0
    assert np.abs(got[sel] / pk[sel] - 1).max() < 1e-3


def test_ensemble_graph_replays_match_eager(cola):
    say("ensemble graph replays")
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    ens = build(cola, cosmo)
    ens.run(graph=False)
    torch.cuda.synchronize()
    eager = snapshot(ens)
    # unrelated eager work on another problem between replays
    side_prob = cola.make_problem(64.0, 8, 3, 19.0, 4)
    side = cola.ParticleState(side_prob)
    side_ws = cola.Workspace(side_prob)
    for rep in range(3):
        for it in ens.items:  # scribble over the state: the graph must rebuild it from its ICs
            it["state"].x.fill_(123.0)
            it["out"][1].fill_(-1.0)
        ens.run(graph=True)
        torch.cuda.synchronize()
        got = snapshot(ens)
        for (xe, pe), (xg, pg) in zip(eager, got):
            assert rel_rms(xg, xe) < 1e-5, rep
            sel = pe > 0
            assert np.abs(pg[sel] / pe[sel] - 1).max() < 1e-4, rep
        cola.ic_2lpt(side_prob, cosmo, [rep + 1], side, side_ws)
        cola.pm_force(side_prob, side, side_ws)
        torch.cuda.synchronize()


def test_ensemble_pm_only_and_sampled_classes(cola):
    """A PM-only class with logarithmic nodes and a COLA class with a^0.8 nodes: batched runs
    match single runs, and graph replays reproduce the eager positions exactly."""
    say("ensemble with PM-only and sampled classes")
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    kinds = [dict(frame="pm", sampling="log", power=1.0, seeds=(31, 32)),
             dict(frame="cola", sampling="power", power=0.8, seeds=(41, 42))]
    spec = []
    for k in kinds:
        prob = cola.make_problem(120.0, 16, 3, 19.0, 6, n_real=2, sampling=k["sampling"],
                                 sampling_power=k["power"], frame=k["frame"])
        spec.append(dict(prob=prob, seeds=k["seeds"], a_out=(1.0,), n_pk=48, n_bins=24))
    ens = cola.Ensemble(spec, cosmo)
    ens.run(graph=False)
    torch.cuda.synchronize()
    eager = snapshot(ens)
    for k, it in zip(kinds, ens.items):
        n = 16 ** 3
        for r, seed in enumerate(k["seeds"]):
            prob = cola.make_problem(120.0, 16, 3, 19.0, 6, sampling=k["sampling"], sampling_power=k["power"],
                                     frame=k["frame"])
            st = cola.ParticleState(prob)
            ws = cola.Workspace(prob, n_pk=48)
            cola.ic_2lpt(prob, cosmo, [seed], st, ws)
            cola.step(prob, cosmo, st, 5, ws)
            assert rel_rms(it["state"].x[:, r * n:(r + 1) * n].cpu().numpy(), st.x.cpu().numpy()) < 1e-5
    for rep in range(2):
        for it in ens.items:
            it["state"].x.fill_(7.0)
        ens.run(graph=True)
        torch.cuda.synchronize()
        for (xe, _), (xg, _) in zip(eager, snapshot(ens)):
            assert np.array_equal(xg, xe), rep


def test_learned_ensemble_matches_single_corrected_runs(cola):
    """A class run with the learned correction (cola_step_lc per class): every member equals the
    same seed advanced alone by cola_step_lc, including its output between nodes (which drifts with
    the cached corrected force), eagerly and in graph replays; a plain class beside it is unchanged."""
    say("learned ensemble vs single corrected runs")
    from oracle import learned as olc
    cosmo = cola.make_cosmology(**W.COSMOLOGY)
    onet = olc.Net(channels=16, seed=5, in_scale=(0.25, 1.0, 1.0, 1.0), out_scale=0.5)
    onet.w3 *= 10.0
    flat = np.asarray(olc.flat_params(onet), dtype=np.float32)
    net = cola.LcNet(16, params=flat, in_scale=onet.in_scale, out_scale=onet.out_scale, training=False)
    box, n_part, n_steps, seeds, a_out = 64.0, 16, 6, (51, 52, 53), (0.5, 1.0)
    prob = cola.make_problem(box, n_part, 1, 19.0, n_steps, n_real=len(seeds))
    plain = cola.make_problem(120.0, 16, 3, 19.0, n_steps, n_real=2)
    spec = [dict(prob=prob, seeds=seeds, a_out=a_out, n_pk=48, n_bins=24, net=net),
            dict(prob=plain, seeds=(61, 62), a_out=(1.0,), n_pk=48, n_bins=24)]
    ens = cola.Ensemble(spec, cosmo)
    ens.run(graph=False)
    torch.cuda.synchronize()
    eager = snapshot(ens)
    n = n_part ** 3
    p1 = cola.make_problem(box, n_part, 1, 19.0, n_steps)
    tab = cola.schedule_table(p1, cosmo)
    lws = cola.lc_workspace(n_part, 16, 1)
    for r, seed in enumerate(seeds):
        st = cola.ParticleState(p1)
        ws = cola.Workspace(p1, n_pk=48)
        cola.ic_2lpt(p1, cosmo, [seed], st, ws)
        for k, a in enumerate(a_out):
            j = int((tab[:, 0] <= a * (1 + 1e-12)).sum()) - 1
            cola.step_lc(p1, cosmo, st, j, net, lws, ws)
            pk = cola.power_spectrum(p1, cosmo, st, a, 48, 24, ws)[1].cpu().numpy()[0]
            got = ens.items[0]["out"][1][k, r].cpu().numpy()
            sel = pk > 0
            assert np.abs(got[sel] / pk[sel] - 1).max() < 1e-4, (seed, a)
        cola.step_lc(p1, cosmo, st, n_steps - 1, net, lws, ws)
        assert rel_rms(ens.items[0]["state"].x[:, r * n:(r + 1) * n].cpu().numpy(), st.x.cpu().numpy()) < 1e-6
    # the plain class beside it is the plain run
    for r, seed in enumerate((61, 62)):
        pp = cola.make_problem(120.0, 16, 3, 19.0, n_steps)
        st = cola.ParticleState(pp)
        ws = cola.Workspace(pp, n_pk=48)
        cola.ic_2lpt(pp, cosmo, [seed], st, ws)
        cola.step(pp, cosmo, st, n_steps - 1, ws)
        assert rel_rms(ens.items[1]["state"].x[:, r * n:(r + 1) * n].cpu().numpy(), st.x.cpu().numpy()) < 1e-5
    for rep in range(2):
        for it in ens.items:
            it["state"].x.fill_(3.0)
            it["out"][1].fill_(-1.0)
        ens.run(graph=True)
        torch.cuda.synchronize()
        for (xe, pe), (xg, pg) in zip(eager, snapshot(ens)):
            assert np.array_equal(xg, xe), rep
            sel = pe > 0
            assert np.abs(pg[sel] / pe[sel] - 1).max() < 1e-4, rep
