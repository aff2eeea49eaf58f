"""Graph replay of lbm_step: bit-identical to launching the steps one by one,
checked after every call, with eager work and synchronisation between the
replays, across step counts that are and are not multiples of the graph,
an omega change, in-place streaming, held planes, and checkpointed runs and
restores in between."""
import numpy as np
import pytest
import torch

from paper_1303_4624_amd import Simulation
from synth_inputs import smooth_ic, tube_ic

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _pair(model, extent, precision, streaming, stream):
    plain = Simulation(model, extent, 1.4, precision=precision, streaming=streaming, stream=stream)
    graph = Simulation(model, extent, 1.4, precision=precision, streaming=streaming, stream=stream)
    graph.set_graph_steps(4)
    return plain, graph


def _check(a, b):
    torch.cuda.synchronize()
    for x, y in zip(a.moments(), b.moments()):
        torch.cuda.synchronize()
        assert torch.equal(x, y)
    assert torch.equal(a.get_populations(), b.get_populations())


@pytest.mark.parametrize("model,extent", [("D3Q95", (12, 6, 5)), ("D2Q33", (40, 9)),
                                          ("D3Q19", (16, 6, 5))])
@pytest.mark.parametrize("precision", ["fp64", "fp32s"])
@pytest.mark.parametrize("streaming", ["ab", "aa"])
def test_graph_replay_equals_single_launches(model, extent, precision, streaming):
    _say("case", model, extent, precision, streaming)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        rho, U, th = smooth_ic(extent, seeds=tuple(range(41, 41 + len(extent) + 2)), amp_u=0.03)
        plain, graph = _pair(model, extent, precision, streaming, stream)
        try:
            for s in (plain, graph):
                s.init_fields(rho, U, th * s.T0)
            for n in (4, 8, 3, 1, 9, 12):      # full graphs, remainders, parity changes
                plain.step(n)
                graph.step(n)
                _check(plain, graph)
            for s in (plain, graph):            # the graph is rebuilt with the new omega
                s.set_omega(1.7)
            plain.step(8)
            graph.step(8)
            _check(plain, graph)
        finally:
            plain.close()
            graph.close()


@pytest.mark.parametrize("streaming", ["ab", "aa"])
def test_graph_replay_with_held_planes(streaming):
    extent = (6, 4, 40)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        rho, U, th = tube_ic(extent, 20, (2.0, 1.0), (1.0, 1.1))
        plain, graph = _pair("D3Q95", extent, "fp64", streaming, stream)
        try:
            for s in (plain, graph):
                s.init_fields(rho, U, th * s.T0)
                st_lo = (2.0, 0.0, 0.0, 0.0, s.T0)
                st_hi = (1.0, 0.0, 0.0, 0.0, 1.1 * s.T0)
                s.set_fixed_planes(5, 5, st_lo, st_hi)
            for n in (8, 5, 16):
                plain.step(n)
                graph.step(n)
                _check(plain, graph)
        finally:
            plain.close()
            graph.close()


@pytest.mark.parametrize("streaming", ["ab", "aa"])
def test_graph_replay_around_checkpointed_runs_and_restores(streaming):
    # Checkpointed runs and restores change the buffer parity or storage
    # form under a captured graph; the replays that follow must still equal
    # single launches.
    extent = (20, 6, 8)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        rho, U, th = smooth_ic(extent, seeds=(71, 72, 73, 74, 75), amp_u=0.03)
        plain, graph = _pair("D3Q95", extent, "fp32s", streaming, stream)
        try:
            cks = []
            for s in (plain, graph):
                s.init_fields(rho, U, th * s.T0)
                s.step(8)
                cks.append(s.run_checkpointed(7, 3))
                s.step(9)
            _check(plain, graph)
            for s, ck in zip((plain, graph), cks):
                s.restore_checkpoint(7, 3, ck, 1)
                s.step(12)
            _check(plain, graph)
        finally:
            plain.close()
            graph.close()


@pytest.mark.parametrize("streaming", ["ab", "aa"])
def test_side_stream_without_making_it_current(streaming):
    # A Simulation on its own stream, driven from code whose current stream
    # is the default one: inputs made on the current stream are waited for,
    # outputs are ready on it, and the results equal a default-stream run.
    from paper_1303_4624_amd import Simulation
    extent = (40, 12, 10)
    rho, U, th = smooth_ic(extent, seeds=(7, 8, 9, 10, 11), amp_u=0.03)
    ref = Simulation("D3Q95", extent, 1.4, precision="fp32s", streaming=streaming)
    ref.init_fields(rho, U, th * ref.T0)
    ref.step(9)
    want = [x.cpu() for x in ref.moments()]
    ref.close()
    side = torch.cuda.Stream()
    sim = Simulation("D3Q95", extent, 1.4, precision="fp32s", stream=side, streaming=streaming)
    for _ in range(3):
        sim.init_fields(rho, U, th * sim.T0)
        sim.step(9)
        got = [x.cpu() for x in sim.moments()]
        assert all(torch.equal(a, b) for a, b in zip(got, want))
        # checkpoints and a restore on the side stream, read back on the default one
        ck = sim.run_checkpointed(6, 3)
        sim.restore_checkpoint(6, 3, ck, 1)
        sim.step(3)
        r1 = sim.moments()[0].cpu()
        sim.restore_checkpoint(6, 3, ck, 2)
        assert torch.equal(r1, sim.moments()[0].cpu())
    sim.close()
