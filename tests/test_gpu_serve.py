"""Forecast serving (continuous batching) on the GPU: requests that arrive
while others run join the running batch as memory frees up, every
request's forecast is bitwise the one it gets alone, a served forecast is
bitwise the oracle's, and the cost model replays the stream."""
import numpy as np
import pytest

import scenarios

pytestmark = pytest.mark.gpu


def alone(site, source, steps, precision):
    from paper_2408_07609_amd import Domain
    d = Domain(site.levels, site.dx0, site.dt, g=site.g, manning_n=site.manning_n, dry_eps=site.dry_eps, bc=site.bc,
               x0=site.x0, y0=site.y0, precision=precision)
    d.set_source(*source)
    d.step(steps)
    out = [d.max_inundation(k) for k in range(len(d.levels))], [d.get_state(k) for k in range(len(d.levels))]
    d.close()
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_served_forecasts_match_alone(precision):
    from paper_2408_07609_amd.serve import ForecastServer, Request, footprint
    sites = [scenarios.small_nested(seed=7, nlev=3), scenarios.small_nested(seed=11, nlev=2, base=(90, 72),
                                                                            child=(45, 54)),
             scenarios.c2(scale=10), scenarios.small_union()]
    reqs = []
    for rid, (k, steps, arrival) in enumerate([(0, 131, 0.0), (2, 97, 0.0), (1, 260, 0.0), (2, 45, 0.0),
                                              (0, 77, 0.3), (1, 20, 0.35), (3, 150, 0.1)]):
        s = sites[k].source
        src = (s.xc, s.yc, s.a, s.b, s.theta, 0.5 + 0.7 * rid, s.shape)
        reqs.append(Request(rid, sites[k], src, steps, arrival))
    # room for the two largest requests at once, so later ones queue for memory
    budget = 2 * max(footprint(s, precision) for s in sites) + 1
    srv = ForecastServer(budget, precision, chunk_steps=16, keep_state=True)
    results = srv.run(reqs)
    srv.close()
    assert sorted(r.rid for r in results) == list(range(len(reqs)))
    assert srv.peak_members >= 2 and srv.peak_bytes <= budget
    assert srv.cell_updates == sum(r.site.cells * r.steps for r in reqs)
    by_id = {r.rid: r for r in results}
    for req in reqs:
        zmax, state = alone(req.site, req.source, req.steps, precision)
        res = by_id[req.rid]
        assert res.time_to_forecast >= 0.0 and res.admitted >= req.arrival - 1e-6
        for k in range(len(zmax)):
            assert np.array_equal(res.maxima[k], zmax[k]), f"request {req.rid} level {k}: maxima differ"
            for x, y in zip(res.state[k], state[k]):
                assert np.array_equal(x, y), f"request {req.rid} level {k}: state differs"


def test_served_forecast_matches_oracle():
    """A request served in a mix (others arriving, leaving and queueing for
    memory) against the CPU oracle: started from the oracle's initial level,
    its forecast (maxima) and final state are bitwise the oracle's."""
    import oracle
    from paper_2408_07609_amd.serve import ForecastServer, Request, footprint
    sites = [scenarios.c2(scale=10), scenarios.small_nested(seed=7, nlev=3),
             scenarios.small_nested(seed=11, nlev=2, base=(90, 72), child=(45, 54))]
    target = sites[0]
    o = oracle.OracleDomain(**target.oracle_kwargs())
    o.set_source(*target.source.astuple())
    initial = [o.get_state(k)[0] for k in range(len(target.levels))]
    steps = 700
    reqs = [Request(0, sites[1], sites[1].source.astuple(), 150, 0.0),
            Request(1, target, target.source.astuple(), steps, 0.0, initial=initial),
            Request(2, sites[2], sites[2].source.astuple(), 333, 0.0),
            Request(3, sites[1], sites[1].source.astuple(), 90, 0.2)]
    budget = footprint(target, 0) + footprint(sites[2], 0) + 1
    srv = ForecastServer(budget, 0, chunk_steps=50, keep_state=True)
    res = {r.rid: r for r in srv.run(reqs)}
    srv.close()
    assert srv.peak_members >= 2
    o.step(steps)
    for k in range(len(target.levels)):
        zo = o.max_inundation(k)
        eo, Mo, No = o.get_state(k)
        assert np.abs(res[1].maxima[k] - zo).max() <= 1e-9 and np.abs(res[1].state[k][0] - eo).max() <= 1e-9
        assert np.array_equal(res[1].maxima[k], zo), f"level {k}: served maxima not bitwise the oracle's"
        for x, y in zip(res[1].state[k], (eo, Mo, No)):
            assert np.array_equal(x, y), f"level {k}: served state not bitwise the oracle's"


def test_cost_model_fits_and_replays_the_stream():
    """The cost model (step time = a * computed cells + b) fitted on a
    serving run's chunks has a positive per-cell cost, and replaying the
    stream through the server's policy gives a time to forecast for every
    request."""
    from paper_2408_07609_amd.serve import ForecastServer, Request, fit_cost_model, footprint, predict
    sites = [scenarios.c2(scale=4), scenarios.c2(scale=10)]          # 626 k and 100 k cells
    reqs = [Request(i, sites[i % 2], sites[i % 2].source.astuple(), 300 + 150 * i, 0.05 * i) for i in range(6)]
    budget = 2 * footprint(sites[0], 0) + 1
    srv = ForecastServer(budget, 0, chunk_steps=60)
    res = srv.run(reqs)
    srv.close()
    a, b = fit_cost_model(srv.chunks)
    frac = sum(c[3] for c in srv.chunks) / sum(c[0] * c[2] for c in srv.chunks)
    pred = predict(reqs, a, b, frac, budget, 0, 60)
    assert a > 0 and b >= 0 and 0 < frac <= 1 and sorted(pred) == list(range(6))
    assert all(v > 0 for v in pred.values())
    print({r.rid: (round(r.time_to_forecast, 4), round(pred[r.rid], 4)) for r in res}, a, b)
