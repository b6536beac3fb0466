"""Forecast serving (continuous batching) on the GPU: requests that arrive
while others run join the running batch as memory frees up, and every
request's forecast is bitwise the one it gets alone."""
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
             scenarios.c2(scale=10)]
    reqs = []
    for rid, (k, steps, arrival) in enumerate([(0, 131, 0.0), (2, 97, 0.0), (1, 260, 0.0), (2, 45, 0.0),
                                              (0, 77, 0.3), (1, 20, 0.35)]):
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
