"""The seeded workload generators and the fixed serving loads (CPU only)."""
import numpy as np

from paper_1201_3114_amd import workloads


def test_serving_loads_follow_from_the_trace():
    """The fixed offered loads use the mean request size of the 200,000-request trace itself."""
    tr = workloads.serve_trace(count=200_000, qps=1.0)
    assert abs(float(tr.sizes.mean()) - workloads.SERVE_MEAN_REQUEST_BYTES) < 0.05
    for load, qps in workloads.SERVE_QPS.items():
        assert abs(qps * workloads.SERVE_MEAN_REQUEST_BYTES - load * workloads.SERVE_CAPACITY_GBPS * 1e9) < 1e-4 * qps * 1e5
    assert sorted(workloads.SERVE_QPS) == [0.3, 0.5, 0.7, 0.9]


def test_serve_trace_rescales_with_qps_only():
    """Two rates give the same requests; only the arrival times scale."""
    a = workloads.serve_trace(count=1000, qps=100.0)
    b = workloads.serve_trace(count=1000, qps=400.0)
    assert np.array_equal(a.sizes, b.sizes) and np.array_equal(a.decrypt, b.decrypt) and a.passwords == b.passwords
    assert np.allclose(a.arrival_s, 4 * b.arrival_s)
    assert a.sizes.min() >= 64 and a.sizes.max() <= 16 << 20
