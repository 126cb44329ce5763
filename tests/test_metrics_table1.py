"""The throughput definition reproduces the paper's printed rates (Table I)."""

import json
import os

from paper_1503_06189_amd import metrics

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_rates.json")


def test_table1_sky_rates():
    g = json.load(open(GOLD))
    assert metrics.SAMPLE_RATE_HZ == g["sample_rate_hz"]
    for ch, key in (("channels_per_link", "sky_gbps_per_link"),
                    ("channels_per_host", "sky_gbps_per_host"),
                    ("channels_system", "sky_gbps_system")):
        bits = metrics.input_bits(g["inputs"], g[ch], int(g["sample_rate_hz"]))
        assert abs(bits / 1e9 - g[key]) < 1e-9, key


def test_table1_output_size():
    g = json.load(open(GOLD))
    mb = metrics.output_bytes(g["inputs"], g["channels_per_host"]) / 1e6
    assert abs(mb - g["output_bytes_per_host_integration_approx_mb"]) < 0.05
