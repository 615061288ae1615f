"""The committed rocprofv3 summaries stay tied to the kernel they describe: the
HBM-traffic block that bench.py reports as `roofline.traffic` must have been
taken on the current sources of the order-2 rollout kernel, in the benchmark
driver's window (5 warm-up and 20 timed steps of the 4096-chain workload, mixed
precision).  After a change to those sources the profile has to be taken again
(the commands are in profiles/k_rollout_chains4096_hbm_traffic.md)."""
import bench
from paper_1709_04145_amd import workloads as W


def test_traffic_profile_matches_the_kernel_sources():
    traffic = bench.measured_traffic(W.CONFIG_NAMES[2], "mixed", 5, 20)
    assert traffic is not None, ("no HBM-traffic block for source digest " + bench.kernel_source_digest() +
                                 " in " + bench.TRAFFIC_PROFILE_GLOB)
    assert traffic > 0
