"""Host-side pieces of bench.py: the committed HBM-traffic summaries are found
under the dominant kernel's template name and are used only while the sources
of that kernel's device code are the ones they were measured on."""
import glob
import os

import bench


def _kv(path):
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    return kv


def test_traffic_summaries_are_found_by_kernel_template_name():
    files = glob.glob(os.path.join(bench.ROOT, "profiles", "*_traffic.txt"))
    assert files
    for path in files:
        kv = _kv(path)
        stem = os.path.basename(path)[: -len("_traffic.txt")]
        kernel = kv["kernel"].split("<")[0]
        assert stem.startswith(kernel + "_"), (path, kernel)
        workload = stem[len(kernel) + 1:]
        # as the library names the dominant kernel in the bench line
        inst = bench.kernel_instance(kv["kernel"]) + "> tz 7"
        got = bench.measured_traffic(inst, workload)
        assert bench.measured_traffic(kernel + "<1,1> tz 7", workload) is None   # another instantiation
        if kv["source_sha256"] == bench.source_digest(kv["kernel"]):
            assert got == int(float(kv["hbm_bytes_per_launch"]))
        else:
            assert got is None
        # the scaled counters (printed to 0.1 KiB and 6 digits) give the total
        hbm = (float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_scale"])
               + float(kv["write_kib_per_dispatch"]) * float(kv["write_scale"])) * 1024
        assert abs(hbm - float(kv["hbm_bytes_per_launch"])) <= 1e-4 * hbm


def test_kernel_instance_names():
    assert bench.kernel_instance("k_rows2<1024,1> tz 43") == "k_rows2<1024,1"
    assert bench.kernel_instance("k_rows2<1024,1,true>") == "k_rows2<1024,1"
    assert bench.kernel_instance("k_slab<1024,1> tz 2 steps/launch 1024") == bench.kernel_instance("k_slab<1024,1>")
    assert bench.kernel_instance("k_slab<768,2>") != bench.kernel_instance("k_slab<1024,1>")


def test_unknown_kernel_or_workload_has_no_traffic():
    assert bench.measured_traffic("k_nonexistent", "rod_b1_ens8") is None
    assert bench.measured_traffic("k_slab", "no_such_workload") is None


def test_source_digest_covers_only_the_kernels_own_sources():
    a = bench.source_digest("k_rows2<1024,1> tz 43")
    assert a == bench.source_digest("k_rows2")
    assert a != bench.source_digest("k_slab<1024,1>")
