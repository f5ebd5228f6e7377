"""Format of the launch-configuration table shipped with the library (no GPU needed)."""
import os


def test_shipped_tuning_table_format():
    """Every entry of the shipped launch table is a well-formed line for one of the study lattices
    with a configuration inside the header's ranges, and no (lattice, format, n, form) repeats."""
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_1409_1510_amd", "tuning", "gfx950.txt")
    lattices = {(32, 32, 32, 8), (48, 48, 48, 12), (64, 64, 64, 16)}
    seen = set()
    count = 0
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        assert len(f) == 14, line
        lx, ly, lz, lt, prec, recon, n, fused, rt, spb, nt, lds, xm = map(int, f[:13])
        ms = float(f[13])
        assert (lx, ly, lz, lt) in lattices
        assert prec in (0, 1, 2) and recon in (14, 18) and (prec != 0 or recon == 18)
        assert 1 <= n <= 64 and fused in (0, 1)
        assert rt in (1, 2, 4, 8, 16) and spb in (32, 64, 256) and nt in (0, 1)
        assert spb != 32 or (lds in (1, 2) and rt <= 2 and fused == 0)
        assert 0 <= lds <= 6 and 0 <= xm <= 3 and (xm == 0 or lds > 0)
        assert not (prec == 0 and (rt == 16 or lds >= 4))
        assert ms > 0
        key = (lx, ly, lz, lt, prec, recon, n, fused)
        assert key not in seen
        seen.add(key)
        count += 1
    assert count >= 50


def test_committed_kernel_profile_matches_sources_and_table():
    """The committed rocprofv3 summary of the benchmarked kernel was taken on the current kernel
    sources (bench.py reports its HBM traffic only then) and in the launch configuration the
    shipped table gives the benchmark's case (32^3 x 8, FP32, 18-real Naik, 16 rhs, plain form);
    its counter traffic is at least the compulsory bytes of that launch."""
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench
    fields = {}
    for line in open(bench.PROFILE_SUMMARY):
        if ":" in line and not line.startswith(" "):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    assert fields["kernel_source_sha256_16"] == bench.kernel_source_hash()
    cfg = None
    for line in open(os.path.join(root, "paper_1409_1510_amd", "tuning", "gfx950.txt")):
        f = line.split()
        if f and not f[0].startswith("#") and list(map(int, f[:8])) == [32, 32, 32, 8, 1, 18, 16, 0]:
            cfg = tuple(map(int, f[8:13]))
    assert cfg is not None and fields["launch_config"] == str(cfg)
    traffic = bench.measured_traffic(cfg)
    compulsory = 32 * 32 * 32 * 8 // 2 * (1152 + 48 * 16)
    assert traffic is not None and traffic >= compulsory
    assert int(fields["algorithmic_bytes_per_launch"]) == compulsory
