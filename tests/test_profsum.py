"""Host logic of the profile summariser: kernel names as rocprofv3 prints
them map to the library's kernels, and the kernels of one library sort are
summed (CPU only)."""
import csv

from paper_1309_1114_amd import profsum


def test_kernel_names():
    s = profsum.short
    assert s("void splotch_dev::k_count<false>(splotch_dev::JobDev const*, unsigned long long*)") == "k_count"
    assert s("void splotch_dev::k_splat<float, 8>(splotch_dev::JobDev const*, int4 const*, unsigned int*, int)") == "k_splat"
    assert s("splotch_dev::k_scatter(splotch_dev::JobDev const*, unsigned long long*)") == "k_scatter"
    assert s("splotch_dev::k_ord_composite(splotch_dev::OrdJob, unsigned int const*, unsigned int)") == "k_ord_composite"
    # k_items must not swallow k_ord_items, nor k_count k_lgcount
    assert s("splotch_dev::k_ord_items(splotch_dev::OrdJob, unsigned int const*, unsigned int, unsigned int)") == "k_ord_items"
    assert s("splotch_dev::k_lgcount(splotch_dev::JobDev const*)") == "k_lgcount"
    assert s("splotch_dev::k_segsum(splotch_dev::JobDev const*)") == "k_segsum"
    assert s("void splotch_dev::k_splat<float, 8, false>(splotch_dev::JobDev const*, int4 const*, unsigned int*, int, unsigned long long*)") == "k_splat"
    assert s("splotch_sort::(anonymous namespace)::k_rs_scatter(unsigned int const*, unsigned int*, unsigned int const*, unsigned int*, unsigned long, unsigned long const*, int, unsigned long const*)") == "radix_sort"
    assert s("splotch_sort::(anonymous namespace)::k_rs_hist(unsigned int const*, unsigned long, unsigned long const*, int, unsigned long*)") == "radix_sort"
    assert s("splotch_sort::(anonymous namespace)::k_key_range(unsigned long const*, unsigned long, unsigned long*)") == "radix_sort"
    assert s("void splotch_sort::(anonymous namespace)::k_rs_scatter<true>(unsigned int const*, unsigned int*)") == "radix_sort"
    assert s("splotch_sort::(anonymous namespace)::k_fix_mark(unsigned int const*, unsigned int const*, unsigned long, unsigned long*, unsigned int*)") == "radix_sort"
    assert s("splotch_dev::k_ord_pass_bounds(unsigned long const*, long, unsigned long, unsigned long, unsigned long*)") == "k_ord_pass_bounds"
    assert s("splotch_sort::(anonymous namespace)::k_scan_down(unsigned long const*, unsigned long*, unsigned long, unsigned long const*)") == "scan"
    assert s("void (anonymous namespace)::k_conv_fwd<1, 2>(unsigned short const*, unsigned short const*)") == "k_conv_fwd"
    assert s("(anonymous namespace)::k_region_check(float const*, float const*, int)") == "k_region_check"
    assert s("void at::native::elementwise_kernel<128, 4, AUnaryFunctor<float> >()") == "copy_ref"
    assert s("some_other_kernel()") is None


def test_kernel_stats_sums_kernels_of_one_name(tmp_path):
    f = tmp_path / "x_kernel_stats.csv"
    rows = [("splotch_sort::(anonymous namespace)::k_rs_hist(unsigned int const*, int)", 4, 4e6, 10.0),
            ("splotch_sort::(anonymous namespace)::k_rs_scatter(unsigned int const*, int)", 28, 24e6, 30.0),
            ("splotch_dev::k_ord_merge(splotch_dev::OrdJob, unsigned int)", 4, 0.8e6, 1.0)]
    with open(f, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        for name, calls, tot, pct in rows:
            w.writerow([name, calls, tot, tot / calls, pct])
    ks = profsum.kernel_stats(str(tmp_path))
    assert ks["radix_sort"]["calls"] == 32
    assert abs(ks["radix_sort"]["avg_ms"] - 28e6 / 32 / 1e6) < 1e-12
    assert abs(ks["radix_sort"]["pct"] - 40.0) < 1e-12
    assert ks["k_ord_merge"]["calls"] == 4


def test_source_hash_ignores_comments_only(tmp_path):
    from paper_1309_1114_amd.profsum import code_only, source_hash
    src = 'int a = 1;  // count\n/* block\n comment */ const char* s = "x // y";\n'
    assert code_only(src) == 'int a = 1; const char* s = "x // y";'
    d = tmp_path / "paper_1309_1114_amd" / "csrc"
    d.mkdir(parents=True)
    for f in ("device.h", "kernels.h", "render.hip"):
        (d / f).write_text(src)
    h0 = source_hash(str(tmp_path))
    (d / "kernels.h").write_text(src.replace("// count", "// a longer comment\n\n"))
    assert source_hash(str(tmp_path)) == h0
    (d / "kernels.h").write_text(src.replace("a = 1", "a = 2"))
    assert source_hash(str(tmp_path)) != h0
