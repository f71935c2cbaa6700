"""Host-side logic of bench.py: labelling of profiled dispatches by iteration group and
reading of the committed HBM-traffic summary (no GPU)."""
import os

import bench


def schedule_names(n_replays=2, scatter_f1=False):
    names = ["fill", "fill"]
    for _ in range(n_replays):
        names.append("k_prepare")
        for t in range(60):
            f = (4, 2, 1)[t // 20]
            bp = "k_bps<32, 16, true>" if scatter_f1 and f == 1 else \
                f"k_bp<{16 if f > 1 else 8}, {1 if f == 4 else 2}, true>"
            names += ["k_fp<true, 4>", bp, "k_tv<32, 6, 1024>"]
        names += ["fill", "fill"]
    names.append("__amd_rocclr_copyBuffer")
    return names


def test_label_dispatches_groups_every_replay():
    names = schedule_names(2)
    lab = bench.label_dispatches(names)
    groups = {}
    for g, j in lab:
        groups.setdefault(g, []).append(j)
    assert groups["prepare_f4"] == [2, 2 + 181 + 2]
    for c in ("fp", "bp", "tv"):
        for f in (4, 2, 1):
            js = groups[f"{c}_f{f}"]
            assert len(js) == 40
            assert all(names[j].startswith("k_" + c) for j in js)
    # a truncated replay is not counted
    lab2 = bench.label_dispatches(names[: 2 + 181 + 2 + 100])
    assert len(lab2) == 181
    # a tuning run (pooling, then repeated projections) is not a replay
    tuning = ["k_prepare"] + ["k_fp<true, 4>"] * 10 + ["k_bp<8, 2, true>"] * 10 + ["k_tv<32, 6, 1024>"] * 10
    assert bench.label_dispatches(tuning + names) == [(g, j + len(tuning)) for g, j in lab]


def test_label_dispatches_accepts_the_scatter_back_projector():
    names = schedule_names(2, scatter_f1=True)
    lab = bench.label_dispatches(names)
    groups = {}
    for g, j in lab:
        groups.setdefault(g, []).append(j)
    assert len(lab) == 2 * 181
    assert all(names[j].startswith("k_bps<32, 16") for j in groups["bp_f1"])
    assert all(names[j].startswith("k_bp<") for j in groups["bp_f2"])


def test_label_dispatches_accepts_the_lds_tap_projector():
    names = schedule_names(1)
    names = [("k_fp_lds<true, 8>" if n.startswith("k_fp") and i < 2 + 1 + 60 else n) for i, n in enumerate(names)]
    lab = bench.label_dispatches(names)
    assert len(lab) == 181
    assert all(names[j].startswith("k_fp_lds") for g, j in lab if g == "fp_f4")
    # an untimed projection (no residual) is not part of an iteration
    bad = [("k_fp<false, 8>" if n.startswith("k_fp") else n) for n in names]
    assert bench.label_dispatches(bad) == []


def test_launch_kernel_names_follow_the_launch_configuration():
    c = dict(fp_seg=8, bp_px=2, bp_vg=16, tv_tile=32, fp_lds=1)
    assert bench.launch_kernel("fp", c) == "k_fp<true, 8>"
    assert bench.launch_kernel("bp", c) == "k_bp<16, 2, true, false>"
    assert bench.launch_kernel("tv", c) == "k_tv<32, 6, 1024>"
    assert bench.launch_kernel("tv", c, tv_iters=7) == "k_tv<32, 9, 1024>"
    s = dict(c, bp_px=32, fp_lds=2, tv_tile=16)
    assert bench.launch_kernel("bp", s) == "k_bps<32, 16, true>"
    assert bench.launch_kernel("fp", s) == "k_fp_lds<true, 8>"
    assert bench.launch_kernel("tv", s) == "k_tv<16, 6, 256>"
    assert bench.bp_form(c) == "gather" and bench.bp_form(s) == "scatter"


def test_launch_traffic_reads_matching_summary(tmp_path):
    p = tmp_path / "t.md"
    row = "| bp_f1 | `k_bp<8, 2, true>` | 40 | 5210.4 | 1024.0 | 10666042 | 1048576 | 11714618 |"
    p.write_text(f"kernel sources sha256: `{bench.kernel_source_hash()}`\n\n{row}\n")
    assert bench.launch_traffic("bp_f1", str(p))[0] == 11714618
    assert bench.launch_traffic("bp_f1", str(p), kernel="k_bp<8, 2, true>")[0] == 11714618
    # a row measured on another launch form of the group is not used
    t, why = bench.launch_traffic("bp_f1", str(p), kernel="k_bps<32, 16, true>")
    assert t is None and "k_bps<32, 16, true>" in why
    assert bench.launch_traffic("fp_f1", str(p))[0] is None
    p.write_text(f"kernel sources sha256: `{'0' * 64}`\n\n{row}\n")
    assert bench.launch_traffic("bp_f1", str(p))[0] is None
    assert bench.launch_traffic("bp_f1", os.path.join(str(tmp_path), "missing.md"))[0] is None


def test_oracle_thread_setting_round_trips():
    """The oracle's thread count (timing support) can be set and restored."""
    import oracle

    before = oracle.set_threads(0)
    assert before >= 1
    assert oracle.set_threads(1) == before
    assert oracle.set_threads(before) == 1
    assert oracle.set_threads(0) == before

