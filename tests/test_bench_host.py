"""Host-side parts of bench.py that need no GPU: the one-GPU refusal and the traffic
lookup against the committed counter summary."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert not r.stdout.strip().startswith("{")


def test_traffic_lookup_follows_the_source_hash(tmp_path, monkeypatch):
    import bench
    with open(os.path.join(ROOT, "profiles", "traffic_256cubed.json")) as f:
        rec = json.load(f)
    if rec["source_hash"] != bench.kernel_source_hash():
        # taken on other kernel sources: the bench must not use it
        assert bench.measured_traffic("fp64", "k_fused") is None
        return
    for prec, word in (("fp64", 8), ("fp32", 4)):
        state = 6 * 256 ** 3 * word
        # every pass, the combined x kernel included, reads and writes the state once
        for k in ("k_c2c", "k_fused", "k_x_fwd", "k_x_inv", "k_x_invfwd"):
            t = bench.measured_traffic(prec, k)
            assert t is not None and abs(t / (2 * state) - 1) < 0.05, (prec, k, t)
    # a summary stamped with other sources is ignored
    stale = dict(rec, source_hash="0" * 16)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic_256cubed.json").write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("fp64", "k_fused") is None


def test_oracle_timing_script_runs_on_a_small_grid():
    # the all-core oracle timing (tests/oracle_timing.py) on a 16^3 sample, 2 processes
    from tests import oracle_timing
    out = oracle_timing.run(2, 16)
    assert out["single"]["value"] > 0 and out["parallel"]["processes"] == 2
    assert out["parallel"]["value"] > 0 and out["parallel"]["wall_s"] > 0


def test_cpu_baseline_reports_one_thread_and_all_processes():
    # the bench's CPU leg on a 16^3 input: one-thread rate beside the concurrent-process rate
    import bench
    from paper_2210_06232_amd import inputs
    H, E = inputs.random_fields((16, 16, 16), tuple(bench.WORKLOAD["domain"]), workload=2, p=2.0)
    out = bench.cpu_baseline(H, E)
    assert out["kind"] == "oracle" and out["cores"] >= 1 and out["value"] > 0
    assert out["single_thread"]["cores"] == 1 and out["single_thread"]["value"] > 0
    assert "16^3" in out["sample"] and out["seconds"] > 0


def test_sq_summary_reads_counter_csvs(tmp_path):
    # two counter passes of one dispatch each, as rocprofv3 writes them
    from paper_2210_06232_amd import profiling
    hdr = ('"Correlation_Id","Dispatch_Id","Agent_Id","Queue_Id","Process_Id","Thread_Id","Grid_Size","Kernel_Id",'
           '"Kernel_Name","Workgroup_Size","LDS_Block_Size","Scratch_Size","VGPR_Count","Accum_VGPR_Count",'
           '"SGPR_Count","Counter_Name","Counter_Value","Start_Timestamp","End_Timestamp"\n')
    name = '"void eifp::k_fused<double, eifp::Plan<256, 8>, 4, 0, 1>(int)"'
    passes = {"p1": {"SQ_WAVES": 100, "SQ_WAVE_CYCLES": 1000, "SQ_ACTIVE_INST_VALU": 250, "SQ_ACTIVE_INST_LDS": 50,
                     "SQ_WAIT_INST_ANY": 400},
              "p2": {"SQ_WAVES": 100, "SQ_INSTS_VALU": 557200, "SQ_INSTS_LDS": 84100, "SQ_INSTS_VMEM_RD": 4800,
                     "SQ_INSTS_VMEM_WR": 4800, "SQ_LDS_BANK_CONFLICT": 5}}
    dirs = []
    for d, cs in passes.items():
        (tmp_path / d).mkdir()
        rows = [f'1,1,"Agent 1",1,1,1,256,7,{name},128,78208,0,256,222,40,"{c}",{v},0,1\n' for c, v in cs.items()]
        (tmp_path / d / "run_counter_collection.csv").write_text(hdr + "".join(rows))
        dirs.append(str(tmp_path / d))
    out = tmp_path / "sq.md"
    profiling.sq_summary(dirs, str(out), "test")
    rec = json.loads((tmp_path / "sq.json").read_text())["kernels"]
    k = rec["k_fused<double, Plan<256, 8>, 4, 0, 1>"]
    assert k["waves_per_simd"] == 1 and k["vgpr"] == 256 and k["agpr"] == 222
    assert k["valu_per_wave"] == 5572 and k["lds_per_wave"] == 841 and k["vmem_per_wave"] == 96
    assert k["valu_share"] == 0.25 and k["dep_wait_share"] == 0.4 and k["bank_conflict_per_lds_active"] == 0.1
    assert "k_fused" in out.read_text()


def test_issue_roofline_follows_the_sq_summary(tmp_path, monkeypatch):
    import bench
    with open(os.path.join(ROOT, "profiles", "step_256cubed_sq_counters.json")) as f:
        rec = json.load(f)
    if rec["source_hash"] == bench.kernel_source_hash():
        # one launch of the 256^3 fused pass issues tens of millions of wave instructions
        for prec in ("fp64", "fp32"):
            v = bench.measured_valu(prec, "k_fused")
            assert v is not None and 1e7 < v < 1e9, (prec, v)
        r = bench.summarize("fp32", 20, 0.015, {"x_fwd": 0.2, "z_fwd": 2.6, "y_fused": 5.0, "z_inv": 2.5,
                                                  "x_inv": 3.5, "finalize": 0.1}, {"energy": 1.0})
        assert r["issue"]["bound"] == "alu" and r["issue"]["kernel"] == "k_fused"
        assert abs(r["issue"]["achieved"] - bench.measured_valu("fp32", "k_fused") / 0.25e-3 / 1e9) < 0.1
        assert r["issue"]["peak"] == 614.4
    stale = dict(rec, source_hash="0" * 16)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "step_256cubed_sq_counters.json").write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_valu("fp64", "k_fused") is None


def test_kernel_hash_ignores_comments_and_whitespace():
    from paper_2210_06232_amd.profiling import code_text
    a = 'int f(int x) {  // twice\n  return 2 * x; /* doubled */ }\nasm volatile("" : "+v"(x));'
    b = 'int f(int x) {\n    return 2 * x;   }\n// a note\nasm volatile("" : "+v"(x));'
    assert code_text(a) == code_text(b)
    assert code_text(a) != code_text(a.replace("2 * x", "3 * x"))
    assert code_text('s = "//not a comment";') == 's = "//not a comment";'


def test_kernel_hash_covers_per_source_compiler_flags(monkeypatch):
    # a source's extra compiler flags change its code, so they change the hash that
    # decides whether committed counter summaries still describe the built kernels
    from paper_2210_06232_amd import build, profiling
    h0 = profiling.kernel_source_hash()
    flags = dict(build.FILE_FLAGS)
    flags["passes_c2c_f64.hip"] = []
    monkeypatch.setattr(build, "FILE_FLAGS", flags)
    assert profiling.kernel_source_hash() != h0
