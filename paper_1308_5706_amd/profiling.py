"""Summaries of rocprofv3 runs of ``bench.py`` (kernel trace and HBM counters).

Usage (after the rocprofv3 runs listed in the summary header have written their
databases under one directory)::

    python -m paper_1308_5706_amd.profiling DIR NAME "COMMANDS"

writes ``profiles/NAME_kernels.md`` (per-kernel device time from the trace) and
``profiles/NAME_hbm_traffic.txt`` (JSON: HBM bytes per dispatch from FETCH_SIZE and
WRITE_SIZE, each scaled by what the same counter reads for a plain device copy of known
size, grouped by the library's stage names, with a hash of the kernel sources so that a
reader can tell whether the kernels changed since the counters were taken).

Expected layout of DIR: ``trace/``, ``fetch/``, ``write/``, ``cfetch/``, ``cwrite/``, each
holding one ``*_results.db`` (rocpd SQLite) from, in order: ``--kernel-trace --stats`` on
the bench, ``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE`` on the bench, and the two
counters on ``bench.py --copy-calibration GIB``.
"""
from __future__ import annotations

import glob
import hashlib
import json
import os
import sqlite3
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# library stage name -> substring of the kernel symbol (demangled) that implements it
STAGE_KERNELS = {  # first match wins: the fused passes before the gamma passes they contain
    "alpha_gamma_fwd": ("alpha_gamma_fwd_kernel", "alpha_gamma_fwd_pfa_kernel"),
    "gamma_alpha_adj": ("gamma_alpha_adj_kernel", "gamma_alpha_adj_pfa_kernel"),
    "wigner_fwd": ("wig_fwd_kernel",),
    "wigner_adj": ("wig_adj_kernel",),
    "beta_fwd": ("beta_fwd_fft_kernel", "beta_fwd_pair_kernel", "beta_fwd_pfa_kernel"),
    "alpha_fwd": ("alpha_fwd_fft_kernel", "alpha_fwd_blk_kernel", "alpha_fwd_pfa_kernel"),
    "gamma_fwd": ("gamma_fwd_kernel",),
    "gamma_adj": ("gamma_adj_kernel",),
    "alpha_adj": ("alpha_adj_fft_kernel", "alpha_adj_blk_kernel", "alpha_adj_pfa_kernel"),
    "beta_adj": ("beta_adj_fft_kernel", "beta_adj_multi_kernel"),
    "syn_final": ("syn_final_kernel",),
    "pad": ("pad_flm_kernel",),
    "scaling": ("scaling_kernel",),
}


def kernel_sources_hash() -> str:
    """sha256 over the HIP/C++ sources of the library (sorted by name)."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        if p.endswith((".hip", ".h", ".cpp")):
            h.update(os.path.basename(p).encode())
            with open(p, "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def stage_of(kernel_name: str):
    for st, subs in STAGE_KERNELS.items():
        if any(sub in kernel_name for sub in subs):
            return st
    return None


def _db(d: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *_results.db under {d}")
    return hits[-1]


def _q(path: str, sql: str):
    con = sqlite3.connect(path)
    try:
        return list(con.execute(sql))
    finally:
        con.close()


def counter_per_dispatch(d: str, counter: str):
    """{kernel name: [counter value per dispatch]} (values in the counter's unit, KiB)."""
    rows = _q(_db(d), "select kernel_name, counter_name, value from counters_collection")
    out = defaultdict(list)
    for k, c, v in rows:
        if c == counter:
            out[k].append(float(v))
    return out


def calibration(d: str, counter: str, copy_bytes: int) -> float:
    """Bytes per counter unit, from a plain device copy of copy_bytes."""
    per = counter_per_dispatch(d, counter)
    vals = [v for k, vs in per.items() if "copyBuffer" in k for v in vs]
    if not vals:
        raise RuntimeError(f"no copy kernel dispatch with {counter} in {d}")
    return copy_bytes / (sum(vals) / len(vals))


def summarize(d: str, copy_bytes: int):
    trace = _q(_db(os.path.join(d, "trace")),
               "select name, count(*), sum(end - start), avg(end - start) from kernels group by name")
    cal = {c: calibration(os.path.join(d, sub), c, copy_bytes)
           for c, sub in (("FETCH_SIZE", "cfetch"), ("WRITE_SIZE", "cwrite"))}
    fetch = counter_per_dispatch(os.path.join(d, "fetch"), "FETCH_SIZE")
    write = counter_per_dispatch(os.path.join(d, "write"), "WRITE_SIZE")
    kernels = {}
    for name, n, tot, avg in trace:
        kernels[name] = {"dispatches": int(n), "total_ns": float(tot), "avg_ns": float(avg)}
    traffic = {}
    for name in set(fetch) | set(write):
        f, w = fetch.get(name, []), write.get(name, [])
        traffic[name] = {
            "dispatches": max(len(f), len(w)),
            "fetch_bytes_per_dispatch": (sum(f) / len(f)) * cal["FETCH_SIZE"] if f else None,
            "write_bytes_per_dispatch": (sum(w) / len(w)) * cal["WRITE_SIZE"] if w else None,
        }
    stages = defaultdict(lambda: {"fetch_bytes": 0.0, "write_bytes": 0.0, "dispatches": 0})
    for name, t in traffic.items():
        st = stage_of(name)
        if st is None or t["fetch_bytes_per_dispatch"] is None or t["write_bytes_per_dispatch"] is None:
            continue
        stages[st]["fetch_bytes"] += t["fetch_bytes_per_dispatch"] * t["dispatches"]
        stages[st]["write_bytes"] += t["write_bytes_per_dispatch"] * t["dispatches"]
        stages[st]["dispatches"] += t["dispatches"]
    for st, v in stages.items():
        v["bytes_per_dispatch"] = (v["fetch_bytes"] + v["write_bytes"]) / max(v["dispatches"], 1)
    return kernels, traffic, dict(stages), cal


def write_profiles(d: str, name: str, commands: str, copy_bytes: int, out_dir: str | None = None):
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    kernels, traffic, stages, cal = summarize(d, copy_bytes)
    src = kernel_sources_hash()
    lines = [f"# rocprofv3 kernel trace: {name}", "", "Commands (run from the repository root):", "",
             "```", commands.strip(), "```", "",
             f"Kernel sources sha256: `{src}`", "",
             "| kernel | dispatches | total ms | avg us | stage | HBM read MB/dispatch | HBM write MB/dispatch |",
             "|---|---:|---:|---:|---|---:|---:|"]
    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["total_ns"]):
        t = traffic.get(k, {})
        fr = t.get("fetch_bytes_per_dispatch")
        wr = t.get("write_bytes_per_dispatch")
        lines.append(f"| `{k[:90]}` | {v['dispatches']} | {v['total_ns'] / 1e6:.3f} | {v['avg_ns'] / 1e3:.2f} | "
                     f"{stage_of(k) or ''} | {'' if fr is None else f'{fr / 1e6:.1f}'} | "
                     f"{'' if wr is None else f'{wr / 1e6:.1f}'} |")
    # per stage (a stage may use several kernels, e.g. the blocked alpha transforms of the
    # coarse scales): the average launch duration the benchmark's live timing reports
    per_stage = defaultdict(lambda: [0, 0.0])
    for k, v in kernels.items():
        st = stage_of(k)
        if st:
            per_stage[st][0] += v["dispatches"]
            per_stage[st][1] += v["total_ns"]
    lines += ["", "| stage | dispatches | total ms | avg us per launch |", "|---|---:|---:|---:|"]
    for st, (n, tot) in sorted(per_stage.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| {st} | {n} | {tot / 1e6:.3f} | {tot / max(n, 1) / 1e3:.2f} |")
    lines += ["", f"HBM counters scaled by a {copy_bytes / 2**30:.0f} GiB device copy: FETCH_SIZE x "
              f"{cal['FETCH_SIZE'] / 1024:.4f}, WRITE_SIZE x {cal['WRITE_SIZE'] / 1024:.4f} (KiB counted -> KiB moved).", ""]
    with open(os.path.join(out_dir, f"{name}_kernels.md"), "w") as f:
        f.write("\n".join(lines))
    with open(os.path.join(out_dir, f"{name}_hbm_traffic.txt"), "w") as f:
        json.dump({"workload": name, "commands": commands.strip(), "kernel_sources_sha256": src,
                   "calibration_bytes_per_counter_unit": cal, "stages": stages,
                   "kernels": {k: {**kernels.get(k, {}), **traffic.get(k, {})} for k in set(kernels) | set(traffic)}},
                  f, indent=1, sort_keys=True)
    return stages


def wigner_valu(d: str, name: str, L: int, N: int, lam: float, J_min: int, commands: str, out_dir: str | None = None):
    """profiles/NAME_wigner_fp64.md from DIR/valu (rocprofv3 --pmc SQ_INSTS_VALU_{ADD,MUL,FMA,
    TRANS}_F64 SQ_ACTIVE_INST_VALU SQ_INSTS_VALU SQ_WAVES GRBM_GUI_ACTIVE on the Wigner kernels)
    and DIR/trace: per Wigner kernel the algorithmic GFLOP (5 per term of the l-sum or the
    m'-contraction, the count the benchmark uses), the executed FP64 GFLOP (64 lanes per wave
    instruction, 2 per FMA; full execution masks assumed, so an upper bound) and the share of
    SIMD cycles with a VALU instruction issued (4 cycles per wave64 instruction over 1024 SIMDs
    for the kernel's duration)."""
    import importlib.util
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    spec = importlib.util.spec_from_file_location("bench_for_profiles", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    from . import s2dw
    kappa, _, _ = s2dw.wavelet_tables(L, N, lam, J_min)
    alg = 5.0 * bench.wigner_terms(kappa, N)
    trace = {n: (int(c), float(a)) for n, c, t, a in
             _q(_db(os.path.join(d, "trace")),
                "select name, count(*), sum(end - start), avg(end - start) from kernels group by name")}
    rows = _q(_db(os.path.join(d, "valu")),
              "select kernel_name, counter_name, sum(value), count(*) from counters_collection "
              "group by kernel_name, counter_name")
    per = defaultdict(dict)
    for k, c, v, n in rows:
        per[k][c] = float(v) / n * 1.0  # per dispatch (counters summed over the device)
        per[k]["_n"] = n
    lines = [f"# FP64 VALU counters of the Wigner kernels: {name}", "", "Commands (run from the repository root):", "",
             "```", commands.strip(), "```", "", f"Kernel sources sha256: `{kernel_sources_hash()}`", "",
             "| kernel | avg us | algorithmic GFLOP | executed FP64 GFLOP | executed / algorithmic | "
             "algorithmic TFLOP/s (% of 78.6) | executed TFLOP/s | VALU busy % | FP64 share of VALU instructions |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for k, c in sorted(per.items()):
        avg_ns = next((a for n, (cnt, a) in trace.items() if n == k), None)
        if avg_ns is None:
            continue
        fma, mul, add, tr = (c.get(x, 0.0) for x in ("SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_MUL_F64",
                                                     "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_TRANS_F64"))
        exe = 64.0 * (2.0 * fma + mul + add + tr)
        valu = c.get("SQ_INSTS_VALU", 0.0)
        busy = 4.0 * valu / (1024.0 * avg_ns * 1e-9 * 2.4e9)
        t = avg_ns * 1e-9
        lines.append(f"| `{k[:60]}` | {avg_ns / 1e3:.1f} | {alg / 1e9:.2f} | {exe / 1e9:.2f} | {exe / alg:.2f} | "
                     f"{alg / t / 1e12:.1f} ({100 * alg / t / 78.6e12:.1f} %) | {exe / t / 1e12:.1f} | "
                     f"{100 * busy:.1f} | {100 * (fma + mul + add + tr) / max(valu, 1):.0f} % |")
    lines += ["", "Counters per dispatch: the value rocprofv3 reports summed over the device, averaged over the "
              "profiled dispatches; VALU busy assumes 2.4 GHz.", ""]
    with open(os.path.join(out_dir, f"{name}_wigner_fp64.md"), "w") as f:
        f.write("\n".join(lines))


def read_stage_traffic(name: str, out_dir: str | None = None):
    """HBM bytes per dispatch for each stage from a committed summary, or None when the
    summary is missing or the kernel sources changed since it was taken."""
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    p = os.path.join(out_dir, f"{name}_hbm_traffic.txt")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("kernel_sources_sha256") != kernel_sources_hash():
        return None
    return d.get("stages")


if __name__ == "__main__":
    if len(sys.argv) >= 2 and sys.argv[1] == "--wigner":
        # python -m paper_1308_5706_amd.profiling --wigner DIR NAME L N LAMBDA J_MIN "COMMANDS"
        a = sys.argv[2:]
        wigner_valu(a[0], a[1], int(a[2]), int(a[3]), float(a[4]), int(a[5]), a[6])
        sys.exit(0)
    if len(sys.argv) < 4:
        print(__doc__)
        sys.exit(2)
    gib = float(os.environ.get("COPY_GIB", "1"))
    st = write_profiles(sys.argv[1], sys.argv[2], sys.argv[3], int(gib * (1 << 30)))
    print(json.dumps(st, indent=1))
