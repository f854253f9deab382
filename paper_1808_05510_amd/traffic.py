"""HBM traffic of one factored operator application, from rocprofv3 counters.

The `run` step does, on the GPU: a plain device-to-device copy of 256 MiB
(the calibration kernel of known size), then two calls of cr_op_apply (FP64,
r = 100) on the cortex-shell workload.  It is meant to run under two counter
passes, one counter each:

    rocprofv3 --pmc FETCH_SIZE -d OUT/fetch -o t --output-format csv -- \\
        python3 -m paper_1808_05510_amd.traffic run
    rocprofv3 --pmc WRITE_SIZE -d OUT/write -o t --output-format csv -- \\
        python3 -m paper_1808_05510_amd.traffic run

`summarize FETCH_CSV WRITE_CSV STEM` then sums the counters (KiB per
dispatch) over the library kernels of the second call, scales each counter by
copy bytes / counter reading of the copy, and writes STEM.md (table and the
commands) and STEM.json (figures plus a hash of the code, comments and layout excluded, of
the file that holds the kernels and of the host function that launches them,
so that a reader can tell whether they changed since the counters were
taken).
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
COPY_BYTES = 256 * 1024 * 1024
RANK = 100


# the kernels that move op_apply's bytes (stencils, X^T V, masked product),
# and the host function that orders them (fork/join, launch order, grids)
KERNEL_SOURCES = ("k_blas.hip",)
ORCHESTRATION = ("api.hip", "static cr_status op_apply_run(", "static cr_status op_apply_impl(")


def _code_only(src: str) -> str:
    """The source with comments removed and whitespace collapsed, so that an
    edit of comments or layout leaves the hash unchanged."""
    src = re.sub(r"//[^\n]*", "", src)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return re.sub(r"\s+", " ", src).strip()


def sources_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(CSRC, name)) as f:
            h.update(name.encode())
            h.update(_code_only(f.read()).encode())
    name, start, end = ORCHESTRATION
    with open(os.path.join(CSRC, name)) as f:
        src = f.read()
    i, j = src.find(start), src.find(end)
    h.update(name.encode())
    h.update(_code_only(src[i:j] if 0 <= i < j else src).encode())
    return h.hexdigest()[:16]


def algorithmic_bytes(n_y, n_x, n_inj, r, s=8):
    return (s * ((n_y + n_x) * r + n_x * n_inj + 2 * (n_y + n_x) * r + n_y * n_inj)
            + n_y * n_inj / 8 + 24 * (n_y + n_x))


def run():
    import torch

    from . import connreg, synth
    a = torch.ones(COPY_BYTES // 8, device="cuda:0", dtype=torch.float64)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    d = synth.config3(seed=0)
    prob = connreg.Problem(d, "fp64", "cuda:0")
    g = torch.Generator(device="cuda:0").manual_seed(1)
    U = torch.randn((RANK, prob.n_y), device="cuda:0", dtype=torch.float64, generator=g).T
    V = torch.randn((RANK, prob.n_x), device="cuda:0", dtype=torch.float64, generator=g).T
    Z = torch.randn((RANK, RANK), device="cuda:0", dtype=torch.float64, generator=g).T
    for _ in range(2):
        prob.op_apply(U, Z, V)
        torch.cuda.synchronize()
    print(json.dumps(dict(n_y=prob.n_y, n_x=prob.n_x, n_inj=prob.n_inj, r=RANK)), flush=True)
    prob.close()


def _rows(path):
    with open(path) as f:
        rows = list(csv.DictReader(f))
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def _short(name):
    name = name.split("(")[0]
    return name.replace("void ", "")[:60]


def summarize(fetch_csv, write_csv, stem, n_y=262136, n_x=131068, n_inj=128):
    out = {}
    for which, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        rows = [r for r in _rows(path) if r["Counter_Name"] == which]
        copies = [r for r in rows if "copyBuffer" in r["Kernel_Name"] or "copy" in r["Kernel_Name"]]
        ref = max(copies, key=lambda r: float(r["Counter_Value"]))
        lib = [r for r in rows if "cr::" in r["Kernel_Name"]]
        # each call launches one masked-product kernel: the distance between
        # the two is the number of dispatches per call, and the second call is
        # that many dispatches from the end
        mk = [i for i, r in enumerate(lib) if "k_masked" in r["Kernel_Name"]]
        per_call = mk[-1] - mk[-2]
        second = lib[len(lib) - per_call:]
        out[which] = dict(copy_kib=float(ref["Counter_Value"]),
                          kernels=[(_short(r["Kernel_Name"]), float(r["Counter_Value"]))
                                   for r in second])
    ff = COPY_BYTES / (1024.0 * out["FETCH_SIZE"]["copy_kib"])
    fw = COPY_BYTES / (1024.0 * out["WRITE_SIZE"]["copy_kib"])
    fetch = sum(v for _, v in out["FETCH_SIZE"]["kernels"]) * 1024.0 * ff
    write = sum(v for _, v in out["WRITE_SIZE"]["kernels"]) * 1024.0 * fw
    alg = algorithmic_bytes(n_y, n_x, n_inj, RANK)
    res = dict(kernel="cr_op_apply FP64 r=100, shell workload (n_y 262,136, n_x 131,068, n_inj 128)",
               fetch_factor=ff, write_factor=fw, fetch_bytes=fetch, write_bytes=write,
               traffic_bytes=fetch + write, algorithmic_bytes=alg,
               traffic_over_algorithmic=(fetch + write) / alg, sources_sha=sources_hash())
    with open(stem + ".json", "w") as f:
        json.dump(res, f, indent=1)
    lines = [f"# HBM traffic of one `cr_op_apply` call (FP64, r = 100, shell workload)", "",
             "Commands (from the repository root, `cd /tmp && export TMPDIR=/tmp` first):", "",
             "```",
             "rocprofv3 --pmc FETCH_SIZE -d OUT/fetch -o t --output-format csv -- "
             "python3 -m paper_1808_05510_amd.traffic run",
             "rocprofv3 --pmc WRITE_SIZE -d OUT/write -o t --output-format csv -- "
             "python3 -m paper_1808_05510_amd.traffic run",
             "python3 -m paper_1808_05510_amd.traffic summarize OUT/fetch/t_counter_collection.csv "
             "OUT/write/t_counter_collection.csv profiles/op_apply_shells_r100_fp64_traffic",
             "```", "",
             f"Calibration: a 256 MiB device copy reads {out['FETCH_SIZE']['copy_kib']:.0f} KiB of "
             f"FETCH_SIZE and {out['WRITE_SIZE']['copy_kib']:.0f} KiB of WRITE_SIZE, so the factors "
             f"are {ff:.3f} (fetch) and {fw:.3f} (write).", "",
             "| kernel (second call, dispatch order) | FETCH_SIZE KiB | WRITE_SIZE KiB |",
             "|---|---:|---:|"]
    for (k, fv), (_, wv) in zip(out["FETCH_SIZE"]["kernels"], out["WRITE_SIZE"]["kernels"]):
        lines.append(f"| `{k}` | {fv:.0f} | {wv:.0f} |")
    lines += ["", f"Scaled: fetch {fetch/1e6:.1f} MB, write {write/1e6:.1f} MB, total "
              f"{(fetch+write)/1e6:.1f} MB against {alg/1e6:.1f} MB algorithmic "
              f"({(fetch+write)/alg:.2f}x).", "",
              f"Kernel sources hash (code only, comments and whitespace excluded): "
              f"`{res['sources_sha']}`."]
    with open(stem + ".md", "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps(res))


if __name__ == "__main__":
    if sys.argv[1] == "run":
        run()
    elif sys.argv[1] == "summarize":
        summarize(sys.argv[2], sys.argv[3], sys.argv[4])
    else:
        raise SystemExit("usage: traffic.py run | summarize FETCH_CSV WRITE_CSV STEM")
