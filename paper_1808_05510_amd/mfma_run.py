"""A short run of the two MFMA kernels of the hot path, for counter
collection: the BF16 Khatri-Rao masked Gram (r = 100) and the masked product
of cr_op_apply (FP64 and FP32, r = 100) on the cortex-shell workload, three
calls each.  Meant to run under

    rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES SQ_BUSY_CU_CYCLES GRBM_GUI_ACTIVE -d OUT -o m \\
        --output-format csv -- python3 -m paper_1808_05510_amd.mfma_run
"""
from __future__ import annotations

import torch

from . import connreg, synth


def main():
    d = synth.config3(seed=0)
    r = 100
    for prec in ("fp64", "mixed"):
        p = connreg.Problem(d, prec, "cuda:0")
        g = torch.Generator(device="cuda:0").manual_seed(3)
        dt = torch.float64 if prec == "fp64" else torch.float32
        U = torch.randn((r, p.n_y), device="cuda:0", dtype=dt, generator=g).T
        V = torch.randn((r, p.n_x), device="cuda:0", dtype=dt, generator=g).T
        Z = torch.randn((r, r), device="cuda:0", dtype=dt, generator=g).T
        for _ in range(3):
            p.op_apply(U, Z, V, fp32=prec == "mixed")
            if prec == "fp64":
                p.masked_gram(U / U.norm(dim=0, keepdim=True), "bf16")
        torch.cuda.synchronize()
        p.close()
    print("done", flush=True)


if __name__ == "__main__":
    main()
