"""Tuner of the fused projection's tile shapes (svlcov_spmm_tune_set).

For every storage type (FP32 base for the FP32/BF16x3 modes, FP64), rank k
and bin of nonzeros per row, it times every tile-shape variant of the fused
projection on a synthetic batch of that shape (device-resident CSR updates of
uniformly scattered columns, one launch of ``requests`` updates of ``rows``
rows each over matrices of ``cols`` columns) and keeps the fastest.  The
result is a JSON cache that ``paper_2401_09703_amd`` applies when it is
imported (``spmm_tuning_gfx950.json`` beside this file, or the file named by
``SVLCOV_SPMM_TUNING``).

    python -m paper_2401_09703_amd.autotune [--out PATH] [--quick]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

# representative nonzeros per row of each row bin (bin edges 16, 64, 256)
BIN_NNZ = (8, 32, 128, 512)


def _device_csr(L, torch, rows, cols, nnz_row, gen):
    nnz = max(rows * nnz_row, 1)
    r = torch.randint(0, rows, (nnz,), generator=gen, device="cuda", dtype=torch.int64)
    c = torch.randint(0, cols, (nnz,), generator=gen, device="cuda", dtype=torch.int64)
    key = torch.unique(r * cols + c)
    r, c = key // cols, key % cols
    rp = torch.zeros(rows + 1, dtype=torch.int64, device="cuda")
    rp[1:] = torch.cumsum(torch.bincount(r, minlength=rows), 0)
    v = 1.0 - torch.rand(key.numel(), generator=gen, device="cuda", dtype=torch.float64)
    return L.DeviceCSR(rows, cols, rp, c.to(torch.int32).contiguous(), v)


def _states(L, torch, prec, k, cols, count, gen):
    out = []
    for _ in range(count):
        m = max(k, 64)
        U = torch.linalg.qr(torch.randn(m, k, generator=gen, device="cuda",
                                        dtype=torch.float64)).Q.contiguous()
        V = torch.linalg.qr(torch.randn(cols, k, generator=gen, device="cuda",
                                        dtype=torch.float64)).Q.contiguous()
        s = torch.linspace(10.0, 1.0, k, device="cuda", dtype=torch.float64)
        out.append(L.TruncatedSVD(U, s, V, precision=prec, validate_device_inputs=False))
    return out


def tune(out_path=None, precisions=("bf16x3", "fp64"), ks=(16, 32, 64, 128), requests=64,
         rows=256, cols=20000, reps=3, log=print):
    import torch
    import paper_2401_09703_amd as L
    variants = L.spmm_variants()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(240109703)
    entries = []
    t0 = time.time()
    for prec in precisions:
        fp64 = 1 if prec == "fp64" else 0
        for k in ks:
            states = _states(L, torch, prec, k, cols, 8, gen)
            for b, nnz_row in enumerate(BIN_NNZ):
                Es = [_device_csr(L, torch, rows, cols, nnz_row, gen) for _ in range(requests)]
                sts = [states[q % len(states)] for q in range(requests)]
                torch.cuda.synchronize()
                times = []
                for v in range(len(variants)):
                    L.spmm_tune_set(fp64, k, b, v)
                    ms = []
                    for _ in range(reps + 1):
                        L.project_batch(sts, [1] * requests, Es, timing=ms)
                    times.append(min(ms[1:]))
                best = int(np.argmin(times))
                L.spmm_tune_set(fp64, k, b, best)
                entries.append(dict(fp64=fp64, k=k, row_bin=b, variant=best,
                                    shape=list(variants[best]), ms=times[best],
                                    ms_default=times[0],
                                    ms_all=[round(x, 5) for x in times]))
                log(f"[autotune] {prec} k={k} nnz/row~{nnz_row}: variant {best} "
                    f"{variants[best]} {times[best]:.4f} ms (default {times[0]:.4f} ms)")
            for st in states:
                st.close()
    props = torch.cuda.get_device_properties(0)
    data = dict(arch=getattr(props, "gcnArchName", "gfx950"),
                batch=dict(requests=requests, rows=rows, cols=cols, reps=reps),
                variants=[list(v) for v in variants], entries=entries,
                seconds=round(time.time() - t0, 1))
    if out_path:
        with open(out_path, "w") as f:
            json.dump(data, f, indent=1)
    return data


def main():
    import paper_2401_09703_amd as L
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=L.TUNING_PATH)
    ap.add_argument("--quick", action="store_true", help="k=64 FP32 storage only")
    args = ap.parse_args()
    if args.quick:
        tune(args.out, precisions=("bf16x3",), ks=(64,))
    else:
        tune(args.out)


if __name__ == "__main__":
    main()
