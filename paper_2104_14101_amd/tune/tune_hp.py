"""Tuner of the batched step's product A^T (A P): for every (precision, ceil(log2 n), ceil(d / 256))
bucket of a list of shapes, times the grouped product of one problem of the bucket's middle shape
under each candidate plan (fused single-read form, two-pass form; rows of A per partial product)
through aes_tune_hp and writes the fastest plan per bucket as one line

    <fp32|fp64> <ceil(log2 n)> <ceil(d / 256)> <fused|twopass> <rows> <ms> <candidates tried>

to the plan file the library reads (tune/hp_plans.txt beside its directory, or AES_TUNE_FILE).

Usage: python -m paper_2104_14101_amd.tune.tune_hp [--out FILE] [--c 32] [--reps 10]
The default shape list covers the batched workload (n = 256 U{32..512}, d = 256 U{1..8}).
"""
import argparse
import ctypes
import datetime
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

FUSED_ROWS = (64, 128, 256, 512, 1024)
TWOPASS_ROWS = (512, 1024, 2048, 4096)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "hp_plans.txt"))
    ap.add_argument("--c", type=int, default=32)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--log2n", default="13,14,15,16,17")
    ap.add_argument("--dblocks", default="1,2,3,4,5,6,7,8")
    args = ap.parse_args()

    import torch

    import paper_2104_14101_amd as aes
    from paper_2104_14101_amd import _binding as B

    lib = B.load()
    dev = torch.device("cuda:0")
    h = aes._handle(dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    lines = [f"# plans of the grouped A^T (A P) product, {args.c} columns, {args.reps} timed launches each",
             f"# written by tune_hp.py on {torch.cuda.get_device_name(0)}, "
             f"{datetime.datetime.now(datetime.timezone.utc).strftime('%Y-%m-%d %H:%M UTC')}",
             "# precision log2n dblocks kind rows ms tried"]
    gen = torch.Generator(device=dev)
    gen.manual_seed(1)
    for lg in [int(v) for v in args.log2n.split(",")]:
        n = max(256, (3 << (lg - 2)) // 256 * 256)  # middle of (2^(lg-1), 2^lg]
        for db in [int(v) for v in args.dblocks.split(",")]:
            d = 256 * db
            A = torch.randn((n, d), dtype=torch.float64, device=dev, generator=gen)
            for prec_name, prec in (("fp32", B.PRECISIONS["mixed_fp32"]), ("fp64", B.PRECISIONS["fp64"])):
                cands = [(0, r) for r in FUSED_ROWS] + [(1, r) for r in TWOPASS_ROWS]
                best = None
                tried = 0
                for twopass, rows in cands:
                    ms = ctypes.c_double(0.0)
                    st = lib.aes_tune_hp(h, stream, n, d, args.c, ctypes.c_void_p(A.data_ptr()), d, prec, twopass, rows,
                                         args.reps, ctypes.byref(ms))
                    if st != B.AES_OK:
                        continue  # the plan does not apply to the shape
                    tried += 1
                    if best is None or ms.value < best[2]:
                        best = (twopass, rows, ms.value)
                if best is None:
                    continue
                kind = "twopass" if best[0] else "fused"
                lines.append(f"{prec_name} {lg} {db} {kind} {best[1]} {best[2]:.4f} {tried}")
                print(lines[-1], flush=True)
            del A
    with open(args.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
