"""Reference copy kernel for calibrating HBM traffic counters.

`python -m paper_1411_3019_amd.probe --bytes N` copies an N-byte device buffer
into another (torch's copy kernel) a few times.  Run under
`rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE), the counters of a copy of known
size give the factor that turns the counter readings of other kernels into
bytes moved to and from HBM.
"""
import argparse


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--bytes", type=int, default=1 << 30)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    import torch
    n = a.bytes // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {n * 8} bytes x {a.reps}")


if __name__ == "__main__":
    main()
