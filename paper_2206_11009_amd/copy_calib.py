"""A plain device-to-device copy of known size, for calibrating the HBM
traffic counters (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE):

    python -m paper_2206_11009_amd.copy_calib

Three copies of 2^27 doubles (1 GiB each way per copy).
"""


def main():
    import torch
    n = 1 << 27
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied", 3, "x", n * 8, "bytes", flush=True)


if __name__ == "__main__":
    main()
