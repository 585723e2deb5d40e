"""Plain device-to-device copy of a known size, used to calibrate the HBM byte
counters (FETCH_SIZE, WRITE_SIZE) that rocprofv3 reports for the step kernel:

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT -- python3 -m paper_1709_09073_amd.copy_probe
    rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT -- python3 -m paper_1709_09073_amd.copy_probe

Each run copies 1 GiB three times; the counter per copy dispatch divided into
1 GiB is the scale factor applied to the step kernel's counter.
"""
import torch

NBYTES = 1 << 30


def main():
    a = torch.ones(NBYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {NBYTES} bytes 3 times", flush=True)


if __name__ == "__main__":
    main()
