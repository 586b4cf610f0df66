"""Plain device copy of a known size, used to calibrate the HBM byte counters
(FETCH_SIZE / WRITE_SIZE) that the benchmark's roofline entry reports."""
import torch

N = 256 * 1024 * 1024          # bytes copied by each launch
src = torch.empty(N, dtype=torch.uint8, device="cuda:0")
src.fill_(1)
dst = torch.empty_like(src)
torch.cuda.synchronize()
for _ in range(3):
    dst.copy_(src)
torch.cuda.synchronize()
print("copied", N, "bytes x3")
