"""Plain device-to-device copy of a known size, used to calibrate the HBM byte counters
(FETCH_SIZE / WRITE_SIZE) of rocprofv3 against a kernel whose traffic is known exactly."""
import torch

N_BYTES = 1 << 30

a = torch.ones(N_BYTES // 4, dtype=torch.float32, device="cuda")
b = torch.empty_like(a)
torch.cuda.synchronize()
b.copy_(a)
torch.cuda.synchronize()
print(f"copied {N_BYTES} bytes", flush=True)
