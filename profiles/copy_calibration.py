"""Plain device copy of a known size, profiled beside the sort/join kernels so
that the FETCH_SIZE / WRITE_SIZE counters can be scaled to bytes: the copy
reads and writes exactly `nbytes` each."""
import sys

import torch

nbytes = int(sys.argv[1]) if len(sys.argv) > 1 else 1 << 30
src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
src.fill_(1)
dst = torch.empty_like(src)
torch.cuda.synchronize()
for _ in range(3):
    dst.copy_(src)
torch.cuda.synchronize()
print("copied %d bytes x3" % nbytes)
