"""Helpers shared by the GPU tests: device placement of seeded inputs."""
import numpy as np
import torch

DEV = torch.device("cuda", 0)


def t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def scene_tensors(s):
    return [t(a) for a in s.arrays()]


def log(msg):
    print(msg, flush=True)
