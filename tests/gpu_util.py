"""Helpers shared by the GPU parity tests (host side only)."""

import sys

import numpy as np

import oracle as O

# Unit roundoff of each operand format and of the accumulator (2^-p).
U_F64 = 2.0 ** -53
U_F32 = 2.0 ** -24
U_BF16 = 2.0 ** -8
U_F16 = 2.0 ** -11
# hi + lo in bf16 represents v to 2^-16 |v|, and the dropped lo*lo product is
# at most 2^-16 |a b|: the three-product form errs by at most 3 * 2^-16 |a b|.
U_BF16X3 = 1.5 * 2.0 ** -16

OPERAND_U = {"fp64": U_F64, "fp32": U_F32, "bf16": U_BF16, "fp16": U_F16, "bf16x3": U_BF16X3}
ACC_U = {"fp64": U_F64, "fp32": U_F32, "bf16": U_F32, "fp16": U_F32, "bf16x3": U_F32}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).to("cuda:0")


def host(t):
    return t.detach().to("cpu").numpy()


def gamma(mode, K):
    """First-order error factor of one GEMM stage with dot length K:
    both operands rounded (2 u_op) plus recursive FP accumulation (K u_acc)."""
    return 2.0 * OPERAND_U[mode] + K * ACC_U[mode]


def abs_forward(K, H, X):
    """sum_k |H_k| |X| |K_k|^T : the magnitude that bounds the error of A_s X."""
    return sum(np.abs(H[k]) @ np.abs(X) @ np.abs(K[k]).T for k in range(K.shape[0]))


def abs_adjoint(K, H, R):
    return sum(np.abs(H[j]).T @ np.abs(R) @ np.abs(K[j]) for j in range(K.shape[0]))


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
