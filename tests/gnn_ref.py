"""Independent FP64 reference of the surrogate network (torch, CPU, float64
autograd) and of its graph construction, used to check the library's
kernels.  Shares no code with the library: features, edges and the network
are written out here from their definitions.
"""
import math

import numpy as np
import torch

import workloads as W

KINDS = ["H", "X", "Y", "Z", "S", "T", "RX", "RY", "RZ", "U", "U1Q",
         "CNOT", "CZ", "CP", "SWAP", "RZZ", "U2Q"]
FIN, HID, NL, GLOB, OUT = 32, 64, 3, 4, 13
ZW = HID + GLOB


def graph(c: W.Circuit):
    """(x[G, 32], neighbour lists, glob[4]) from the definitions."""
    G = len(c.gates)
    qdepth = [0] * c.n
    last = [-1] * c.n
    layer = [0] * G
    nbr = [[] for _ in range(G)]
    for i, g in enumerate(c.gates):
        lv = max(qdepth[q] for q in g.qubits)
        layer[i] = lv
        for q in g.qubits:
            qdepth[q] = lv + 1
            if last[q] >= 0:
                nbr[i].append(last[q])
                nbr[last[q]].append(i)
            last[q] = i
    depth = max(layer) + 1 if G else 0
    x = np.zeros((G, FIN))
    for i, g in enumerate(c.gates):
        x[i, KINDS.index(g.name)] = 1.0
        for j in range(W.GATE_NPARAM[g.name]):
            x[i, 17 + 2 * j] = math.sin(g.params[j])
            x[i, 18 + 2 * j] = math.cos(g.params[j])
        x[i, 23] = layer[i] / depth
        x[i, 24] = len(g.qubits) - 1
        x[i, 25] = c.n / 16.0
        x[i, 26] = 1.0
    glob = np.array([c.n / 16.0, G / 2048.0, c.S / 4096.0, 1.0])
    return x, nbr, glob


def layout():
    off = {}
    o = 0

    def take(name, size):
        nonlocal o
        off[name] = (o, size)
        o += size

    take("w_in", FIN * HID)
    take("b_in", HID)
    for l in range(NL):
        take(f"ws{l}", HID * HID)
        take(f"wn{l}", HID * HID)
        take(f"b{l}", HID)
    take("w_h1", ZW * HID)
    take("b_h1", HID)
    take("w_h2", HID * OUT)
    take("b_h2", OUT)
    return off, o


def loss_and_grad(params: np.ndarray, circuits, labels):
    """Mean squared error of the sigmoid outputs and its gradient (float64)."""
    off, total = layout()
    assert params.size == total
    p = torch.tensor(params.astype(np.float64), requires_grad=True)

    def blk(name, shape):
        o, s = off[name]
        return p[o:o + s].reshape(shape)

    outs = []
    for c in circuits:
        x, nbr, glob = graph(c)
        G = len(nbr)
        A = np.zeros((G, G))
        for v, ns in enumerate(nbr):
            for u in ns:
                A[v, u] += 1.0 / len(ns)
        X = torch.tensor(x)
        Am = torch.tensor(A)
        h = torch.relu(X @ blk("w_in", (FIN, HID)) + blk("b_in", (HID,)))
        for l in range(NL):
            a = Am @ h
            h = torch.relu(h @ blk(f"ws{l}", (HID, HID)) + a @ blk(f"wn{l}", (HID, HID)) + blk(f"b{l}", (HID,)))
        z = torch.cat([h.mean(0), torch.tensor(glob)])
        u = torch.relu(z @ blk("w_h1", (ZW, HID)) + blk("b_h1", (HID,)))
        outs.append(torch.sigmoid(u @ blk("w_h2", (HID, OUT)) + blk("b_h2", (OUT,))))
    out = torch.stack(outs)
    y = torch.tensor(np.asarray(labels, np.float64))
    loss = ((out - y) ** 2).mean()
    loss.backward()
    return float(loss.detach()), p.grad.numpy().copy(), out.detach().numpy()
