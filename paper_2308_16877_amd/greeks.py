"""Black-Scholes prices as a differentiable torch operation whose forward and
backward run in the library's kernels.

    C, P = GreeksFn.apply(S, K, T, r, v, technique, params, items_per_lane)

technique "exact": forward hpac_exact on the price region, backward
hpac_bs_adjoint (derivatives recomputed from the inputs).
technique "iact": forward iACT on the price-and-source region
(HPAC_REGION_BS_PRICE_REF): each item's prices and the index of the item
whose evaluation produced them (itself, or the source of the reused
entry); the backward recomputes the derivatives at that source item
(hpac_bs_vjp_ref), so an approximated item reuses the memoized gradient by
reference: 4 bytes per item carried from forward to backward.
technique "iact_jacobian" / "taf" / "perfo": forward runs that technique on
the price-and-Jacobian region (12 output columns), so an approximated item
returns the prices AND the derivatives of the item it reuses; the backward
contracts that saved Jacobian (hpac_bs_vjp).  Both memo forms give the same
gradients bit for bit.
"""
import torch

from . import hpac


class GreeksFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, S, K, T, r, v, technique="exact", params=None, items_per_lane=16):
        x = [t.contiguous() for t in (S, K, T, r, v)]
        n = x[0].numel()
        params = dict(params or {})
        if technique == "exact":
            C, P = (torch.empty(n, dtype=torch.float32, device=S.device) for _ in range(2))
            hpac.hpac_exact(x, [C, P], items_per_lane=items_per_lane, region=hpac.REGION_BS_PRICE)
            ctx.save_for_backward(*x)
            ctx.mode = "adjoint"
        elif technique == "iact":
            C, P = (torch.empty(n, dtype=torch.float32, device=S.device) for _ in range(2))
            src = torch.empty(n, dtype=torch.int32, device=S.device)
            hpac.hpac_iact(x, [C, P, src], items_per_lane=items_per_lane, region=hpac.REGION_BS_PRICE_REF, **params)
            ctx.save_for_backward(*x, src)
            ctx.mode = "reference"
        else:
            technique = "iact" if technique == "iact_jacobian" else technique
            outs = [torch.zeros(n, dtype=torch.float32, device=S.device) for _ in range(12)]
            fn = {"iact": hpac.hpac_iact, "taf": hpac.hpac_taf, "perfo": hpac.hpac_perfo}[technique]
            fn(x, outs, items_per_lane=items_per_lane, region=hpac.REGION_BS_PRICE_GRAD, **params)
            C, P = outs[0], outs[1]
            ctx.save_for_backward(*outs[2:])
            ctx.mode = "vjp"
        ctx.n = n
        return C, P

    @staticmethod
    def backward(ctx, gC, gP):
        saved = ctx.saved_tensors
        dev = saved[0].device
        grads = [torch.empty(ctx.n, dtype=torch.float32, device=dev) for _ in range(5)]
        gC = gC.contiguous().to(torch.float32) if gC is not None else None
        gP = gP.contiguous().to(torch.float32) if gP is not None else None
        if ctx.mode == "adjoint":
            hpac.hpac_bs_adjoint(list(saved), gC, gP, grads)
        elif ctx.mode == "reference":
            hpac.hpac_bs_vjp_ref(list(saved[:5]), saved[5], gC, gP, grads)
        else:
            hpac.hpac_bs_vjp(list(saved), gC, gP, grads)
        return tuple(grads) + (None, None, None)


def bs_prices(S, K, T, r, v, technique="exact", params=None, items_per_lane=16):
    return GreeksFn.apply(S, K, T, r, v, technique, params, items_per_lane)
