"""Network geometry of the VGG-19 prefix used by the energy (Sec. 3.1).

Style layers are the post-ReLU outputs of conv k_1 (k = 1..5) and the content
layer is the post-ReLU output of conv4_2 (Sec. 3.1).  Only conv1_1 .. conv5_1
influence the energy.  Pooling is 2x2 stride-2 max pooling in floor mode after
conv1_2, conv2_2, conv3_4 and conv4_4 (the paper does not state the pooling
type; max pooling of the standard VGG-19 is the reading taken here).
"""
from __future__ import annotations

from dataclasses import dataclass, field

VGG19_CONVS = [(3, 64), (64, 64), (64, 128), (128, 128), (128, 256), (256, 256),
               (256, 256), (256, 256), (256, 512), (512, 512), (512, 512),
               (512, 512), (512, 512)]
VGG19_NAMES = ["conv1_1", "conv1_2", "conv2_1", "conv2_2", "conv3_1", "conv3_2",
               "conv3_3", "conv3_4", "conv4_1", "conv4_2", "conv4_3", "conv4_4",
               "conv5_1"]


@dataclass(frozen=True)
class NetSpec:
    convs: tuple                      # ((c_in, c_out), ...)
    pool_after: frozenset             # conv indices followed by a 2x2/2 max pool
    style: tuple                      # conv indices whose ReLU output is a style layer
    content: int | None               # conv index of the content layer (None: texture)
    names: tuple = field(default=())
    avg_pool: bool = False            # 2x2/2 average pools instead of max pools

    @property
    def n_conv(self) -> int:
        return len(self.convs)

    def strides(self):
        """Cumulative stride s_i of the output of conv i (1, 2, 4, ...)."""
        s, out = 1, []
        for i in range(self.n_conv):
            out.append(s)
            if i in self.pool_after:
                s *= 2
        return out

    def align(self) -> int:
        """Product of all pooling factors that precede the last conv (S)."""
        return self.strides()[-1]


def vgg19(style_weights=None, content=True, avg_pool=False) -> NetSpec:
    return NetSpec(convs=tuple(VGG19_CONVS), pool_after=frozenset({1, 3, 7, 11}),
                   style=(0, 2, 4, 8, 12), content=(9 if content else None),
                   names=tuple(VGG19_NAMES), avg_pool=avg_pool)


def vgg19_tiny(content=True, avg_pool=False) -> NetSpec:
    """Prefix conv1_1 .. conv3_1; style relu1_1, relu2_1, relu3_1; content relu2_2."""
    return NetSpec(convs=tuple(VGG19_CONVS[:5]), pool_after=frozenset({1, 3}),
                   style=(0, 2, 4), content=(3 if content else None),
                   names=tuple(VGG19_NAMES[:5]), avg_pool=avg_pool)


def receptive_fields(net: NetSpec):
    """Per conv i, (a_i, b_i): output row q depends on input rows [s q - a, s q + b].

    Closed form by composition: a 3x3 conv at cumulative stride s widens the
    interval by s on both sides; a 2x2/2 floor pool keeps the start, extends
    the end by s and doubles s.
    """
    a = b = 0
    s = 1
    out = []
    for i in range(net.n_conv):
        a += s
        b += s
        out.append((a, b))
        if i in net.pool_after:
            b += s
            s *= 2
    return out


def min_halo(net: NetSpec) -> int:
    """Smallest margin m* that makes the tiled gradient exact: max_i (a_i + b_i)
    over the convs up to the deepest layer the energy uses."""
    used = max(list(net.style) + ([net.content] if net.content is not None else []))
    rf = receptive_fields(net)
    return max(a + b for (a, b) in rf[: used + 1])
