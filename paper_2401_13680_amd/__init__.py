"""MI355X (gfx950) MPdist-profile and snippet library: the snippet-finding hot
path of the PaSTiLa labelling method (MPdist profiles of every segment, greedy
minimum-area snippet selection, and the snippet-length criterion).

The compute runs in the HIP library ``libpst.so`` behind the C ABI in
``include/pst.h``; this package is its Python binding.
"""


def __getattr__(name):
    if name in ("mpdist_profile", "profile_set", "snippets", "select_length", "Context", "context"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
