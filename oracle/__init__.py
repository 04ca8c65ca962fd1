"""CPU oracle of the Falconn++ hot path. Test infrastructure only: the product path never imports it."""
from . import falconn  # noqa: F401
