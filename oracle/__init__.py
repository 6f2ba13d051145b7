"""Plain CPU oracle of the CRSH path: test infrastructure, never the product path."""
