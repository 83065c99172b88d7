"""HN exact top-1 search on MI355X (see hnsearch.h for the C ABI)."""
